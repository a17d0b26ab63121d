"""Per-antenna beam patterns (paper section 2.2.3) through fv_simulate_beams
against the oracle's pair-by-pair sum."""
import numpy as np
import pytest

import oracle
import synth
from oracle import beams as obeams

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(torch.device("cuda:0"))


def _case(seed, n_ant=37, n_src=400, n_freq=2, n_beam=3, hex_layout=True):
    p = synth.small_problem(seed, n_ant=n_ant, n_src=n_src, n_freq=n_freq, hex_layout=hex_layout)
    rng = np.random.default_rng(seed)
    pats = rng.uniform(0.3, 1.0, (n_beam, n_freq, n_src)) * np.sqrt(p.beam)[None]
    which = rng.integers(0, n_beam, n_ant)
    return p, pats, which


def _run(fv, ctx, p, pats, which, eps):
    import torch
    vis = torch.empty((p.n_freq, p.n_pairs, 2), dtype=torch.float64, device="cuda:0")
    rep = ctx.simulate_beams(_dev(p.ant_enu), _dev(p.src_lmn), _dev(p.freq_hz), _dev(p.flux), _dev(pats), which,
                             vis, eps=eps)
    torch.cuda.synchronize()
    o = vis.cpu().numpy()
    return o[..., 0] + 1j * o[..., 1], rep


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("eps", [1e-6, 1e-10])
def test_three_patterns_on_a_hex_array(gpu_lib, ctx, eps):
    p, pats, which = _case(150)
    v, rep = _run(gpu_lib, ctx, p, pats, which, eps)
    ref = obeams.beams_vis(p.ant_enu, p.src_lmn, p.freq_hz, p.flux, pats, which)
    assert oracle.rel_l2(v, ref) <= eps
    assert rep["lattice"] == 1


def test_two_patterns_on_a_random_array(gpu_lib, ctx):
    p, pats, which = _case(151, n_ant=30, n_beam=2, hex_layout=False)
    v, rep = _run(gpu_lib, ctx, p, pats, which, 1e-6)
    ref = obeams.beams_vis(p.ant_enu, p.src_lmn, p.freq_hz, p.flux, pats, which)
    assert oracle.rel_l2(v, ref) <= 1e-6
    assert rep["lattice"] == 0


def test_one_pattern_matches_the_shared_beam_call(gpu_lib, ctx):
    import torch
    p, pats, _ = _case(152, n_beam=1)
    v, _ = _run(gpu_lib, ctx, p, pats, np.zeros(p.n_ant, dtype=int), 1e-10)
    w = torch.empty((p.n_freq, p.n_pairs, 2), dtype=torch.float64, device="cuda:0")
    ctx.simulate_dev(_dev(p.ant_enu), _dev(p.src_lmn), _dev(p.freq_hz), _dev(p.flux), _dev(pats[0] ** 2), w,
                     eps=1e-10)
    torch.cuda.synchronize()
    o = w.cpu().numpy()
    assert oracle.rel_l2(v, o[..., 0] + 1j * o[..., 1]) <= 2e-10


def test_unused_patterns_and_a_dead_antenna(gpu_lib, ctx):
    p, pats, which = _case(153, n_ant=19, n_beam=5)
    which = np.where(which == 3, 0, which)   # pattern 3 unused
    pats[4] = 0.0
    which[2] = 4                              # antenna 2 is dead
    v, _ = _run(gpu_lib, ctx, p, pats, which, 1e-6)
    ref = obeams.beams_vis(p.ant_enu, p.src_lmn, p.freq_hz, p.flux, pats, which)
    assert oracle.rel_l2(v, ref) <= 1e-6
    iu, ju = np.triu_indices(p.n_ant)
    assert np.all(v[:, (iu == 2) | (ju == 2)] == 0)


def test_bad_pattern_index_and_non_finite_beam(gpu_lib, ctx):
    fv = gpu_lib
    p, pats, which = _case(154, n_ant=7, n_src=50, n_beam=2)
    bad = which.copy()
    bad[0] = 2
    with pytest.raises(fv.FvError, match="EINVAL"):
        _run(fv, ctx, p, pats, bad, 1e-6)
    pats2 = pats.copy()
    pats2[1, 0, 7] = np.inf
    which[:] = 1
    with pytest.raises(fv.FvError, match="EINVAL"):
        _run(fv, ctx, p, pats2, which, 1e-6)
    v, _ = _run(fv, ctx, p, pats, which, 1e-6)   # still usable
    assert oracle.rel_l2(v, obeams.beams_vis(p.ant_enu, p.src_lmn, p.freq_hz, p.flux, pats, which)) <= 1e-6
