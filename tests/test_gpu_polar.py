"""Polarised feed products (paper section 2.1, Jones form, shared beam)
through fv_simulate_polar against the oracle's source-by-source matrix sum."""
import numpy as np
import pytest

import oracle
import synth
from oracle import polar as opolar

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(torch.device("cuda:0"))


def _case(seed, n_ant=37, n_src=500, n_freq=2, hex_layout=True, feeds=True):
    p = synth.small_problem(seed, n_ant=n_ant, n_src=n_src, n_freq=n_freq, hex_layout=hex_layout)
    rng = np.random.default_rng(seed)
    I = p.flux
    QUV = rng.uniform(-0.2, 0.2, (3, n_freq, n_src)) * I[None]
    stokes = np.concatenate([I[None], QUV])
    jones = None
    if feeds:
        g = np.sqrt(p.beam)[..., None, None]
        jones = g * (np.eye(2)[None, None] + 0.1 * (rng.normal(size=(n_freq, n_src, 2, 2))
                                                     + 1j * rng.normal(size=(n_freq, n_src, 2, 2))))
    return p, stokes, jones


def _run(fv, ctx, p, stokes, jones, eps):
    import torch
    vis = torch.empty((4, p.n_freq, p.n_pairs, 2), dtype=torch.float64, device="cuda:0")
    jd = None if jones is None else _dev(np.stack([jones.real, jones.imag], axis=-1))
    rep = ctx.simulate_polar(_dev(p.ant_enu), _dev(p.src_lmn), _dev(p.freq_hz), _dev(stokes), jd, vis, eps=eps)
    torch.cuda.synchronize()
    o = vis.cpu().numpy()
    v = o[..., 0] + 1j * o[..., 1]                       # [4, f, pair]
    return np.moveaxis(v.reshape(2, 2, p.n_freq, p.n_pairs), (0, 1), (2, 3)), rep   # [f, pair, 2, 2]


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("eps", [1e-6, 1e-10])
def test_complex_feeds_on_a_hex_array(gpu_lib, ctx, eps):
    p, stokes, jones = _case(180)
    v, rep = _run(gpu_lib, ctx, p, stokes, jones, eps)
    ref = opolar.polar_vis(p.ant_enu, p.src_lmn, p.freq_hz, stokes, jones)
    for a in range(2):
        for b in range(2):
            assert oracle.rel_l2(v[..., a, b], ref[..., a, b]) <= eps, (a, b)
    assert rep["lattice"] == 1


def test_ideal_feeds_on_a_random_array(gpu_lib, ctx):
    p, stokes, _ = _case(181, n_ant=25, hex_layout=False, feeds=False)
    v, rep = _run(gpu_lib, ctx, p, stokes, None, 1e-6)
    ref = opolar.polar_vis(p.ant_enu, p.src_lmn, p.freq_hz, stokes)
    for a in range(2):
        for b in range(2):
            assert oracle.rel_l2(v[..., a, b], ref[..., a, b]) <= 1e-6, (a, b)
    assert rep["lattice"] == 0


def test_unpolarised_sky_matches_the_scalar_call(gpu_lib, ctx):
    import torch
    p, stokes, _ = _case(182, feeds=False)
    stokes[1:] = 0.0
    v, _ = _run(gpu_lib, ctx, p, stokes, None, 1e-10)
    w = torch.empty((p.n_freq, p.n_pairs, 2), dtype=torch.float64, device="cuda:0")
    ctx.simulate_dev(_dev(p.ant_enu), _dev(p.src_lmn), _dev(p.freq_hz), _dev(stokes[0]), None, w, eps=1e-10)
    torch.cuda.synchronize()
    o = w.cpu().numpy()
    s = o[..., 0] + 1j * o[..., 1]
    assert oracle.rel_l2(v[..., 0, 0], s) <= 2e-10 and oracle.rel_l2(v[..., 1, 1], s) <= 2e-10
    assert np.abs(v[..., 0, 1]).max() <= 1e-12 * np.abs(s).max()


def test_non_finite_stokes_is_rejected(gpu_lib, ctx):
    fv = gpu_lib
    p, stokes, jones = _case(183, n_ant=7, n_src=40)
    stokes[2, 1, 3] = np.nan
    with pytest.raises(fv.FvError, match="EINVAL"):
        _run(fv, ctx, p, stokes, jones, 1e-6)
