"""Spectral-basis evaluation (paper appendix A) through fv_simulate_basis
against the oracle's step-by-step basis evaluation, and against the exact sum
where the basis holds the spectra exactly."""
import dataclasses

import numpy as np
import pytest

import oracle
import synth
from oracle import basis as obasis

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(torch.device("cuda:0"))


def _run(fv, ctx, p, K, eps):
    import torch
    vis = torch.empty((p.n_freq, p.n_pairs, 2), dtype=torch.float64, device="cuda:0")
    rep = ctx.simulate_basis(_dev(p.ant_enu), _dev(p.src_lmn), _dev(p.freq_hz), _dev(p.flux),
                             None if p.beam is None else _dev(p.beam), vis, K, eps=eps)
    torch.cuda.synchronize()
    o = vis.cpu().numpy()
    return o[..., 0] + 1j * o[..., 1], rep


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("eps,K", [(1e-6, 6), (1e-10, 10)])
def test_matches_the_oracle_basis_steps(gpu_lib, ctx, eps, K):
    p = synth.small_problem(190, n_ant=24, n_src=800, n_freq=12, hex_layout=False)
    v, rep = _run(gpu_lib, ctx, p, K, eps)
    ref = obasis.basis_vis(p.ant_enu, p.src_lmn, p.freq_hz, p.flux, p.beam, K)
    assert oracle.rel_l2(v, ref) <= eps
    assert rep["lattice"] == 0


def test_complete_basis_is_the_exact_sum(gpu_lib, ctx):
    p = synth.small_problem(191, n_ant=19, n_src=500, n_freq=6, hex_layout=True)
    v, _ = _run(gpu_lib, ctx, p, 6, 1e-10)
    assert oracle.rel_l2(v, oracle.direct_problem(p)) <= 1e-10


def test_polynomial_spectra_are_exact_at_the_product_degree(gpu_lib, ctx):
    p = synth.small_problem(192, n_ant=30, n_src=600, n_freq=10, three_d=True)
    rng = np.random.default_rng(5)
    x = (p.freq_hz - p.freq_hz.mean()) / (0.5 * np.ptp(p.freq_hz))
    flux = rng.uniform(0.5, 1.5, p.n_src)[None] + rng.uniform(-0.3, 0.3, p.n_src)[None] * x[:, None]
    beam = rng.uniform(0.5, 1.0, p.n_src)[None] + rng.uniform(-0.2, 0.2, p.n_src)[None] * x[:, None]
    q = dataclasses.replace(p, flux=flux, beam=beam)
    v, rep = _run(gpu_lib, ctx, q, 3, 1e-6)
    assert rep["dim"] == 3
    assert oracle.rel_l2(v, oracle.direct_problem(q)) <= 1e-6


def test_bad_basis_size_and_empty_sky(gpu_lib, ctx):
    fv = gpu_lib
    p = synth.small_problem(193, n_ant=7, n_src=30, n_freq=4)
    with pytest.raises(fv.FvError, match="EINVAL"):
        _run(fv, ctx, p, 5, 1e-6)
    with pytest.raises(fv.FvError, match="EINVAL"):
        _run(fv, ctx, p, 0, 1e-6)
    e = synth.small_problem(194, n_ant=7, n_src=0, n_freq=3)
    v, _ = _run(fv, ctx, e, 2, 1e-6)
    assert np.all(v == 0)
