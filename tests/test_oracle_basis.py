"""Pins of the oracle's spectral-basis evaluation (no GPU): a complete basis
reproduces the direct sum, polynomial spectra are exact once the basis holds
their product's degree, the basis is orthonormal with symmetric structure
constants, and the error falls with the basis size for smooth spectra."""
import numpy as np

import oracle
import synth
from oracle import basis


def _setup(seed=1, n_freq=12):
    p = synth.small_problem(seed, n_ant=9, n_src=60, n_freq=n_freq)
    return p


def test_orthonormal_basis_and_symmetric_structure_constants():
    M = basis.spectral_basis(np.linspace(100e6, 200e6, 16), 6)
    assert np.allclose(M.T @ M, np.eye(6), atol=1e-13)
    d = basis.structure_constants(M)
    assert np.allclose(d, np.transpose(d, (1, 0, 2))) and np.allclose(d, np.transpose(d, (2, 1, 0)))
    # the first column is the constant, so d[0, j, k] = delta_jk / sqrt(n)
    assert np.allclose(d[0], np.eye(6) * M[0, 0], atol=1e-13)


def test_complete_basis_is_the_direct_sum():
    p = _setup(2, n_freq=8)
    v = basis.basis_vis(p.ant_enu, p.src_lmn, p.freq_hz, p.flux, p.beam, K=8)
    assert oracle.rel_l2(v, oracle.direct_problem(p)) < 1e-12


def test_polynomial_spectra_exact_at_product_degree():
    import dataclasses
    p = _setup(3, n_freq=10)
    rng = np.random.default_rng(3)
    x = (p.freq_hz - 150e6) / 50e6
    a, b = rng.uniform(0.5, 1.5, p.n_src), rng.uniform(-0.3, 0.3, p.n_src)
    c, e = rng.uniform(0.5, 1.0, p.n_src), rng.uniform(-0.2, 0.2, p.n_src)
    flux = a[None] + b[None] * x[:, None]                 # degree 1 in frequency
    beam = c[None] + e[None] * x[:, None]                 # degree 1
    q = dataclasses.replace(p, flux=flux, beam=beam)
    ref = oracle.direct_problem(q)
    assert oracle.rel_l2(basis.basis_vis(q.ant_enu, q.src_lmn, q.freq_hz, flux, beam, K=3), ref) < 1e-12
    assert oracle.rel_l2(basis.basis_vis(q.ant_enu, q.src_lmn, q.freq_hz, flux, beam, K=2), ref) > 1e-4
    # constant spectra need one function
    q1 = dataclasses.replace(p, flux=np.broadcast_to(a, flux.shape).copy(), beam=None)
    assert oracle.rel_l2(basis.basis_vis(q1.ant_enu, q1.src_lmn, q1.freq_hz, q1.flux, None, K=1),
                         oracle.direct_problem(q1)) < 1e-12


def test_error_falls_with_basis_size_for_smooth_spectra():
    p = _setup(4, n_freq=24)
    ref = oracle.direct_problem(p)
    errs = [oracle.rel_l2(basis.basis_vis(p.ant_enu, p.src_lmn, p.freq_hz, p.flux, p.beam, K=k), ref)
            for k in (2, 4, 6, 8)]
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
