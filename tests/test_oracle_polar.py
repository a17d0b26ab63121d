"""Pins of the oracle's polarised sum (no GPU): unpolarised sky through ideal
feeds, Stokes V alone, the Hermitian pair symmetry, feed rotation leaving
the trace unchanged, and a zenith closed form."""
import math

import numpy as np

import oracle
import synth
from oracle import polar


def _setup(seed, n_ant=7, n_src=30, n_freq=2):
    rng = np.random.default_rng(seed)
    ant = synth.hex_array(n_ant)
    src = synth.workloads.isotropic_hemisphere(rng, n_src)
    freq = np.linspace(120e6, 180e6, n_freq)
    I = rng.uniform(0.5, 2.0, (n_freq, n_src))
    QUV = rng.uniform(-0.3, 0.3, (3, n_freq, n_src))
    return rng, ant, src, freq, np.concatenate([I[None], QUV])


def test_unpolarised_sky_through_ideal_feeds():
    _, ant, src, freq, st = _setup(1)
    st[1:] = 0.0
    v = polar.polar_vis(ant, src, freq, st)
    d = oracle.direct_vis(ant, src, freq, st[0])
    assert np.allclose(v[..., 0, 0], d, atol=1e-12) and np.allclose(v[..., 1, 1], d, atol=1e-12)
    assert np.all(np.abs(v[..., 0, 1]) < 1e-12) and np.all(np.abs(v[..., 1, 0]) < 1e-12)


def test_stokes_v_alone_is_imaginary_cross_hand():
    _, ant, src, freq, st = _setup(2)
    st[:3] = 0.0
    v = polar.polar_vis(ant, src, freq, st)
    d = oracle.direct_vis(ant, src, freq, st[3])
    assert np.allclose(v[..., 0, 1], 1j * d, atol=1e-12) and np.allclose(v[..., 1, 0], -1j * d, atol=1e-12)
    assert np.all(np.abs(v[..., 0, 0]) < 1e-12)


def test_hermitian_pair_symmetry_with_complex_feeds():
    rng, ant, src, freq, st = _setup(3)
    jones = rng.normal(size=(len(freq), src.shape[0], 2, 2)) + 1j * rng.normal(size=(len(freq), src.shape[0], 2, 2))
    v = polar.polar_vis(ant, src, freq, st, jones)
    # reversing the array order swaps i and j: V_ji = V_ij^H for a shared beam
    w = polar.polar_vis(ant[::-1], src, freq, st, jones)
    n = len(ant)
    iu, ju = np.triu_indices(n)
    idx = {(i, j): k for k, (i, j) in enumerate(zip(iu, ju))}
    for k, (i, j) in enumerate(zip(iu, ju)):
        kk = idx[(n - 1 - j, n - 1 - i)]
        assert np.allclose(w[:, kk], np.conj(np.swapaxes(v[:, k], -1, -2)), atol=1e-10)


def test_feed_rotation_keeps_the_trace():
    _, ant, src, freq, st = _setup(4)
    th = 0.7
    R = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    jones = np.broadcast_to(R, (len(freq), src.shape[0], 2, 2))
    v = polar.polar_vis(ant, src, freq, st, jones)
    d = oracle.direct_vis(ant, src, freq, st[0])
    assert np.allclose(v[..., 0, 0] + v[..., 1, 1], 2 * d, atol=1e-11)


def test_zenith_source_closed_form():
    ant = synth.hex_array(7)
    src = np.array([[0.0, 0.0, 1.0]])
    st = np.array([1.0, 0.2, -0.1, 0.05]).reshape(4, 1, 1)
    A = np.array([[[[0.9, 0.1j], [0.05, 0.8]]]])
    v = polar.polar_vis(ant, src, np.array([150e6]), st, A)
    C = np.array([[1.2, -0.1 + 0.05j], [-0.1 - 0.05j, 0.8]])
    want = A[0, 0] @ C @ A[0, 0].conj().T
    assert np.allclose(v[0], want[None], atol=1e-14)
