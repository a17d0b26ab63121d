"""Pins for the oracle: values fixed by the paper's equations and by
mathematics, not by the oracle itself.  CPU only."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import es_kernel, type3

C = 299792458.0
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _vis(ant, src, freq, flux, beam=None, **kw):
    return oracle.direct_vis(np.asarray(ant, float), np.asarray(src, float), np.asarray(freq, float),
                             np.asarray(flux, float), beam, **kw)


def _pairs(n):
    i, j = np.triu_indices(n)
    return i, j


# ---------------------------------------------------------------- closed forms
def test_sign_and_orientation_fixture():
    fx = json.load(open(os.path.join(GOLD, "sign_convention.json")))
    V = _vis(fx["ant_enu"], fx["src_lmn"], fx["freq_hz"], fx["flux"])
    assert np.allclose(V[0].real, fx["vis_re"], atol=1e-12)
    assert np.allclose(V[0].imag, fx["vis_im"], atol=1e-12)


def test_zenith_source_coplanar_is_constant():
    p = synth.small_problem(1, n_ant=9, n_src=1, n_freq=3)
    src = np.array([[0.0, 0.0, 1.0]])
    V = _vis(p.ant_enu, src, p.freq_hz, np.full((3, 1), 3.5))
    assert np.allclose(V, 3.5, rtol=0, atol=1e-13)


def test_zenith_source_noncoplanar_phase_is_up_term():
    ant = np.array([[0.0, 0.0, 0.0], [3.0, -2.0, 0.25], [-1.0, 4.0, -0.5]])
    nu = 150e6
    V = _vis(ant, [[0.0, 0.0, 1.0]], [nu], [[1.0]])
    i, j = _pairs(3)
    expect = np.exp(-2j * math.pi * nu / C * (ant[i, 2] - ant[j, 2]))
    assert np.allclose(V[0], expect, atol=1e-13)
    assert np.allclose(np.abs(V[0]), 1.0, atol=1e-14)


def test_autos_equal_beam_weighted_flux_sum():
    p = synth.small_problem(2, n_ant=7, n_src=60, n_freq=2)
    V = oracle.direct_problem(p)
    i, j = _pairs(p.n_ant)
    autos = V[:, i == j]
    tot = p.strengths().sum(1)
    assert np.allclose(autos, tot[:, None], rtol=1e-13, atol=0)


def test_empty_sky_is_zero():
    p = synth.small_problem(3, n_ant=5, n_src=4, n_freq=2)
    V = _vis(p.ant_enu, np.zeros((0, 3)), p.freq_hz, np.zeros((2, 0)))
    assert V.shape == (2, 15) and np.all(V == 0)


def test_single_antenna_autos_only():
    V = _vis([[1.0, 2.0, 3.0]], [[0.6, 0.0, 0.8], [0.0, 0.6, 0.8]], [1e8], [[1.0, 2.0]])
    assert V.shape == (1, 1) and abs(V[0, 0] - 3.0) < 1e-14


def test_monopole_matches_analytic_hemisphere():
    # Uniform brightness I0 over the hemisphere: for a horizontal baseline of
    # |u| wavelengths, V = 2 pi I0 sin(2 pi |u|) / (2 pi |u|)
    # (int over the unit disk of exp(-2 pi i u.r) / sqrt(1 - r^2) d^2 r).
    npix = 400_000
    pix = synth.fibonacci_sphere(npix)
    up = pix[pix[:, 2] > 0]
    omega = 4 * math.pi / npix
    ant = np.array([[0.0, 0.0, 0.0], [0.5, 0.0, 0.0], [0.0, 1.5, 0.0], [2.0, 2.0, 0.0]])
    V = _vis(ant, up, [C], np.full((1, up.shape[0]), omega))[0]
    i, j = _pairs(4)
    u = np.hypot(ant[i, 0] - ant[j, 0], ant[i, 1] - ant[j, 1])
    x = 2 * math.pi * u
    expect = 2 * math.pi * np.where(u > 0, np.sin(x) / np.where(u > 0, x, 1), 1.0)
    assert np.max(np.abs(V - expect)) < 3e-3 * 2 * math.pi


# ---------------------------------------------------------------- invariants
def test_hermitian_under_mirrored_array():
    p = synth.small_problem(4, n_ant=8, n_src=30, n_freq=2, three_d=True)
    V = oracle.direct_problem(p)
    W = _vis(-p.ant_enu, p.src_lmn, p.freq_hz, p.flux, p.beam)
    assert np.allclose(W, np.conj(V), atol=1e-12 * np.abs(V).max())


def test_swapped_antenna_order_conjugates():
    p = synth.small_problem(5, n_ant=6, n_src=25, n_freq=1, three_d=True)
    V = oracle.direct_problem(p)
    rev = p.ant_enu[::-1].copy()
    W = _vis(rev, p.src_lmn, p.freq_hz, p.flux, p.beam)
    n = p.n_ant
    i, j = _pairs(n)
    lookup = {(a, b): k for k, (a, b) in enumerate(zip(i, j))}
    for k, (a, b) in enumerate(zip(i, j)):
        # pair (a,b) of the reversed array is antennas (n-1-a, n-1-b) = (jj, ii) with jj >= ii
        kk = lookup[(n - 1 - b, n - 1 - a)]
        assert abs(W[0, k] - np.conj(V[0, kk])) < 1e-12 * np.abs(V).max()


def test_linearity_in_strength():
    p = synth.small_problem(6, n_ant=6, n_src=20, n_freq=2)
    rng = np.random.default_rng(0)
    f2 = rng.normal(size=p.flux.shape)
    V1 = _vis(p.ant_enu, p.src_lmn, p.freq_hz, p.flux)
    V2 = _vis(p.ant_enu, p.src_lmn, p.freq_hz, f2)
    V3 = _vis(p.ant_enu, p.src_lmn, p.freq_hz, 2.0 * p.flux - 3.0 * f2)
    assert np.allclose(V3, 2 * V1 - 3 * V2, atol=1e-12 * np.abs(V3).max())


def test_common_translation_invariance():
    p = synth.small_problem(7, n_ant=7, n_src=25, n_freq=2, three_d=True)
    V = oracle.direct_problem(p)
    W = _vis(p.ant_enu + np.array([123.0, -45.0, 6.0]), p.src_lmn, p.freq_hz, p.flux, p.beam)
    assert np.allclose(W, V, atol=1e-10 * np.abs(V).max())


def test_joint_rotation_invariance():
    p = synth.small_problem(8, n_ant=7, n_src=25, n_freq=1, three_d=True)
    V = oracle.direct_problem(p)
    a, b = 0.7, -0.3
    Rz = np.array([[math.cos(a), -math.sin(a), 0], [math.sin(a), math.cos(a), 0], [0, 0, 1]])
    Rx = np.array([[1, 0, 0], [0, math.cos(b), -math.sin(b)], [0, math.sin(b), math.cos(b)]])
    R = Rx @ Rz
    W = _vis(p.ant_enu @ R.T, p.src_lmn @ R.T, p.freq_hz, p.flux, p.beam)
    assert np.allclose(W, V, atol=1e-10 * np.abs(V).max())


def test_frequency_length_scaling_invariance():
    p = synth.small_problem(9, n_ant=6, n_src=25, n_freq=2, three_d=True)
    V = oracle.direct_problem(p)
    W = _vis(p.ant_enu / 2.5, p.src_lmn, p.freq_hz * 2.5, p.flux, p.beam)
    assert np.allclose(W, V, atol=1e-10 * np.abs(V).max())


def test_drop_up_equals_full_on_flat_array():
    p = synth.small_problem(10, n_ant=7, n_src=30, n_freq=2)
    assert np.all(p.ant_enu[:, 2] == 0)
    assert np.array_equal(oracle.direct_problem(p), oracle.direct_problem(p, drop_up=True))


def test_pair_subset_matches_full_output():
    p = synth.small_problem(11, n_ant=9, n_src=15, n_freq=2)
    V = oracle.direct_problem(p)
    sub = synth.subset_pairs(p.n_ant, 11, 0)
    assert np.array_equal(oracle.direct_problem(p, pairs=sub), V[:, sub])


# ---------------------------------------------------------------- brute force
def test_brute_force_mpmath_tiny():
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 50
    p = synth.small_problem(12, n_ant=5, n_src=8, n_freq=2, three_d=True)
    V = oracle.direct_problem(p)
    c = p.strengths()
    i, j = _pairs(p.n_ant)
    worst = 0.0
    for f in range(p.n_freq):
        k = mp.mpf(p.freq_hz[f]) / mp.mpf(C)
        for q in range(len(i)):
            acc = mp.mpc(0)
            for s in range(p.n_src):
                dot = sum((mp.mpf(p.ant_enu[i[q], a]) - mp.mpf(p.ant_enu[j[q], a])) * mp.mpf(p.src_lmn[s, a])
                          for a in range(3))
                acc += mp.mpf(c[f, s]) * mp.expjpi(-2 * k * dot)
            ref = complex(acc)
            worst = max(worst, abs(V[f, q] - ref) / max(abs(ref), 1e-300))
    assert worst < 1e-13


# ---------------------------------------------------------------- ES kernel
@pytest.mark.parametrize("xi", [0.0, 0.7, 3.0, 9.5])
def test_phihat_beta_zero_is_box_transform(xi):
    # beta = 0: phi = 1 on [-1, 1], whose cosine transform is 2 sin(xi)/xi.
    got = es_kernel.es_phihat([xi], 0.0)[0]
    want = 2.0 if xi == 0 else 2 * math.sin(xi) / xi
    assert abs(got - want) < 1e-14


@pytest.mark.parametrize("w,xi", [(6, 0.0), (8, 2.5), (12, 9.4), (8, 6.28)])
def test_phihat_against_adaptive_quadrature(w, xi):
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 30
    beta = es_kernel.es_beta(w)
    f = lambda z: mp.e ** (beta * (mp.sqrt(1 - z * z) - 1)) * mp.cos(xi * z)
    ref = float(mp.quad(f, [-1, 0, 1]))
    got = es_kernel.es_phihat([xi], beta)[0]
    assert abs(got - ref) <= 1e-14 * abs(ref)


def test_phi_support_and_peak():
    z = np.array([-1.5, -1.0, 0.0, 0.5, 1.0, 1.0000001])
    v = es_kernel.es_phi(z, 10.0)
    assert v[0] == 0 and v[-1] == 0 and v[2] == 1.0
    assert abs(v[1] - math.exp(-10.0)) < 1e-18 and abs(v[4] - math.exp(-10.0)) < 1e-18


# ---------------------------------------------------------------- type-3 steps
def test_kernel_width_rule():
    assert [type3.kernel_width(e) for e in (1e-4, 1e-6, 1e-10, 1e-12)] == [6, 8, 12, 14]


def test_smooth_sizes():
    assert type3.next_smooth_even(1523) == 1536
    assert type3.next_smooth_even(750) == 750
    assert type3.next_smooth_even(7) == 8
    for n in range(2, 400):
        m = type3.next_smooth_even(n)
        assert m >= n and m % 2 == 0


def test_grid_size_matches_full_sky_equation():
    # full-sky sources (S = 1 per axis): the grid-size equation reduces to
    # n = ceil(4 sigma b_max nu / c + w) with b_max the half-width of the
    # centred baseline box (paper, full-sky form of the grid-size equation).
    # This fixes X as an angular frequency (radians).
    ant = np.array([[-40.0, 0.0, 0], [40.0, 0.0, 0], [0.0, -25.0, 0], [0.0, 25.0, 0], [7.0, 3.0, 0]])
    src = np.array([[-1.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, -1.0, 0.0], [0.0, 1.0, 0.0]])
    nu = 150e6
    pl = type3.make_plan(ant, src, np.array([nu]), 1e-6, 2)
    b = type3.baselines(ant)[:, :2]
    bf, _ = type3.fold_targets(b, pl.fold_axis)
    assert np.all(bf[:, pl.fold_axis] >= 0)
    for a in range(2):
        half = 0.5 * (bf[:, a].max() - bf[:, a].min())
        n_eq = math.ceil(4 * 2.0 * half * nu / C + pl.w)
        assert pl.n1[0][a] == type3.next_smooth_even(n_eq)


def test_fft_step_against_explicit_dft():
    p = synth.small_problem(13, n_ant=4, n_src=6, n_freq=1)
    pl = type3.make_plan(p.ant_enu, p.src_lmn, p.freq_hz, 1e-3, 2)
    rng = np.random.default_rng(1)
    n1 = pl.n1[0]
    bt = rng.normal(size=(n1[1], n1[0])) + 1j * rng.normal(size=(n1[1], n1[0]))
    g = type3.fft_upsampled(pl, 0, bt)
    n2 = pl.n2(0)
    my = np.arange(n1[1]) - n1[1] // 2
    mx = np.arange(n1[0]) - n1[0] // 2
    for (py, px) in [(0, 0), (1, 3), (n2[1] - 1, 5), (7, n2[0] - 2)]:
        ref = np.sum(bt * np.exp(2j * math.pi * (np.outer(my * py / n2[1], np.ones(n1[0]))
                                                + np.outer(np.ones(n1[1]), mx * px / n2[0]))))
        assert abs(g[py, px] - ref) < 1e-10 * np.abs(bt).sum()


def test_spread_step_against_cellwise_sum():
    p = synth.small_problem(14, n_ant=5, n_src=7, n_freq=1)
    pl = type3.make_plan(p.ant_enu, p.src_lmn, p.freq_hz, 1e-4, 2)
    c = p.strengths()[0]
    bt = type3.spread(pl, 0, p.src_lmn, c)
    # undo the mode deconvolution, then compare every cell with a direct sum
    n1, w = pl.n1[0], pl.w
    X = pl.X[0]
    for a in range(2):
        alpha2 = w * math.pi / (2 * n1[a])
        m = np.arange(n1[a]) - n1[a] // 2
        p2 = alpha2 * es_kernel.es_phihat(alpha2 * m, pl.beta)
        bt = bt * (p2[None, :] if a == 0 else p2[:, None])
    s = p.src_lmn[:, :2]
    cp = c * np.exp(1j * ((s - pl.s_c) @ pl.x_c[0]))
    gx = n1[0] / 2 + (s[:, 0] - pl.s_c[0]) * 2 * X[0] / math.pi
    gy = n1[1] / 2 + (s[:, 1] - pl.s_c[1]) * 2 * X[1] / math.pi
    for ly in range(n1[1]):
        for lx in range(0, n1[0], 3):
            zx = (lx - gx) / (w / 2)
            zy = (ly - gy) / (w / 2)
            ref = np.sum(cp * es_kernel.es_phi(zx, pl.beta) * es_kernel.es_phi(zy, pl.beta))
            assert abs(bt[ly, lx] - ref) < 1e-12 * np.abs(c).sum()


@pytest.mark.parametrize("dim,eps", [(2, 1e-4), (2, 1e-6), (2, 1e-10), (3, 1e-6)])
def test_type3_steps_within_eps_of_direct_sum(dim, eps):
    p = synth.small_problem(20 + dim, n_ant=14, n_src=80, n_freq=2, three_d=(dim == 3), radius=80.0)
    V = oracle.direct_problem(p)
    V3 = type3.type3_vis(p.ant_enu, p.src_lmn, p.freq_hz, p.strengths(), eps, dim)
    assert oracle.rel_l2(V3, V) <= eps


@pytest.mark.parametrize("dim", [2, 3])
def test_unfolded_type3_steps_within_eps_of_direct_sum(dim):
    # the paper's plain targets (no reflection into a half-space): the same
    # steps on the unfolded baseline box stay within eps of the exact sum, and
    # that box is the tight box of the baselines as given
    p = synth.small_problem(40 + dim, n_ant=13, n_src=70, n_freq=2, three_d=(dim == 3), radius=70.0)
    V = oracle.direct_problem(p)
    V3 = type3.type3_vis(p.ant_enu, p.src_lmn, p.freq_hz, p.strengths(), 1e-8, dim, fold=False)
    assert oracle.rel_l2(V3, V) <= 1e-8
    pu = type3.make_plan(p.ant_enu, p.src_lmn, p.freq_hz, 1e-8, dim, fold=False)
    pf = type3.make_plan(p.ant_enu, p.src_lmn, p.freq_hz, 1e-8, dim)
    assert pu.fold_axis == -1 and pf.fold_axis >= 0
    b = type3.baselines(p.ant_enu)[:, :dim]
    assert np.allclose(pu.b_c - pu.B, b.min(0), rtol=0, atol=1e-12)
    assert np.allclose(pu.b_c + pu.B, b.max(0), rtol=0, atol=1e-12)


def test_type3_error_falls_with_eps():
    p = synth.config1()
    V = oracle.direct_problem(p)
    errs = [oracle.rel_l2(type3.type3_vis(p.ant_enu, p.src_lmn, p.freq_hz, p.strengths(), e, 2), V)
            for e in (1e-3, 1e-5, 1e-7, 1e-9, 1e-11)]
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert all(e <= t for e, t in zip(errs, (1e-3, 1e-5, 1e-7, 1e-9, 1e-11)))


def test_fold_reflects_into_halfspace():
    b = np.array([[1.0, -2.0], [0.0, 0.0], [-3.0, 0.0], [2.0, 5.0], [-1.0, -1.0]])
    bf, flip = type3.fold_targets(b, 1)
    assert np.all(bf[:, 1] >= 0)
    assert list(flip) == [True, False, True, False, True]
