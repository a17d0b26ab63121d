"""Drift scans with the front end on the device (rotation to ENU per
sidereal time and the analytic beam, paper sections 2.3 and 2.4) against the
oracle's own rotation, beam and exact sum."""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import frontend

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(torch.device("cuda:0"))


def _run(fv, ctx, d, eps=None, flags=0, beam_fwhm=None):
    import torch
    vis = torch.empty((len(d.lst), len(d.freq_hz), d.n_pairs, 2), dtype=torch.float64, device="cuda:0")
    rep = ctx.simulate_drift(d.ant_enu, _dev(d.src_eq), d.freq_hz, _dev(d.flux), d.lst, d.latitude,
                             d.beam_fwhm if beam_fwhm is None else beam_fwhm, d.beam_nu_ref, vis,
                             eps=d.eps if eps is None else eps, flags=flags)
    torch.cuda.synchronize()
    o = vis.cpu().numpy()
    return o[..., 0] + 1j * o[..., 1], rep


def _ref(d, beam_fwhm=None):
    return frontend.drift_vis(d.ant_enu, d.src_eq, d.freq_hz, d.flux, d.lst, d.latitude,
                              d.beam_fwhm if beam_fwhm is None else beam_fwhm, d.beam_nu_ref)


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("eps", [1e-4, 1e-6, 1e-10])
def test_hex_drift_matches_oracle(gpu_lib, ctx, eps):
    d = synth.small_drift(1, n_ant=37, n_src=800, n_freq=3, n_time=4)
    v, rep = _run(gpu_lib, ctx, d, eps=eps)
    ref = _ref(d)
    for t in range(len(d.lst)):
        assert oracle.rel_l2(v[t], ref[t]) <= eps
    assert rep["lattice"] == 1


def test_random_array_drift_takes_type3(gpu_lib, ctx):
    d = synth.small_drift(2, n_ant=24, n_src=600, n_freq=2, n_time=3, hex_layout=False)
    v, rep = _run(gpu_lib, ctx, d)
    ref = _ref(d)
    for t in range(len(d.lst)):
        assert oracle.rel_l2(v[t], ref[t]) <= d.eps
    assert rep["lattice"] == 0 and rep["dim"] == 2


def test_non_coplanar_array_drift_runs_3d(gpu_lib, ctx):
    d = synth.small_drift(3, n_ant=16, n_src=300, n_freq=2, n_time=2, hex_layout=False, three_d=True)
    v, rep = _run(gpu_lib, ctx, d)
    ref = _ref(d)
    for t in range(len(d.lst)):
        assert oracle.rel_l2(v[t], ref[t]) <= d.eps
    assert rep["dim"] == 3


def test_unit_beam_and_single_time(gpu_lib, ctx):
    d = synth.small_drift(4, n_ant=19, n_src=400, n_freq=2, n_time=1)
    v, _ = _run(gpu_lib, ctx, d, beam_fwhm=0.0)
    assert oracle.rel_l2(v, _ref(d, beam_fwhm=0.0)) <= d.eps


def test_transiting_source_gives_its_flux(gpu_lib, ctx):
    import dataclasses
    d = synth.small_drift(5, n_ant=19, n_src=1, n_freq=2, n_time=1)
    ra, dec = float(d.lst[0]), d.latitude
    src = np.array([[math.cos(dec) * math.cos(ra), math.cos(dec) * math.sin(ra), math.sin(dec)]])
    d = dataclasses.replace(d, src_eq=src, flux=np.array([[2.0], [3.0]]))
    v, _ = _run(gpu_lib, ctx, d, eps=1e-10)
    assert np.allclose(v[0, 0], 2.0, atol=1e-8) and np.allclose(v[0, 1], 3.0, atol=1e-8)


def test_empty_sky_and_invalid_inputs(gpu_lib, ctx):
    import dataclasses
    fv = gpu_lib
    d = synth.small_drift(6, n_ant=7, n_src=0, n_freq=2, n_time=2)
    v, _ = _run(fv, ctx, d)
    assert np.all(v == 0)
    d = synth.small_drift(7, n_ant=7, n_src=50, n_freq=1, n_time=2)
    bad = dataclasses.replace(d, src_eq=d.src_eq * 1.01)
    with pytest.raises(fv.FvError, match="EINVAL"):
        _run(fv, ctx, bad)
    with pytest.raises(fv.FvError, match="EINVAL"):
        _run(fv, ctx, dataclasses.replace(d, latitude=2.0))
    flux = d.flux.copy()
    flux[0, 3] = np.nan
    with pytest.raises(fv.FvError, match="EINVAL"):
        _run(fv, ctx, dataclasses.replace(d, flux=flux))
    # the context stays usable
    v, _ = _run(fv, ctx, d)
    assert oracle.rel_l2(v, _ref(d)) <= d.eps


def test_drift_equals_device_calls_on_the_oracle_snapshots(gpu_lib, ctx):
    # each time of the drift is the plain device entry point on the snapshot the
    # oracle's rotation and beam produce
    d = synth.small_drift(8, n_ant=37, n_src=500, n_freq=2, n_time=2)
    v, _ = _run(gpu_lib, ctx, d)
    alpha, delta = frontend.radec(d.src_eq)
    for t, lst in enumerate(d.lst):
        e = frontend.enu(alpha, delta, float(lst), d.latitude)
        b = frontend.gaussian_beam(e, d.freq_hz, d.beam_fwhm, d.beam_nu_ref)
        hp = gpu_lib.HostProblem(d.ant_enu, e / np.linalg.norm(e, axis=1, keepdims=True), d.freq_hz, d.flux, b, d.eps)
        w = ctx.simulate_problem(hp)
        assert oracle.rel_l2(v[t], w) <= 2 * d.eps


def test_config4_drift_sampled(gpu_lib, ctx):
    d = synth.config4_drift(n_lst=4, n_freq=6, n_cap=20000, n_iso=500)
    v, rep = _run(gpu_lib, ctx, d)
    sub = synth.subset_pairs(d.ant_enu.shape[0], 300, 3)
    ref = frontend.drift_vis(d.ant_enu, d.src_eq, d.freq_hz, d.flux, d.lst, d.latitude, d.beam_fwhm,
                             d.beam_nu_ref, pairs=sub)
    assert oracle.rel_l2(v[:, :, sub], ref) <= d.eps


def test_horizon_sources_are_dropped_and_counted(gpu_lib, ctx):
    d = synth.small_drift(9, n_ant=19, n_src=1000, n_freq=2, n_time=3)
    v, rep = _run(gpu_lib, ctx, d)
    alpha, delta = frontend.radec(d.src_eq)
    visible = sum(int((frontend.enu(alpha, delta, float(t), d.latitude)[:, 2] > 0).sum()) for t in d.lst)
    assert 0 < visible < 3 * 1000
    assert rep["src_pairs"] == visible * d.n_pairs * len(d.freq_hz)
    assert oracle.rel_l2(v, _ref(d)) <= d.eps


def test_invalid_source_below_the_horizon_is_still_rejected(gpu_lib, ctx):
    import dataclasses
    d = synth.small_drift(10, n_ant=7, n_src=60, n_freq=1, n_time=1)
    alpha, delta = frontend.radec(d.src_eq)
    below = int(np.argmin(frontend.enu(alpha, delta, float(d.lst[0]), d.latitude)[:, 2]))
    src = d.src_eq.copy()
    src[below] *= np.nan
    with pytest.raises(gpu_lib.FvError, match="EINVAL"):
        _run(gpu_lib, ctx, dataclasses.replace(d, src_eq=src))
