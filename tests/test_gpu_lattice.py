"""GPU type-1 path for lattice arrays (paper section 2.2.1) against the oracle."""
import numpy as np
import pytest

import oracle
import synth
from oracle import type1

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context(0)
    yield c
    c.close()


def _run(fv, ctx, p, eps=None, flags=0):
    v = ctx.simulate_problem(fv.HostProblem.of(p, eps=eps, flags=flags))
    return v, ctx.last_report


@pytest.mark.parametrize("eps", [1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-8, 1e-10, 1e-12])
def test_hex_array_takes_the_lattice_path_within_eps(gpu_lib, ctx, eps):
    p = synth.small_problem(130, n_ant=61, n_src=3000, n_freq=3, hex_layout=True)
    v, rep = _run(gpu_lib, ctx, p, eps=eps)
    assert rep["lattice"] == 1 and rep["prec_bits"] == (32 if eps >= 1e-6 else 64)
    assert rep["w"] == type1.kernel_width_type1(eps)   # every FP32 width 3..7 is met
    assert oracle.rel_l2(v, oracle.direct_problem(p)) <= eps


def test_lattice_and_type3_paths_agree(gpu_lib, ctx):
    fv = gpu_lib
    p = synth.small_problem(131, n_ant=37, n_src=2000, n_freq=2, hex_layout=True)
    v1, r1 = _run(fv, ctx, p, eps=1e-10)
    v3, r3 = _run(fv, ctx, p, eps=1e-10, flags=fv.NO_LATTICE)
    assert r1["lattice"] == 1 and r3["lattice"] == 0
    assert oracle.rel_l2(v1, v3) <= 2e-10


def test_lattice_grid_matches_the_oracle_plan(gpu_lib, ctx):
    p = synth.small_problem(132, n_ant=127, n_src=500, n_freq=1, hex_layout=True)
    v, rep = _run(gpu_lib, ctx, p, eps=1e-6)
    lat = type1.find_lattice(p.ant_enu, type1.lattice_tolerance(1e-6, p.freq_hz))
    nf = type1.grid_sizes(lat, rep["w"])
    assert sorted(rep["n1"][:2]) == sorted(nf.tolist())
    assert oracle.rel_l2(v, oracle.direct_problem(p)) <= 1e-6


def test_square_grid_array_and_many_sources(gpu_lib, ctx):
    d = 5.0
    ant = np.array([[i * d, j * d, 0.0] for i in range(12) for j in range(9)])
    rng = np.random.default_rng(3)
    src = synth.workloads.isotropic_hemisphere(rng, 20000)
    freq = np.array([120e6, 180e6])
    flux = synth.workloads.powerlaw_fluxes(rng, 20000)[None, :] * np.ones((2, 1))
    V = gpu_lib.Context.simulate(ctx, ant, src, freq, flux, None, eps=1e-6)
    assert ctx.last_report["lattice"] == 1
    sub = synth.subset_pairs(ant.shape[0], 600, 4)
    ref = oracle.direct_vis(ant, src, freq, flux, pairs=sub)
    assert oracle.rel_l2(V[:, sub], ref) <= 1e-6


def test_random_and_3d_arrays_stay_on_type3(gpu_lib, ctx):
    p = synth.small_problem(133, n_ant=30, n_src=300, n_freq=1)
    v, rep = _run(gpu_lib, ctx, p, eps=1e-6)
    assert rep["lattice"] == 0
    p3 = synth.small_problem(134, n_ant=19, n_src=300, n_freq=1, three_d=True)
    v, rep = _run(gpu_lib, ctx, p3, eps=1e-6)
    assert rep["lattice"] == 0 and rep["dim"] == 3


def test_lattice_in_batch_and_graph_calls(gpu_lib, ctx):
    fv = gpu_lib
    a = synth.small_problem(135, n_ant=37, n_src=800, n_freq=2, hex_layout=True)
    b = synth.small_problem(136, n_ant=20, n_src=600, n_freq=2)
    outs = ctx.simulate_batch([fv.HostProblem.of(a), fv.HostProblem.of(b)])
    for p, v in zip((a, b), outs):
        assert oracle.rel_l2(v, oracle.direct_problem(p)) <= p.eps
    for _ in range(3):
        v, _ = _run(fv, ctx, a, flags=fv.GRAPH)
        assert oracle.rel_l2(v, oracle.direct_problem(a)) <= a.eps


@pytest.mark.parametrize("scale", [1e-30, 1e30])
def test_lattice_fixed_point_grid_keeps_extreme_and_signed_strengths(gpu_lib, ctx, scale):
    # 9000 sources span three spreading chunks of 4096: the first chunk holds
    # only zero strengths, the others mixed signs at an extreme magnitude.
    import dataclasses
    p = synth.small_problem(137, n_ant=37, n_src=9000, n_freq=2, hex_layout=True, beam=False)
    rng = np.random.default_rng(11)
    flux = p.flux * scale * np.where(rng.random(p.flux.shape) < 0.5, -1.0, 1.0)
    flux[:, :4096] = 0.0
    p = dataclasses.replace(p, flux=flux)
    v, rep = _run(gpu_lib, ctx, p, eps=1e-6)
    assert rep["lattice"] == 1
    assert oracle.rel_l2(v, oracle.direct_problem(p)) <= 1e-6


@pytest.mark.parametrize("eps", [1e-6, 1e-12])
@pytest.mark.parametrize("n_src", [37, 300, 1500])
def test_lattice_few_sources_per_chunk(gpu_lib, ctx, eps, n_src):
    # chunks far below the fixed-point bound's source count: one product per
    # cell must still stay within the FMA rounding range
    p = synth.small_problem(138, n_ant=37, n_src=n_src, n_freq=2, hex_layout=True)
    v, rep = _run(gpu_lib, ctx, p, eps=eps)
    assert rep["lattice"] == 1
    assert oracle.rel_l2(v, oracle.direct_problem(p)) <= eps
