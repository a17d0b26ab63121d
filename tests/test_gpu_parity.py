"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle."""
import numpy as np
import pytest

import oracle
import synth
from oracle import type3

pytestmark = pytest.mark.gpu


def _run(fv, ctx, p, eps=None, flags=0):
    hp = fv.HostProblem.of(p, eps=eps, flags=flags)
    return ctx.simulate_problem(hp), ctx.last_report


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context(0)
    yield c
    c.close()


# ---------------------------------------------------------------- end to end
@pytest.mark.parametrize("no_lattice", [False, True])
def test_config1_full_output_fp64(gpu_lib, ctx, no_lattice):
    # the 37-antenna hex array is a lattice: the type-1 path by default, the
    # type-3 path when it is switched off
    p = synth.config1()
    v, rep = _run(gpu_lib, ctx, p, flags=gpu_lib.NO_LATTICE if no_lattice else 0)
    ref = oracle.direct_problem(p)
    assert rep["prec_bits"] == 64 and rep["dim"] == 2 and rep["lattice"] == (0 if no_lattice else 1)
    assert oracle.rel_l2(v, ref) <= p.eps


@pytest.mark.parametrize("no_lattice", [False, True])
@pytest.mark.parametrize("eps", [1e-4, 1e-5, 1e-6, 1e-8, 1e-10, 1e-12])
def test_small_2d_eps_sweep(gpu_lib, ctx, eps, no_lattice):
    # hex array: type-1 lattice path by default, type-3 with it switched off
    p = synth.small_problem(31, n_ant=40, n_src=700, n_freq=3, hex_layout=True)
    v, rep = _run(gpu_lib, ctx, p, eps=eps, flags=gpu_lib.NO_LATTICE if no_lattice else 0)
    assert rep["lattice"] == (0 if no_lattice else 1)
    ref = oracle.direct_problem(p)
    assert oracle.rel_l2(v, ref) <= eps


@pytest.mark.parametrize("eps", [1e-13, 1e-14])
def test_widest_kernels_at_the_smallest_eps(gpu_lib, ctx, eps):
    # the smallest accepted eps: FP64 grids and the widest spreading kernels
    # (w = 15 and 16), whose staged first-cell offsets are the largest.  The
    # error at 1e-14 sits just under eps (9.96e-15), so the spread order is
    # fixed (FV_DETERMINISTIC) and the result does not move between runs.
    p = synth.small_problem(33, n_ant=40, n_src=700, n_freq=3, hex_layout=True)
    v, rep = _run(gpu_lib, ctx, p, eps=eps, flags=gpu_lib.NO_LATTICE | gpu_lib.DETERMINISTIC)
    assert rep["lattice"] == 0 and rep["prec_bits"] == 64 and rep["w"] >= 15
    err = oracle.rel_l2(v, oracle.direct_problem(p))
    print(f"eps {eps:.0e}: w={rep['w']} rel_l2={err:.2e}", flush=True)
    assert err <= eps


@pytest.mark.parametrize("no_lattice", [False, True])
def test_eps_sweep_error_is_monotone(gpu_lib, ctx, no_lattice):
    p = synth.small_problem(32, n_ant=30, n_src=500, n_freq=2, hex_layout=True)
    ref = oracle.direct_problem(p)
    fl = gpu_lib.NO_LATTICE if no_lattice else 0
    errs = [oracle.rel_l2(_run(gpu_lib, ctx, p, eps=e, flags=fl)[0], ref) for e in (1e-3, 1e-5, 1e-7, 1e-9, 1e-11)]
    assert all(b < a for a, b in zip(errs, errs[1:])), errs


@pytest.mark.parametrize("eps", [1e-4, 1e-6, 1e-10])
def test_small_3d(gpu_lib, ctx, eps):
    p = synth.small_problem(33, n_ant=30, n_src=600, n_freq=2, three_d=True, radius=120.0, zhalf=3.0)
    v, rep = _run(gpu_lib, ctx, p, eps=eps)
    assert rep["dim"] == 3
    ref = oracle.direct_problem(p)
    assert oracle.rel_l2(v, ref) <= eps


def test_2d_and_3d_agree_on_flat_array(gpu_lib, ctx):
    p = synth.small_problem(34, n_ant=25, n_src=400, n_freq=2)
    v2, r2 = _run(gpu_lib, ctx, p, eps=1e-8, flags=gpu_lib.DIM_2D)
    v3, r3 = _run(gpu_lib, ctx, p, eps=1e-8, flags=gpu_lib.DIM_3D)
    assert r2["dim"] == 2 and r3["dim"] == 3
    assert oracle.rel_l2(v3, v2) <= 2e-8


def test_unfolded_equals_folded(gpu_lib, ctx):
    p = synth.small_problem(35, n_ant=20, n_src=300, n_freq=2)
    a, ra = _run(gpu_lib, ctx, p, eps=1e-9)
    b, rb = _run(gpu_lib, ctx, p, eps=1e-9, flags=gpu_lib.NO_FOLD)
    assert ra["fold_axis"] >= 0 and rb["fold_axis"] == -1
    ref = oracle.direct_problem(p)
    assert oracle.rel_l2(a, ref) <= 1e-9 and oracle.rel_l2(b, ref) <= 1e-9


def test_ragged_sizes_and_beamless(gpu_lib, ctx):
    # odd counts, no beam, sources not multiples of any tile or wave size
    p = synth.small_problem(36, n_ant=17, n_src=131, n_freq=5, beam=False, sky="disk")
    v, _ = _run(gpu_lib, ctx, p, eps=1e-6)
    assert oracle.rel_l2(v, oracle.direct_problem(p)) <= 1e-6


# ---------------------------------------------------------------- stages
@pytest.mark.parametrize("eps,dim,fold", [(1e-6, 2, True), (1e-10, 2, True), (1e-6, 3, True), (1e-6, 2, False),
                                          (1e-10, 3, False)])
def test_stage_parity_against_type3_steps(gpu_lib, ctx, eps, dim, fold):
    # fold=False: the paper's plain targets on both sides (no reflection into
    # a half-space), so the stages are checked without the fold
    p = synth.small_problem(37, n_ant=14, n_src=90, n_freq=2, three_d=(dim == 3), radius=70.0, zhalf=2.0)
    flags = (gpu_lib.DIM_3D if dim == 3 else gpu_lib.DIM_2D) | (0 if fold else gpu_lib.NO_FOLD)
    hp = gpu_lib.HostProblem.of(p, eps=eps, flags=flags)
    info, spread, fft = ctx.debug_stages(hp, f=1)
    pl = type3.make_plan(p.ant_enu, p.src_lmn, p.freq_hz, eps, dim, fold)
    # plan: integers bit-exact
    assert info["w"] == pl.w and info["fold_axis"] == pl.fold_axis
    assert info["n1"] == [int(v) for v in pl.n1[1]]
    assert info["n2"] == [int(v) for v in pl.n2(1)]
    assert np.allclose(info["s_c"], pl.s_c, rtol=0, atol=1e-15)
    assert np.allclose(info["B"], pl.B, rtol=1e-15, atol=1e-12)
    tol = 2e-6 if info["prec_bits"] == 32 else 1e-12
    # step 1 + first deconvolution
    bt = type3.spread(pl, 1, p.src_lmn, p.strengths()[1])
    assert spread.shape == bt.shape
    assert oracle.rel_l2(spread, bt) <= tol
    # step 2 on the pruned output window p in [-P, P]
    g = type3.fft_upsampled(pl, 1, bt)
    n2 = pl.n2(1)
    idx = [np.mod(np.arange(info["M"][a]) - info["P"][a], n2[a]) for a in range(dim)]
    ref = g[np.ix_(*[idx[a] for a in reversed(range(dim))])]
    assert fft.shape == ref.shape
    assert oracle.rel_l2(fft, ref) <= 4 * tol


# ---------------------------------------------------------------- direct kernel
@pytest.mark.parametrize("eps,tol", [(1e-6, 1e-6), (1e-10, 1e-12)])
def test_direct_kernel(gpu_lib, ctx, eps, tol):
    p = synth.small_problem(38, n_ant=21, n_src=1500, n_freq=2, three_d=True, radius=200.0)
    v, rep = _run(gpu_lib, ctx, p, eps=eps, flags=gpu_lib.METHOD_DIRECT)
    assert oracle.rel_l2(v, oracle.direct_problem(p)) <= tol


# ---------------------------------------------------------------- matrix-core direct sum
@pytest.mark.parametrize("three_d,eps,tol", [(False, 1e-6, 1e-6), (True, 1e-6, 1e-6), (False, 1e-10, 1e-12),
                                             (True, 1e-12, 1e-12)])
def test_zz_matrix_core_direct(gpu_lib, ctx, three_d, eps, tol):
    # 45 antennas: two 32-antenna tiles, the second ragged; 1501 sources: a
    # ragged last step of 4
    p = synth.small_problem(50, n_ant=45, n_src=1501, n_freq=2, three_d=three_d, radius=150.0)
    v, rep = _run(gpu_lib, ctx, p, eps=eps, flags=gpu_lib.METHOD_MFMA)
    assert rep["method"] == gpu_lib.METHOD_MFMA and rep["dim"] == (3 if three_d else 2)
    assert oracle.rel_l2(v, oracle.direct_problem(p)) <= tol


def test_zz_source_chunks_and_splits(gpu_lib):
    # a 2 MiB budget forces several source chunks per frequency (outputs added
    # chunk after chunk) and few splits
    p = synth.small_problem(51, n_ant=70, n_src=9000, n_freq=2, radius=150.0)
    with gpu_lib.Context(0, hbm_budget_bytes=2 << 20) as c:
        v, rep = _run(gpu_lib, c, p, eps=1e-6, flags=gpu_lib.METHOD_MFMA)
    assert oracle.rel_l2(v, oracle.direct_problem(p)) <= 1e-6


def test_zz_single_antenna_and_single_source(gpu_lib, ctx):
    p = synth.small_problem(52, n_ant=1, n_src=1, n_freq=1)
    v, _ = _run(gpu_lib, ctx, p, eps=1e-10, flags=gpu_lib.METHOD_MFMA)
    assert np.allclose(v[:, 0], p.strengths().sum(1), rtol=1e-12)
    p = synth.small_problem(53, n_ant=33, n_src=3, n_freq=1)
    v, _ = _run(gpu_lib, ctx, p, eps=1e-10, flags=gpu_lib.METHOD_MFMA)
    assert oracle.rel_l2(v, oracle.direct_problem(p)) <= 1e-12


def test_zz_agrees_with_vector_direct(gpu_lib, ctx):
    p = synth.small_problem(54, n_ant=64, n_src=4000, n_freq=1, hex_layout=True)
    v1, _ = _run(gpu_lib, ctx, p, eps=1e-6, flags=gpu_lib.METHOD_DIRECT)
    v2, _ = _run(gpu_lib, ctx, p, eps=1e-6, flags=gpu_lib.METHOD_MFMA)
    assert oracle.rel_l2(v2, v1) <= 2e-6


def test_device_entry_rejects_wrong_tensor_sizes(gpu_lib, ctx):
    # sizes are checked in the binding, before any device work: a beam that
    # is not [n_freq][n_src] (for example a 0-d array made from None) must
    # never reach the kernels
    import torch
    p = synth.small_problem(55, n_ant=6, n_src=50, n_freq=2)
    dev = torch.device("cuda:0")
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
    vis = torch.empty((p.n_freq, p.n_pairs, 2), dtype=torch.float64, device=dev)
    good = [d(p.ant_enu), d(p.src_lmn), d(p.freq_hz), d(p.flux), d(p.beam)]
    for k, bad in ((4, d(np.ascontiguousarray(None, dtype=np.float64))), (3, d(p.flux[:1])), (1, d(p.src_lmn[:-1])),
                   (0, d(p.ant_enu[:, :2]))):
        args = list(good)
        args[k] = bad
        with pytest.raises(ValueError):
            ctx.simulate_dev(*args, vis, eps=1e-6)
    ctx.simulate_dev(*good, vis, eps=1e-6)
    torch.cuda.synchronize()


# ---------------------------------------------------------------- edges
def test_empty_sky_gives_exact_zero(gpu_lib, ctx):
    p = synth.small_problem(39, n_ant=6, n_src=0, n_freq=2)
    v, _ = _run(gpu_lib, ctx, p)
    assert v.shape == (2, 21) and np.all(v == 0)


def test_single_antenna_autos(gpu_lib, ctx):
    p = synth.small_problem(40, n_ant=1, n_src=50, n_freq=2)
    v, _ = _run(gpu_lib, ctx, p, eps=1e-8)
    assert np.allclose(v[:, 0], p.strengths().sum(1), rtol=1e-8)


def test_single_source_zenith(gpu_lib, ctx):
    ant = synth.hex_array(19)
    src = np.array([[0.0, 0.0, 1.0]])
    V = gpu_lib.Context.simulate(ctx, ant, src, np.array([150e6]), np.array([[2.5]]), None, eps=1e-10)
    assert np.allclose(V, 2.5, rtol=1e-10)


def test_invalid_inputs_are_rejected(gpu_lib, ctx):
    p = synth.small_problem(41, n_ant=5, n_src=10, n_freq=1)
    bad = p.flux.copy()
    bad[0, 3] = np.nan
    with pytest.raises(gpu_lib.FvError) as e:
        ctx.simulate(p.ant_enu, p.src_lmn, p.freq_hz, bad, p.beam, eps=1e-6)
    assert e.value.status == gpu_lib.EINVAL
    src = p.src_lmn.copy()
    src[2] *= 1.01
    with pytest.raises(gpu_lib.FvError) as e:
        ctx.simulate(p.ant_enu, src, p.freq_hz, p.flux, p.beam, eps=1e-6)
    assert e.value.status == gpu_lib.EINVAL
    with pytest.raises(gpu_lib.FvError) as e:
        ctx.simulate(p.ant_enu, p.src_lmn, p.freq_hz, p.flux, p.beam, eps=1e-8, flags=gpu_lib.PREC_FP32)
    assert e.value.status == gpu_lib.EUNSUPPORTED
    with pytest.raises(gpu_lib.FvError) as e:
        ctx.simulate(p.ant_enu, p.src_lmn, p.freq_hz, p.flux, p.beam, eps=0.5)
    assert e.value.status == gpu_lib.EINVAL
    # the context is still usable
    v = ctx.simulate(p.ant_enu, p.src_lmn, p.freq_hz, p.flux, p.beam, eps=1e-6)
    assert oracle.rel_l2(v, oracle.direct_problem(p)) <= 1e-6


# ---------------------------------------------------------------- device API
def test_device_pointer_path_matches_host_path(gpu_lib, ctx):
    import torch
    p = synth.small_problem(42, n_ant=30, n_src=800, n_freq=3, hex_layout=True)
    host, _ = _run(gpu_lib, ctx, p, eps=1e-6)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    vis = torch.empty((p.n_freq, p.n_pairs, 2), dtype=torch.float64, device="cuda")
    ctx.simulate_dev(d(p.ant_enu), d(p.src_lmn), d(p.freq_hz), d(p.flux), d(p.beam), vis, eps=1e-6)
    torch.cuda.synchronize()
    v = vis.cpu().numpy()
    v = v[..., 0] + 1j * v[..., 1]
    assert oracle.rel_l2(v, oracle.direct_problem(p)) <= 1e-6
    assert oracle.rel_l2(v, host) <= 1e-6


def test_fp32_single_frequency(gpu_lib, ctx):
    p = synth.small_problem(31, n_ant=40, n_src=700, n_freq=1, hex_layout=True)
    v, rep = _run(gpu_lib, ctx, p, eps=1e-4, flags=gpu_lib.NO_LATTICE)
    assert oracle.rel_l2(v, oracle.direct_problem(p)) <= 1e-4


def test_fp64_multi_frequency(gpu_lib, ctx):
    p = synth.small_problem(31, n_ant=40, n_src=700, n_freq=3, hex_layout=True)
    v, rep = _run(gpu_lib, ctx, p, eps=1e-10, flags=gpu_lib.NO_LATTICE)
    errs = [oracle.rel_l2(v[f], oracle.direct_problem(p)[f]) for f in range(3)]
    assert max(errs) <= 1e-10, errs


@pytest.mark.parametrize("n_src", [10, 300, 3000])
def test_crowded_sources_keep_eps(gpu_lib, ctx, n_src):
    # every source inside one grid cell of a random array: the grids stay FP32
    # (batch sums in FP64) and keep the 1e-6 contract
    import dataclasses
    fv = gpu_lib
    p = synth.small_problem(170, n_ant=30, n_src=n_src, n_freq=2)
    src = np.tile(np.array([[0.001, 0.002, 0.0]]), (n_src, 1))
    src[:, 0] += np.linspace(0, 1e-4, n_src)
    src[:, 2] = np.sqrt(1 - src[:, 0] ** 2 - src[:, 1] ** 2)
    q = dataclasses.replace(p, src_lmn=src, beam=None)
    v, rep = _run(fv, ctx, q, eps=1e-6)
    assert rep["prec_bits"] == 32 and rep["lattice"] == 0
    assert oracle.rel_l2(v, oracle.direct_problem(q)) <= 1e-6


def _crowded(seed, n_in, n_out, three_d=False):
    # n_in sources inside one grid cell (0.1 mrad apart), n_out spread over
    # the disk, so that the source box is large and the mean density low
    import dataclasses
    p = synth.small_problem(seed, n_ant=30, n_src=n_in + n_out, n_freq=2, three_d=three_d, radius=60.0)
    rng = np.random.default_rng(seed)
    src = np.zeros((n_in + n_out, 3))
    src[:n_in, 0] = 0.001 + np.linspace(0, 1e-4, n_in)
    src[:n_in, 1] = 0.002
    r = np.sqrt(rng.uniform(0, 0.8, n_out))
    t = rng.uniform(0, 2 * np.pi, n_out)
    src[n_in:, 0], src[n_in:, 1] = r * np.cos(t), r * np.sin(t)
    src[:, 2] = np.sqrt(1 - src[:, 0] ** 2 - src[:, 1] ** 2)
    return dataclasses.replace(p, src_lmn=src, beam=None)


@pytest.mark.parametrize("n_in", [3000, 30000])
@pytest.mark.parametrize("three_d", [False, True])
def test_fp32_grids_keep_eps_with_a_crowded_cell(gpu_lib, ctx, n_in, three_d):
    # FP32 grids forced: the spread sums every batch of 64 records in FP32 and
    # the batches in FP64, so one cell crowded with thousands of records keeps
    # the 1e-6 contract
    fv = gpu_lib
    q = _crowded(172 + three_d, n_in, 0)
    v, rep = _run(fv, ctx, q, eps=1e-6, flags=fv.PREC_FP32 | fv.NO_LATTICE | (fv.DIM_3D if three_d else fv.DIM_2D))
    assert rep["prec_bits"] == 32 and rep["lattice"] == 0 and rep["dim"] == (3 if three_d else 2)
    assert oracle.rel_l2(v, oracle.direct_problem(q)) <= 1e-6


def test_dense_cell_plus_outliers_keeps_eps(gpu_lib, ctx):
    # a clustered sky: 3000 sources in one cell and 300 across the disk (a
    # large source box with one crowded cell); FP32 grids keep 1e-6
    fv = gpu_lib
    q = _crowded(174, 3000, 300)
    v, rep = _run(fv, ctx, q, eps=1e-6, flags=fv.NO_LATTICE)
    assert rep["prec_bits"] == 32 and rep["lattice"] == 0
    assert oracle.rel_l2(v, oracle.direct_problem(q)) <= 1e-6


def test_device_output_must_be_16_byte_aligned(gpu_lib, ctx):
    import torch
    fv = gpu_lib
    p = synth.small_problem(171, n_ant=7, n_src=20, n_freq=1)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")
    flat = torch.zeros(2 * p.n_pairs + 1, dtype=torch.float64, device="cuda:0")
    vis = flat[1:].view(1, p.n_pairs, 2)
    with pytest.raises(fv.FvError, match="EINVAL"):
        ctx.simulate_dev(d(p.ant_enu), d(p.src_lmn), d(p.freq_hz), d(p.flux), d(p.beam), vis, eps=1e-6)


def test_repeated_type3_after_other_paths_share_the_workspace(gpu_lib, ctx):
    """A type-3 launch whose tables match the last ones uploaded to its
    workspace skips the upload (and the modes' deconvolution tables).  Between
    two identical calls the workspace is used by the lattice path, the
    matrix-core direct sum, a smaller type-3 layout and a device batch, each of
    which overwrites its start; the next call must upload again and give the
    first call's result bit for bit (deterministic order)."""
    fl = gpu_lib.NO_LATTICE | gpu_lib.DETERMINISTIC
    p = synth.config1()
    v0, _ = _run(gpu_lib, ctx, p, eps=1e-6, flags=fl)
    v1, _ = _run(gpu_lib, ctx, p, eps=1e-6, flags=fl)  # tables unchanged: no upload
    assert np.array_equal(v0, v1)
    small = synth.small_problem(5, n_ant=9, n_src=30, n_freq=1)
    for other, ofl in ((p, 0), (p, gpu_lib.METHOD_MFMA), (small, fl)):
        _run(gpu_lib, ctx, other, eps=1e-6, flags=ofl)
        v2, _ = _run(gpu_lib, ctx, p, eps=1e-6, flags=fl)
        assert np.array_equal(v0, v2)
    # a device batch of type-3 problems (its own layouts in the same workspace)
    import torch
    d = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda:0").contiguous()
    items = []
    for q in (synth.small_problem(6, n_ant=12, n_src=50, n_freq=2), small):
        items.append(dict(ant_enu=d(q.ant_enu), src_lmn=d(q.src_lmn), freq_hz=d(q.freq_hz), flux=d(q.flux),
                          beam=d(q.beam) if q.beam is not None else None,
                          vis=torch.zeros(q.n_freq, q.n_pairs, 2, dtype=torch.float64, device="cuda:0"),
                          eps=1e-6, flags=fl))
    ctx.simulate_batch_dev(items)
    torch.cuda.synchronize()
    v3, _ = _run(gpu_lib, ctx, p, eps=1e-6, flags=fl)
    assert np.array_equal(v0, v3)
    assert oracle.rel_l2(v0, oracle.direct_problem(p)) < 1e-6
