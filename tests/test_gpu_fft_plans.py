"""The planned FFT passes (paper section 2.2, step 2) against the plain
definition: for every distinct grid of the 350-antenna workload's 64
frequencies (and a few 3-D and small grids), the pruned FFT output of the
device equals numpy's FFT of the zero-padded device spread grid, evaluated in
FP64 on the same input, to FP32 rounding.  The spread grid is the device's own,
so the comparison isolates the FFT passes."""
import os
import re

import numpy as np
import pytest

import oracle
import synth
from oracle import type3

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context(0)
    yield c
    c.close()


def _planned_sizes(kind):
    src = open(os.path.join(ROOT, "paper_2506_02130_amd", "csrc", f"fft_plans_{kind}.inc")).read()
    return {int(m) for m in re.findall(r"FV_FFT_PLAN\((\d+),", src)}


def _check(gpu_lib, ctx, p, f, eps, flags):
    hp = gpu_lib.HostProblem.of(p, eps=eps, flags=flags)
    info, spread, fft = ctx.debug_stages(hp, f=f)
    dim = info["dim"]
    pl = type3.make_plan(p.ant_enu, p.src_lmn, p.freq_hz, eps, dim)
    assert info["n1"] == [int(v) for v in pl.n1[f]]
    g = type3.fft_upsampled(pl, f, spread)
    n2 = pl.n2(f)
    idx = [np.mod(np.arange(info["M"][a]) - info["P"][a], n2[a]) for a in range(dim)]
    ref = g[np.ix_(*[idx[a] for a in reversed(range(dim))])]
    assert fft.shape == ref.shape
    return info, oracle.rel_l2(fft, ref)


def test_every_grid_of_the_hera350_workload(gpu_lib, ctx):
    p = synth.config2(n_src=2000)
    pl = type3.make_plan(p.ant_enu, p.src_lmn, p.freq_hz, p.eps, 2)
    rows, cols = _planned_sizes("rows"), _planned_sizes("cols")
    seen = {}
    for f in range(p.n_freq):
        key = tuple(int(v) for v in pl.n1[f])
        seen.setdefault(key, f)
    assert len(seen) >= 20
    worst = 0.0
    for key, f in sorted(seen.items()):
        assert key[0] in rows and key[1] in cols, key
        info, err = _check(gpu_lib, ctx, p, f, p.eps, gpu_lib.NO_LATTICE)
        assert info["prec_bits"] == 32
        print(f"n1={key} rel_l2={err:.2e}", flush=True)
        worst = max(worst, err)
        assert err <= 1e-6, (key, err)
    print(f"worst {worst:.2e} over {len(seen)} grids", flush=True)


@pytest.mark.parametrize("seed,n_ant,radius,three_d", [(51, 14, 70.0, True), (52, 30, 150.0, True),
                                                        (53, 9, 30.0, False), (54, 60, 400.0, False)])
def test_small_and_3d_grids(gpu_lib, ctx, seed, n_ant, radius, three_d):
    p = synth.small_problem(seed, n_ant=n_ant, n_src=300, n_freq=3, three_d=three_d, radius=radius, zhalf=3.0)
    for f in range(p.n_freq):
        info, err = _check(gpu_lib, ctx, p, f, 1e-6, gpu_lib.DIM_3D if three_d else gpu_lib.DIM_2D)
        print(f"n1={info['n1']} rel_l2={err:.2e}", flush=True)
        assert err <= 1e-6, (info["n1"], err)


@pytest.mark.parametrize("radius", [450.0, 600.0])
def test_rows_longer_than_2048(gpu_lib, ctx, radius):
    """Row plans go up to 4608 points (rows are contiguous, so a workgroup of
    one or two long rows still reads whole lines), column plans up to 2304
    (1728- and 2250-point columns here)."""
    p = synth.small_problem(55, n_ant=20, n_src=300, n_freq=1, three_d=False, radius=radius,
                            f_lo=150e6, f_hi=170e6)
    info, err = _check(gpu_lib, ctx, p, 0, 1e-6, gpu_lib.DIM_2D | gpu_lib.NO_LATTICE)
    print(f"n1={info['n1']} rel_l2={err:.2e}", flush=True)
    assert info["prec_bits"] == 32
    assert 2048 < info["n1"][0] <= 4608 and info["n1"][0] in _planned_sizes("rows")
    assert err <= 1e-6, (info["n1"], err)
