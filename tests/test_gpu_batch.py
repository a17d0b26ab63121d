"""GPU parity of the batched entry point (many snapshots, one launch per stage)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context(0)
    yield c
    c.close()


def _hp(fv, p, eps=None, flags=0):
    return fv.HostProblem.of(p, eps=eps, flags=flags)


def test_mixed_batch_matches_single_calls_and_oracle(gpu_lib, ctx):
    fv = gpu_lib
    probs = [
        (synth.small_problem(60, n_ant=20, n_src=400, n_freq=3, hex_layout=True), 1e-6, 0),
        (synth.small_problem(61, n_ant=17, n_src=350, n_freq=2, three_d=True, radius=90.0), 1e-6, 0),
        (synth.small_problem(62, n_ant=12, n_src=300, n_freq=2), 1e-10, 0),
        (synth.small_problem(63, n_ant=9, n_src=0, n_freq=2), 1e-6, 0),
        (synth.small_problem(64, n_ant=11, n_src=200, n_freq=1), 1e-6, fv.METHOD_DIRECT),
        (synth.small_problem(65, n_ant=40, n_src=500, n_freq=4, hex_layout=True), 1e-6, 0),
    ]
    hps = [_hp(fv, p, e, f) for p, e, f in probs]
    outs = ctx.simulate_batch(hps)
    rep = ctx.last_report
    assert rep["src_pairs"] == sum(p.n_src * p.n_pairs * p.n_freq for p, _, _ in probs)
    for (p, e, f), hp, v in zip(probs, hps, outs):
        assert v.shape == (p.n_freq, p.n_pairs)
        if p.n_src == 0:
            assert np.all(v == 0)
            continue
        ref = oracle.direct_problem(p)
        assert oracle.rel_l2(v, ref) <= e
        single = ctx.simulate_problem(hp)
        # same kernels; only the order of FP32 additions inside a sub-bin may differ
        assert oracle.rel_l2(v, single) <= max(e / 4, 1e-13)


def test_config4_like_batch_every_snapshot(gpu_lib, ctx):
    # 4 LSTs x 5 frequencies of the 127-antenna hex with a 25-degree cap sky,
    # reduced in source count; per-LST source counts differ (horizon cut)
    probs = synth.config4(n_lst=4, n_freq=5, n_cap=3000, n_iso=200)
    counts = [p.n_src for p in probs]
    assert len(set(counts)) > 1
    outs = ctx.simulate_batch([_hp(gpu_lib, p) for p in probs])
    for p, v in zip(probs, outs):
        ref = oracle.direct_problem(p)
        assert oracle.rel_l2(v, ref) <= p.eps, p.name


def test_empty_batch_is_ok(gpu_lib, ctx):
    assert ctx.simulate_batch([]) == []


def test_batch_rejects_a_bad_member(gpu_lib, ctx):
    good = synth.small_problem(66, n_ant=5, n_src=20, n_freq=1)
    bad = synth.small_problem(67, n_ant=5, n_src=20, n_freq=1)
    flux = bad.flux.copy()
    flux[0, 0] = np.inf
    hb = gpu_lib.HostProblem(bad.ant_enu, bad.src_lmn, bad.freq_hz, flux, bad.beam, 1e-6)
    with pytest.raises(gpu_lib.FvError) as ei:
        ctx.simulate_batch([_hp(gpu_lib, good), hb])
    assert ei.value.status == -1
