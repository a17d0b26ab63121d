"""GPU parity of the batched entry point (many snapshots, one launch per stage)."""
import dataclasses

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


def _dev(torch, p, flags=0, eps=None):
    d = "cuda:0"
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(d)
    return {"ant_enu": t(p.ant_enu), "src_lmn": t(p.src_lmn), "freq_hz": t(p.freq_hz), "flux": t(p.flux),
            "beam": None if p.beam is None else t(p.beam),
            "vis": torch.zeros((p.n_freq, p.n_pairs, 2), dtype=torch.float64, device=d),
            "eps": p.eps if eps is None else eps, "flags": flags}


def _cplx(v):
    a = v.cpu().numpy()
    return a[..., 0] + 1j * a[..., 1]


def test_lattice_batch_is_one_launch_per_stage(gpu_lib, ctx):
    # every snapshot of a 4-LST batch goes through the lattice path, and the
    # whole batch costs one launch per stage
    probs = synth.config4(n_lst=4, n_freq=5, n_cap=3000, n_iso=200)
    outs = ctx.simulate_batch([_hp(gpu_lib, p, flags=gpu_lib.TIMING) for p in probs])
    rep = ctx.last_report
    assert rep["lattice"] == 1
    assert rep["stage_launches"][gpu_lib.STAGES.index("spread")] == 1
    assert rep["stage_launches"][gpu_lib.STAGES.index("interp")] == 1
    for p, v in zip(probs, outs):
        assert oracle.rel_l2(v, oracle.direct_problem(p)) <= p.eps, p.name


def test_device_batch_matches_oracle_and_host_batch(gpu_lib, ctx):
    import torch
    probs = synth.config4(n_lst=3, n_freq=4, n_cap=2500, n_iso=150)
    mixed = probs + [synth.small_problem(70, n_ant=17, n_src=350, n_freq=2, three_d=True, radius=90.0),
                     synth.small_problem(71, n_ant=9, n_src=0, n_freq=2)]
    host = ctx.simulate_batch([_hp(gpu_lib, p) for p in mixed])
    items = [_dev(torch, p) for p in mixed]
    rep = ctx.simulate_batch_dev(items)
    torch.cuda.synchronize()
    assert rep["src_pairs"] == sum(p.n_src * p.n_pairs * p.n_freq for p in mixed)
    for p, it, h in zip(mixed, items, host):
        v = _cplx(it["vis"])
        if p.n_src == 0:
            assert np.all(v == 0)
            continue
        assert oracle.rel_l2(v, oracle.direct_problem(p)) <= p.eps
        assert oracle.rel_l2(v, h) <= p.eps / 4


def test_captured_lattice_batch_replays(gpu_lib, ctx):
    # FV_GRAPH: the batch's launch sequence is captured on the first call and
    # replayed on later calls with new fluxes (same shapes); every replay, with
    # eager work and host waits between them, equals the eager result
    import torch
    probs = synth.config4(n_lst=3, n_freq=4, n_cap=2000, n_iso=100)
    rng = np.random.default_rng(7)
    stream = torch.cuda.Stream()
    items = [_dev(torch, p, flags=gpu_lib.GRAPH) for p in probs]
    eager = [_dev(torch, p) for p in probs]
    for rep_i in range(4):
        scale = rng.uniform(0.5, 2.0, size=len(probs))
        for k, p in enumerate(probs):
            for d in (items[k], eager[k]):
                d["flux"].copy_(torch.from_numpy(p.flux * scale[k]).to(d["flux"].device))
        with torch.cuda.stream(stream):
            ctx.simulate_batch_dev(eager, stream=stream)
        stream.synchronize()
        ref = [_cplx(d["vis"]) for d in eager]
        with torch.cuda.stream(stream):
            ctx.simulate_batch_dev(items, stream=stream)
        stream.synchronize()
        for k, p in enumerate(probs):
            got = _cplx(items[k]["vis"])
            assert np.array_equal(got, ref[k]), (rep_i, k)
            if rep_i == 3:
                q = dataclasses.replace(p, flux=p.flux * scale[k])
                assert oracle.rel_l2(got, oracle.direct_problem(q)) <= p.eps


def test_device_batch_rejects_bad_values(gpu_lib, ctx):
    import torch
    good = synth.small_problem(72, n_ant=7, n_src=30, n_freq=1, hex_layout=True)
    items = [_dev(torch, good), _dev(torch, good)]
    items[1]["flux"][0, 0] = float("nan")
    with pytest.raises(gpu_lib.FvError) as ei:
        ctx.simulate_batch_dev(items)
    assert ei.value.status == -1
    torch.cuda.synchronize()


def test_repeated_device_batch_follows_changed_contents(gpu_lib, ctx):
    # a repeated batch (same pointers and sizes) is first enqueued on the last
    # batch's plan; when the arrays' contents change (antenna positions of a
    # lattice problem, source directions of a type-3 problem) the result must
    # still be that of the new contents
    import torch
    lat = synth.small_problem(73, n_ant=19, n_src=400, n_freq=3, hex_layout=True)
    t3 = synth.small_problem(74, n_ant=15, n_src=300, n_freq=2, three_d=True, radius=80.0)
    items = [_dev(torch, lat), _dev(torch, t3)]
    for q, it in zip((lat, t3), items):
        ctx.simulate_batch_dev(items)
        torch.cuda.synchronize()
        assert oracle.rel_l2(_cplx(it["vis"]), oracle.direct_problem(q)) <= q.eps
    # same contents again: the speculative plan holds
    ctx.simulate_batch_dev(items)
    torch.cuda.synchronize()
    for q, it in zip((lat, t3), items):
        assert oracle.rel_l2(_cplx(it["vis"]), oracle.direct_problem(q)) <= q.eps
    # new contents behind the same pointers
    lat2 = dataclasses.replace(lat, ant_enu=lat.ant_enu * 1.5)
    lmn = t3.src_lmn.copy()
    lmn[:, :2] *= 0.5
    lmn[:, 2] = np.sqrt(1.0 - (lmn[:, :2] ** 2).sum(1))
    t3b = dataclasses.replace(t3, src_lmn=lmn)
    items[0]["ant_enu"].copy_(torch.from_numpy(lat2.ant_enu))
    items[1]["src_lmn"].copy_(torch.from_numpy(lmn))
    ctx.simulate_batch_dev(items)
    torch.cuda.synchronize()
    for q, it in zip((lat2, t3b), items):
        assert oracle.rel_l2(_cplx(it["vis"]), oracle.direct_problem(q)) <= q.eps


def test_repeated_device_batch_still_reports_bad_values(gpu_lib, ctx):
    # the strength check runs beside a repeated batch's transforms; a NaN
    # planted between two identical calls is still reported, and the next good
    # call is correct
    import torch
    p = synth.small_problem(76, n_ant=19, n_src=500, n_freq=2, hex_layout=True)
    items = [_dev(torch, p)]
    ctx.simulate_batch_dev(items)
    torch.cuda.synchronize()
    keep = items[0]["flux"][1, 7].item()
    items[0]["flux"][1, 7] = float("inf")
    with pytest.raises(gpu_lib.FvError) as ei:
        ctx.simulate_batch_dev(items)
    assert ei.value.status == -1
    torch.cuda.synchronize()
    items[0]["flux"][1, 7] = keep
    ctx.simulate_batch_dev(items)
    torch.cuda.synchronize()
    assert oracle.rel_l2(_cplx(items[0]["vis"]), oracle.direct_problem(p)) <= p.eps


def test_device_batch_mixed_methods_and_graph(gpu_lib, ctx):
    # one device batch with every method and path: lattice and type-3 NUFFT,
    # the vector direct sum and the matrix-core direct sum, FP64 and FP32, an
    # empty sky; the lattice group captured (FV_GRAPH) and replayed
    import torch
    fv = gpu_lib
    cases = [
        (synth.small_problem(77, n_ant=19, n_src=600, n_freq=3, hex_layout=True), 1e-6, fv.GRAPH),
        (synth.small_problem(78, n_ant=19, n_src=400, n_freq=2, hex_layout=True), 1e-10, fv.GRAPH),
        (synth.small_problem(79, n_ant=16, n_src=300, n_freq=2, three_d=True, radius=90.0), 1e-6, 0),
        (synth.small_problem(80, n_ant=13, n_src=250, n_freq=2), 1e-6, fv.METHOD_DIRECT),
        (synth.small_problem(81, n_ant=21, n_src=350, n_freq=2), 1e-6, fv.METHOD_MFMA),
        (synth.small_problem(82, n_ant=9, n_src=0, n_freq=2), 1e-6, 0),
    ]
    items = [_dev(torch, p, flags=f, eps=e) for p, e, f in cases]
    batch = ctx.prepare_batch_dev(items)
    for rep_i in range(3):
        for it in items:
            it["vis"].zero_()
        ctx.run_batch_dev(batch)
        torch.cuda.synchronize()
        for (p, e, f), it in zip(cases, items):
            v = _cplx(it["vis"])
            if p.n_src == 0:
                assert np.all(v == 0)
                continue
            tol = e if (f & 0x30) == 0 else max(e, 1e-6)  # the direct sums: FP32 at eps 1e-6
            assert oracle.rel_l2(v, oracle.direct_problem(p)) <= tol, (rep_i, p.name)
