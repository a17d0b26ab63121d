"""Full-size workloads (the benchmark configurations) checked against the FP64
oracle on seeded samples of their outputs: every frequency of a few sampled
pairs would be the whole output; the oracle evaluates the sampled
(frequency, pair) entries one by one."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _sample_check(v, p, n_pairs=256, n_freq=2, seed=11):
    sub = synth.subset_pairs(p.n_ant, n_pairs, seed)
    fsel = np.unique(np.linspace(0, p.n_freq - 1, n_freq).round().astype(int))
    ref = oracle.direct_vis(p.ant_enu, p.src_lmn, p.freq_hz[fsel], p.flux[fsel],
                            None if p.beam is None else p.beam[fsel], pairs=sub)
    got = v[fsel][:, sub]
    return oracle.rel_l2(got, ref)


def test_hera350_full_size_device_path(gpu_lib):
    """350-antenna hex, 1e5 sources, 64 frequencies, eps 1e-6: the benchmark's
    workload through fv_simulate_dev on a torch stream, as bench.py runs it."""
    import torch
    fv = gpu_lib
    p = synth.config2()
    dev = torch.device("cuda:0")
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
    vis = torch.empty((p.n_freq, p.n_pairs, 2), dtype=torch.float64, device=dev)
    stream = torch.cuda.Stream(device=dev)
    with fv.Context(0) as c:
        rep = c.simulate_dev(d(p.ant_enu), d(p.src_lmn), d(p.freq_hz), d(p.flux), d(p.beam), vis, eps=p.eps,
                             flags=fv.TIMING, stream=stream)
        torch.cuda.synchronize()
    assert rep["dim"] == 2 and rep["prec_bits"] == 32
    o = vis.cpu().numpy()
    v = o[..., 0] + 1j * o[..., 1]
    assert _sample_check(v, p, n_pairs=512, n_freq=4) <= p.eps


def test_disk1000_3d_full_size(gpu_lib):
    """1000 antennas in a 500 m disk with +-5 m heights (3-D), 393k horizon-cut
    equal-area pixels, 16 frequencies 150-170 MHz, eps 1e-6."""
    fv = gpu_lib
    p = synth.config3()
    with fv.Context(0) as c:
        v = c.simulate_problem(fv.HostProblem.of(p))
        rep = c.last_report
    assert rep["dim"] == 3 and rep["prec_bits"] == 32
    assert rep["n1"][2] >= 16
    assert _sample_check(v, p) <= p.eps


def test_batched_1032_snapshots_full_size(gpu_lib):
    """127-antenna hex, 24 LSTs x 43 frequencies, 973-101k sources per LST,
    one batch call; sampled pairs of a few LSTs checked."""
    fv = gpu_lib
    probs = synth.config4()
    with fv.Context(0) as c:
        outs = c.simulate_batch([fv.HostProblem.of(q) for q in probs])
    for k in (0, 7, 13, 23):
        assert _sample_check(outs[k], probs[k], n_pairs=256, n_freq=3, seed=20 + k) <= probs[k].eps, probs[k].name


def test_successive_device_calls_on_different_streams_are_ordered(gpu_lib):
    """A large call on one stream, then a small one on another stream and a
    host-buffer call, with no synchronisation between them: the later calls
    reuse the context's workspace and must wait for the first one."""
    import torch
    fv = gpu_lib
    dev = torch.device("cuda:0")
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
    big = synth.config2(n_src=30000, n_freq=16)
    small = synth.small_problem(140, n_ant=37, n_src=500, n_freq=2, hex_layout=True)
    other = synth.small_problem(141, n_ant=20, n_src=300, n_freq=2)
    args_b = [d(x) for x in (big.ant_enu, big.src_lmn, big.freq_hz, big.flux, big.beam)]
    args_s = [d(x) for x in (small.ant_enu, small.src_lmn, small.freq_hz, small.flux, small.beam)]
    vis_b = torch.empty((big.n_freq, big.n_pairs, 2), dtype=torch.float64, device=dev)
    vis_s = torch.empty((small.n_freq, small.n_pairs, 2), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(device=dev), torch.cuda.Stream(device=dev)
    with fv.Context(0) as c:
        for _ in range(2):
            c.simulate_dev(*args_b, vis_b, eps=big.eps, stream=s1)
            c.simulate_dev(*args_s, vis_s, eps=small.eps, stream=s2)
            v_o = c.simulate_problem(fv.HostProblem.of(other))
            torch.cuda.synchronize()
            o = vis_b.cpu().numpy()
            assert _sample_check(o[..., 0] + 1j * o[..., 1], big, n_pairs=128, n_freq=2) <= big.eps
            o = vis_s.cpu().numpy()
            assert oracle.rel_l2(o[..., 0] + 1j * o[..., 1], oracle.direct_problem(small)) <= small.eps
            assert oracle.rel_l2(v_o, oracle.direct_problem(other)) <= other.eps
