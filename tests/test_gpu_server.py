"""Serving loop: admission by HBM footprint, concurrent slots, tickets."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _out(p):
    return np.empty((p.n_freq, p.n_pairs, 2), dtype=np.float64)


def _c(o):
    return o[..., 0] + 1j * o[..., 1]


def _mix():
    return [
        (synth.small_problem(80, n_ant=30, n_src=2000, n_freq=4, hex_layout=True), 1e-6, 0),
        (synth.small_problem(81, n_ant=18, n_src=700, n_freq=2, three_d=True, radius=100.0), 1e-6, 0),
        (synth.small_problem(82, n_ant=15, n_src=500, n_freq=3), 1e-10, 0),
        (synth.small_problem(83, n_ant=25, n_src=900, n_freq=1), 1e-6, 0x20),  # matrix-core direct
        (synth.small_problem(84, n_ant=9, n_src=0, n_freq=2), 1e-6, 0),
        (synth.small_problem(85, n_ant=44, n_src=3000, n_freq=5, hex_layout=True), 1e-6, 0),
        (synth.small_problem(86, n_ant=12, n_src=400, n_freq=2), 1e-4, 0),
        (synth.small_problem(87, n_ant=20, n_src=1200, n_freq=2, three_d=True, radius=80.0), 1e-8, 0),
    ]


def test_mixed_requests_match_solo_runs_and_oracle(gpu_lib):
    fv = gpu_lib
    probs = _mix()
    with fv.Context(0) as c:
        hps = [fv.HostProblem.of(p, eps=e, flags=f) for p, e, f in probs]
        solo = [c.simulate_problem(h) for h in hps]
        c.server_start(3)
        outs = [_out(p) for p, _, _ in probs]
        tickets = [c.submit(h, o) for h, o in zip(hps, outs)]
        for (p, e, f), t, o, s in zip(probs, tickets, outs, solo):
            st, rep = c.wait(t)
            assert st == 0, (p.name, st)
            assert rep["t_total_ms"] > 0
            v = _c(o)
            if p.n_src == 0:
                assert np.all(v == 0)
                continue
            assert oracle.rel_l2(v, oracle.direct_problem(p)) <= e, p.name
            assert oracle.rel_l2(v, s) <= max(e / 10, 1e-13), p.name
        c.server_stop()


def test_deterministic_mix_is_bitwise_equal_to_solo(gpu_lib):
    """With FV_DETERMINISTIC every request of the mix (type-3 forced where the
    array is a lattice) gives the same bits in the serving mix as alone."""
    fv = gpu_lib
    probs = [(p, e, f | fv.DETERMINISTIC | (fv.NO_LATTICE if i % 2 == 0 else 0))
             for i, (p, e, f) in enumerate(_mix())]
    with fv.Context(0) as c:
        hps = [fv.HostProblem.of(p, eps=e, flags=f) for p, e, f in probs]
        solo = [c.simulate_problem(h) for h in hps]
        c.server_start(3)
        outs = [_out(p) for p, _, _ in probs]
        tickets = [c.submit(h, o) for h, o in zip(hps, outs)]
        for (p, e, f), t, o, s in zip(probs, tickets, outs, solo):
            st, _ = c.wait(t)
            assert st == 0, (p.name, st)
            assert np.array_equal(_c(o), s), p.name
            if p.n_src:
                assert oracle.rel_l2(s, oracle.direct_problem(p)) <= e, p.name
        c.server_stop()


def test_budget_admission_and_oversize_rejection(gpu_lib):
    fv = gpu_lib
    small = [synth.small_problem(90 + k, n_ant=20, n_src=800, n_freq=2, hex_layout=True) for k in range(5)]
    big = synth.config2(n_src=2000, n_freq=8)
    with fv.Context(0, hbm_budget_bytes=48 << 20) as c:
        c.server_start(4)
        outs = [_out(p) for p in small]
        ts = [c.submit(fv.HostProblem.of(p), o) for p, o in zip(small, outs)]
        ob = _out(big)
        tb = c.submit(fv.HostProblem.of(big), ob)
        for p, t, o in zip(small, ts, outs):
            st, _ = c.wait(t)
            assert st == 0
            assert oracle.rel_l2(_c(o), oracle.direct_problem(p)) <= p.eps
        st, _ = c.wait(tb)
        assert st == fv.ENOMEM
        c.server_stop()


def test_stop_cancels_queued_and_finishes_running(gpu_lib):
    fv = gpu_lib
    first = synth.config2(n_src=20000, n_freq=16)
    rest = [synth.small_problem(100 + k, n_ant=10, n_src=200, n_freq=1) for k in range(6)]
    with fv.Context(0) as c:
        c.server_start(1)
        of = _out(first)
        tf = c.submit(fv.HostProblem.of(first), of)
        outs = [_out(p) for p in rest]
        ts = [c.submit(fv.HostProblem.of(p), o) for p, o in zip(rest, outs)]
        c.server_stop()
        st, _ = c.wait(tf)
        assert st in (0, fv.ECANCELLED)
        codes = [c.wait(t)[0] for t in ts]
        assert all(s in (0, fv.ECANCELLED) for s in codes)
        assert fv.ECANCELLED in codes + [st]
        for p, o, s in zip(rest, outs, codes):
            if s == 0:
                assert oracle.rel_l2(_c(o), oracle.direct_problem(p)) <= p.eps
        with pytest.raises(fv.FvError) as ei:
            c.submit(fv.HostProblem.of(rest[0]), outs[0])
        assert ei.value.status == fv.EBUSY


def test_wait_timeout_then_completion_and_bad_submit(gpu_lib):
    fv = gpu_lib
    p = synth.config2(n_src=30000, n_freq=16)
    with fv.Context(0) as c:
        c.server_start(2)
        o = _out(p)
        t = c.submit(fv.HostProblem.of(p), o)
        st, _ = c.wait(t, timeout_s=0.0)
        assert st in (fv.ETIMEOUT, 0)
        if st == fv.ETIMEOUT:
            st, _ = c.wait(t)
        assert st == 0
        sub = synth.subset_pairs(p.n_ant, 256, 3)
        fsel = np.array([0, p.n_freq - 1])
        ref = oracle.direct_vis(p.ant_enu, p.src_lmn, p.freq_hz[fsel], p.flux[fsel], p.beam[fsel], pairs=sub)
        got = _c(o)[fsel][:, sub]
        assert oracle.rel_l2(got, ref) <= p.eps
        bad = synth.small_problem(110, n_ant=5, n_src=10, n_freq=1)
        with pytest.raises(fv.FvError) as ei:
            c.submit(fv.HostProblem(bad.ant_enu, bad.src_lmn, bad.freq_hz, bad.flux, bad.beam, 0.5), _out(bad))
        assert ei.value.status == fv.EINVAL
        assert c.wait(123456789)[0] == fv.EINVAL
        c.server_stop()


def test_device_requests_mixed_with_host_requests(gpu_lib):
    """Requests with device-resident inputs (fv_submit_dev) run in the same
    serving mix as host requests; each result matches the oracle and its solo
    device run, and a bad device request fails alone."""
    import torch
    fv = gpu_lib
    probs = _mix()
    dev = "cuda:0"
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)

    def dev_args(p):
        return (t(p.ant_enu), t(p.src_lmn).reshape(-1, 3), t(p.freq_hz), t(p.flux.reshape(p.n_freq, p.n_src)),
                None if p.beam is None else t(p.beam))

    with fv.Context(0) as c:
        args = [dev_args(p) for p, _, _ in probs]
        vis = [torch.zeros((p.n_freq, p.n_pairs, 2), dtype=torch.float64, device=dev) for p, _, _ in probs]
        solo = []
        for (p, e, f), a in zip(probs, args):
            v = torch.zeros((p.n_freq, p.n_pairs, 2), dtype=torch.float64, device=dev)
            c.simulate_dev(*a, v, eps=e, flags=f)
            torch.cuda.synchronize()
            solo.append(v.cpu().numpy())
        hps = [fv.HostProblem.of(p, eps=e, flags=f) for p, e, f in probs]
        houts = [_out(p) for p, _, _ in probs]
        c.server_start(3)
        tickets = []
        for i, ((p, e, f), a, v) in enumerate(zip(probs, args, vis)):
            tickets.append(c.submit_dev(*a, v, eps=e, flags=f))
            if i % 2 == 0:
                tickets.append(c.submit(hps[i], houts[i]))
        # a device request with a NaN flux fails on its own
        bad = dev_args(probs[0][0])
        bad[3][0, 0] = float("nan")
        bv = torch.zeros_like(vis[0])
        tb = c.submit_dev(*bad, bv, eps=1e-6)
        for tk in tickets:
            st, rep = c.wait(tk)
            assert st == 0
        st, _ = c.wait(tb)
        assert st == -1
        torch.cuda.synchronize()
        for (p, e, f), v, s in zip(probs, vis, solo):
            got = v.cpu().numpy()
            if p.n_src == 0:
                assert np.all(got == 0)
                continue
            assert oracle.rel_l2(_c(got), oracle.direct_problem(p)) <= e, p.name
            assert oracle.rel_l2(_c(got), _c(s)) <= max(e / 10, 1e-13), p.name
        for i, (p, e, f) in enumerate(probs):
            if i % 2 == 0 and p.n_src:
                assert oracle.rel_l2(_c(houts[i]), oracle.direct_problem(p)) <= e, p.name
        c.server_stop()
