"""The allocation-free entry point (fv_simulate_mfma_noalloc) against the
context's device entry point with FV_METHOD_MFMA (the same matrix-core direct
form, paper section 5.1) and against the exact sum: two calls in a row, the
second with a smaller input, then an empty sky and the host-side limits."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _dev(p):
    import torch
    dev = torch.device("cuda:0")
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
    return [d(p.ant_enu), d(p.src_lmn), d(p.freq_hz), d(p.flux), None if p.beam is None else d(p.beam)]


def _c(t):
    o = t.cpu().numpy()
    return o[..., 0] + 1j * o[..., 1]


def test_noalloc_matches_device_entry_point_twice(gpu_lib):
    import torch
    fv = gpu_lib
    # first call: enough sources that Z is built in several chunks of the
    # static array; second call: a smaller problem reusing the same array
    big = synth.small_problem(190, n_ant=127, n_src=150000, n_freq=2, hex_layout=True)
    small = synth.small_problem(191, n_ant=37, n_src=2000, n_freq=3, hex_layout=True)
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream(device=torch.device("cuda:0"))
    with fv.Context(0) as c:
        for p in (big, small):
            args = _dev(p)
            v_na = torch.full((p.n_freq, p.n_pairs, 2), float("nan"), dtype=torch.float64, device="cuda:0")
            v_ref = torch.empty_like(v_na)
            torch.cuda.synchronize()  # the fill above ran on torch's default stream
            print(f"noalloc: {p.name} n_ant={p.n_ant} n_src={p.n_src} n_freq={p.n_freq}", flush=True)
            fv.simulate_mfma_noalloc(*args, v_na, eps=p.eps, stream=stream)
            c.simulate_dev(*args, v_ref, eps=p.eps, flags=fv.METHOD_MFMA, stream=stream)
            torch.cuda.synchronize()
            a, b = _c(v_na), _c(v_ref)
            assert np.all(np.isfinite(a))
            assert oracle.rel_l2(a, b) <= p.eps / 10, p.name
            sub = synth.subset_pairs(p.n_ant, 256, 7)
            ref = oracle.direct_vis(p.ant_enu, p.src_lmn, p.freq_hz, p.flux, p.beam, pairs=sub)
            assert oracle.rel_l2(a[:, sub], ref) <= p.eps, p.name


def test_noalloc_empty_sky_and_limits(gpu_lib):
    import torch
    fv = gpu_lib
    p = synth.small_problem(192, n_ant=9, n_src=0, n_freq=2)
    args = _dev(p)
    v = torch.full((p.n_freq, p.n_pairs, 2), 7.0, dtype=torch.float64, device="cuda:0")
    fv.simulate_mfma_noalloc(*args, v, eps=1e-6)
    torch.cuda.synchronize()
    assert torch.all(v == 0)
    # host-side refusals, before any device work: another method, too many antennas
    q = synth.small_problem(193, n_ant=12, n_src=50, n_freq=1)
    args = _dev(q)
    v = torch.empty((q.n_freq, q.n_pairs, 2), dtype=torch.float64, device="cuda:0")
    with pytest.raises(fv.FvError):
        fv._lib.fv_simulate_mfma_noalloc  # exported
        c = fv.Problem(q.n_ant, args[0].data_ptr(), q.n_src, args[1].data_ptr(), q.n_freq, args[2].data_ptr(),
                       args[3].data_ptr(), args[4].data_ptr(), 1e-6, fv.METHOD_DIRECT)
        fv._check(fv._lib.fv_simulate_mfma_noalloc(fv.ctypes.byref(c), v.data_ptr(), None))
    big_ant = torch.zeros((1025, 3), dtype=torch.float64, device="cuda:0")
    v2 = torch.empty((1, 1025 * 1026 // 2, 2), dtype=torch.float64, device="cuda:0")
    with pytest.raises(fv.FvError):
        fv.simulate_mfma_noalloc(big_ant, args[1], args[2][:1].contiguous(), args[3][:1].contiguous(),
                                 args[4][:1].contiguous(), v2, eps=1e-6)
