"""Benchmark: source x baseline pairs per second of the type-3 NUFFT visibility
simulator on one MI355X, on the HERA-350 workload (350-antenna hexagonal array,
1e5 power-law point sources, Gaussian beam, 64 frequencies in 100-200 MHz,
eps = 1e-6, FP32 grids), inputs resident in HBM.

One step = one call of the whole pipeline (tables, sort, spread, FFT passes,
interpolation) over all 64 frequencies through the C ABI (fv_simulate_dev).

Prints one JSON line with the throughput, the roofline of the dominant kernel
(algorithmic bytes / HIP-event time of that kernel), the direct-sum kernels'
rates on the same workload, the per-step latency percentiles, a parity check
against the FP64 oracle on a seeded subset, and the oracle's own CPU rate.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
LDS_PEAK_GBS = 256 * 128 * 2.4  # MI355X LDS: 256 CUs x 128 bytes per clock x 2.4 GHz
FP32_VALU_PEAK_TFLOPS = 157.3  # MI355X vector FP32 (packed)
FP32_MATRIX_PEAK_TFLOPS = 157.3  # MI355X dense FP32 matrix cores
METRIC = "src×baseline pairs/s at 1e-6 rel err, NUFFT vs direct DFT; p99 latency"
KERNEL_OF_STAGE = {"spread": "k_spread_mfma", "fft_x": "k_fft_rows", "fft_y": "k_fft_cols", "fft_z": "k_fft_cols",
                   "interp": "k_interp",
                   "sort": "k_bin/k_scan/k_scatter", "direct": "k_direct", "other": "k_ipsi"}
KERNEL_OF_STAGE_T1 = {"spread": "k_t1_spread", "fft_x": "k_t1_rows", "fft_y": "k_t1_cols", "interp": "k_t1_out"}


def _pct(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q
    lo, hi = math.floor(k), math.ceil(k)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


# device sources of the kernels of each path (the byte counters of a path stay
# valid while these files are unchanged)
PATH_SOURCES = {"type1": ["lattice.hip", "dev_common.h"],
                "type3": ["nufft_impl.h", "nufft.hip", "nufft_f32_2d.hip", "nufft_f32_3d.hip", "nufft_f64_2d.hip",
                          "nufft_f64_3d.hip", "dev_common.h", "fft_reg.h", "fft_reg.hip", "fft_reg_cols.hip",
                          "fft_plans_rows.inc", "fft_plans_cols.inc", "nufft_layout.h"]}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _kernel_source_hash(files=None) -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2506_02130_amd", "csrc")
    names = files if files is not None else sorted(fn for fn in os.listdir(csrc) if fn.endswith((".hip", ".h", ".cpp")))
    for fn in names:
        h.update(fn.encode())
        h.update(open(os.path.join(csrc, fn), "rb").read())
    return h.hexdigest()[:16]


def _traffic_from_profiles(stage: str, path_name: str):
    """HBM bytes per launch of a stage, from a committed pair of rocprofv3
    --pmc runs (FETCH_SIZE, WRITE_SIZE) scaled by the calibration copy
    (profiles/traffic_c2_<path>.json), only while the device sources of the
    path they were taken on are unchanged."""
    path = os.path.join(ROOT, "profiles", f"traffic_c2_{path_name}.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    files = d.get("sources")
    if d.get("path") != path_name or not files or d.get("source_hash") != _kernel_source_hash(files):
        return None
    k = d.get("stages", {}).get(stage)
    return None if k is None else k.get("bytes_per_launch")


# pipeline stage of each kernel (the FFT kernel of the type-3 path takes
# fft_x, fft_y, fft_z in launch order)
STAGE_OF_KERNEL = {"k_order_count": "sort", "k_order_scan": "sort", "k_order_place": "sort", "k_bin": "sort",
                   "k_scan": "sort", "k_scatter": "sort", "k_fill_int": "sort", "k_spread_mfma": "spread",
                   "k_spread": "spread", "k_interp": "interp", "k_ipsi": "other", "k_t1_spread": "spread",
                   "k_t1_rows": "fft_x", "k_t1_cols": "fft_y", "k_t1_out": "interp", "k_validate": "other",
                   "k_validate_reduce": "other", "k_targets": "other"}


def reduce_traffic(fetch_csv: str, write_csv: str, calib_mib: int, cmd: str, workload: str):
    """HBM bytes per launch of each stage from two rocprofv3 --pmc runs of
    `bench.py --profile --calib-copy-mib M` (FETCH_SIZE, then WRITE_SIZE, in
    KiB per dispatch), each scaled by what the same counter reads for the M MiB
    device copy issued after the timed steps.  Rows are the dispatches of the
    last step (from its input-check kernel to the copy).  Writes
    profiles/traffic_c2_<path>.json (read back by the roofline, tagged with a
    hash of the path's device sources) and prints a markdown table."""
    import csv

    def load(path):
        rows = sorted(csv.DictReader(open(path)), key=lambda r: int(r["Dispatch_Id"]))
        out = []
        for r in rows:
            name = r["Kernel_Name"].replace("void ", "").replace("fv::(anonymous namespace)::", "").split("(")[0]
            out.append((name, float(r["Counter_Value"])))
        return out

    fetch, write = load(fetch_csv), load(write_csv)
    if [x[0] for x in fetch] != [x[0] for x in write]:
        raise SystemExit("the two counter runs dispatched different kernels")
    ci = max((i for i, x in enumerate(write) if "copyBuffer" in x[0]), key=lambda i: write[i][1])
    f_scale = calib_mib * 1024 / fetch[ci][1]
    w_scale = calib_mib * 1024 / write[ci][1]
    s0 = [i for i, x in enumerate(fetch) if x[0] == "k_validate" and i < ci][-1]
    stages, rows, nfft = {}, [], 0
    for i in range(s0, ci):
        name = fetch[i][0]
        base = name.split("<")[0]
        if base in ("k_fft", "k_fft_rows", "k_fft_cols"):
            st = ("fft_x", "fft_y", "fft_z")[min(nfft, 2)]  # the passes run in axis order
            nfft += 1
        else:
            st = STAGE_OF_KERNEL.get(base)
        fb, wb = fetch[i][1] * f_scale * 1024, write[i][1] * w_scale * 1024
        rows.append((name, st, fetch[i][1], write[i][1], fb, wb))
        if st is None or "copyBuffer" in name:
            continue
        e = stages.setdefault(st, {"fetch_bytes": 0.0, "write_bytes": 0.0, "launches": 0})
        e["fetch_bytes"] += fb
        e["write_bytes"] += wb
        e["launches"] += 1
    for e in stages.values():
        e["bytes_per_launch"] = (e["fetch_bytes"] + e["write_bytes"]) / e["launches"]
    path = "type1" if any(x[0].startswith("k_t1_") for x in fetch) else "type3"
    d = {"path": path, "sources": PATH_SOURCES[path], "source_hash": _kernel_source_hash(PATH_SOURCES[path]),
         "command": cmd, "workload": workload,
         "calibration": {"copy_MiB": calib_mib, "FETCH_SIZE_KiB": fetch[ci][1], "WRITE_SIZE_KiB": write[ci][1],
                         "fetch_scale": f_scale, "write_scale": w_scale},
         "stages": stages}
    json.dump(d, open(os.path.join(ROOT, "profiles", f"traffic_c2_{path}.json"), "w"), indent=1)
    print(f"Calibration: the {calib_mib} MiB device copy after the steps reads FETCH_SIZE {fetch[ci][1]:.1f} KiB "
          f"and WRITE_SIZE {write[ci][1]:.1f} KiB, so FETCH_SIZE is scaled by {f_scale:.3f} and WRITE_SIZE by "
          f"{w_scale:.3f}.  Rows are the dispatches of the last step.\n")
    print("| kernel | stage | FETCH_SIZE KiB | WRITE_SIZE KiB | read MB (scaled) | write MB (scaled) |")
    print("|---|---|---|---|---|---|")
    for name, st, fk, wk, fb, wb in rows:
        print(f"| `{name}` | {st or '-'} | {fk:.0f} | {wk:.0f} | {fb / 1e6:.2f} | {wb / 1e6:.2f} |")


def stats_md(path: str):
    """Markdown table (kernel, calls, average, total, share) of a rocprofv3
    --kernel-trace --stats kernel summary CSV."""
    import csv
    import re

    rows = list(csv.DictReader(open(path)))
    tot = sum(int(r["TotalDurationNs"]) for r in rows)
    print("| kernel | calls | avg us | total us | % |\n|---|---|---|---|---|")
    for r in sorted(rows, key=lambda r: -int(r["TotalDurationNs"])):
        name = re.sub(r"\(.*$", "", re.sub(r"fv::\(anonymous namespace\)::", "", re.sub(r"^void ", "", r["Name"])))
        print(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | {int(r['TotalDurationNs']) / 1e3:.1f} | "
              f"{100 * int(r['TotalDurationNs']) / tot:.1f} |")


def overlap_md(path: str) -> None:
    """Kernel concurrency across streams in a kernel trace: per stream, the
    union of its kernels' intervals; then the time during which 1, 2, ...
    streams have a kernel running.  The plain paths run on one stream; the
    server's slots each have their own."""
    import csv
    rows = list(csv.DictReader(open(path)))
    by = {}
    for r in rows:
        by.setdefault(r["Stream_Id"], []).append((int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
    ev = []
    for sid, iv in by.items():
        iv.sort()
        cs, ce = iv[0]
        for a, b in iv[1:]:
            if a > ce:
                ev += [(cs, 1), (ce, -1)]
                cs, ce = a, b
            else:
                ce = max(ce, b)
        ev += [(cs, 1), (ce, -1)]
    ev.sort()
    hist, cur, last = {}, 0, None
    for t, d in ev:
        if last is not None and cur > 0:
            hist[cur] = hist.get(cur, 0) + (t - last)
        cur += d
        last = t
    busy = sum(hist.values())
    print(f"Kernel trace `{os.path.basename(path)}`: {len(rows)} kernels on {len(by)} streams; "
          f"GPU time with at least one kernel running: {busy / 1e6:.1f} ms.\n")
    print("| streams with a kernel running | ms | share of busy time |")
    print("|---|---|---|")
    for k in sorted(hist):
        print(f"| {k} | {hist[k] / 1e6:.1f} | {100 * hist[k] / busy:.1f}% |")
    per = sorted(((sum(b - a for a, b in iv), sid, len(iv)) for sid, iv in by.items()), reverse=True)
    print("\n| stream | kernels | kernel ms (sum of durations) |")
    print("|---|---|---|")
    for tot, sid, n in per:
        print(f"| {sid} | {n} | {tot / 1e6:.1f} |")


def serving_leg(fv, synth, np, torch, n_req: int, slots: int = 4) -> dict:
    """The serving mix: the first n_req requests of the seeded request stream
    (hex arrays of 37-350 antennas, log-uniform 1e3-1e6 sources, 1-64
    frequencies, eps in {1e-4, 1e-6, 1e-10}, Poisson arrivals at 100 Hz),
    drawn on the device.  One arrival trace is replayed by a single-stream FIFO
    of plain blocking calls and by the server, each once with host buffers and
    once with device-resident inputs; a saturation run then submits every
    request at t = 0 to each.  Latency = completion - scheduled arrival, so
    queueing counts in every mode.  gpu_busy_ms sums each request's stage
    event time; above the makespan it shows requests overlapping on the device."""
    reqs = synth.config5_requests(n_req)
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    din = [r.materialize_torch(dev) for r in reqs]
    torch.cuda.synchronize()
    hin = [tuple(x.cpu().numpy() for x in d) for d in din]
    t_mat = time.perf_counter() - t0
    npair = [r.n_ant * (r.n_ant + 1) // 2 for r in reqs]
    pairs = sum(float(r.n_src) * q * r.n_freq for r, q in zip(reqs, npair))
    trace = np.array([r.arrival_s for r in reqs])
    hps = [fv.HostProblem(*h, eps=r.eps, flags=fv.TIMING) for h, r in zip(hin, reqs)]
    houts = [np.empty((r.n_freq, q, 2)) for r, q in zip(reqs, npair)]
    douts = [torch.empty((r.n_freq, q, 2), dtype=torch.float64, device=dev) for r, q in zip(reqs, npair)]
    in_bytes = sum(sum(x.numel() * 8 for x in d) for d in din)

    def summary(lat_ms, done_s, busy_ms, arr):
        span = max(done_s) - min(arr)
        return {"pairs_per_s": pairs / span, "makespan_s": span,
                "latency_ms": {"p50": _pct(lat_ms, 0.5), "p90": _pct(lat_ms, 0.9), "p99": _pct(lat_ms, 0.99)},
                "gpu_busy_ms": busy_ms, "gpu_busy_over_makespan": busy_ms * 1e-3 / span}

    st = torch.cuda.Stream(device=dev)

    def plain(arr, device=False):
        lat, done, busy = [], [], 0.0
        ts = time.perf_counter()
        for k, at in enumerate(arr):
            now = time.perf_counter() - ts
            if now < at:
                time.sleep(at - now)
            if device:
                a = din[k]
                rep = c.simulate_dev(a[0], a[1], a[2], a[3], a[4], douts[k], eps=reqs[k].eps, flags=fv.TIMING,
                                     stream=st)
                st.synchronize()
            else:
                rep = c.simulate_into(hps[k], houts[k])
            t_done = time.perf_counter() - ts
            lat.append((t_done - at) * 1e3)
            done.append(t_done)
            busy += sum(rep["t_stage_ms"])
        return summary(lat, done, busy, arr)

    def served(arr, device):
        c.server_start(slots)
        sub = []
        ts = time.perf_counter()
        for k, at in enumerate(arr):
            now = time.perf_counter() - ts
            if now < at:
                time.sleep(at - now)
            t_sub = time.perf_counter() - ts
            if device:
                a = din[k]
                tk = c.submit_dev(a[0], a[1], a[2], a[3], a[4], douts[k], eps=reqs[k].eps, flags=fv.TIMING)
            else:
                tk = c.submit(hps[k], houts[k])
            sub.append((tk, t_sub))
        lat, done, busy = [], [], 0.0
        for k, (tk, t_sub) in enumerate(sub):
            st, rep = c.wait(tk)
            if st != 0:
                raise RuntimeError(f"serving request {k} failed with status {st}")
            t_done = t_sub + rep["t_total_ms"] * 1e-3
            lat.append((t_done - arr[k]) * 1e3)
            done.append(t_done)
            busy += sum(rep["t_stage_ms"])
        c.server_stop()
        return summary(lat, done, busy, arr)

    with fv.Context(0) as c:
        seen = set()
        for k, r in enumerate(reqs):  # warm: code objects and the tables of each (array, eps)
            if (r.n_ant, r.eps) not in seen:
                seen.add((r.n_ant, r.eps))
                c.simulate_into(hps[k], houts[k])
        res = {"trace": {"plain_fifo": plain(trace), "server_host": served(trace, False),
                         "plain_fifo_device": plain(trace, True), "server_device": served(trace, True)}}
        zero = np.zeros_like(trace)
        res["saturation"] = {"plain_fifo": plain(zero), "server_host": served(zero, False),
                             "plain_fifo_device": plain(zero, True), "server_device": served(zero, True)}
    torch.cuda.synchronize()
    for m in ("trace", "saturation"):
        for k in res[m].values():
            k.pop("latency_ms") if m == "saturation" else None
    res.update({"requests": len(reqs), "slots": slots, "arrival_rate_hz": len(reqs) / float(trace[-1] - trace[0]),
                "pairs": pairs, "input_bytes": in_bytes, "materialize_s": t_mat,
                "mix": {"n_ant": [min(r.n_ant for r in reqs), max(r.n_ant for r in reqs)],
                        "n_src": [min(r.n_src for r in reqs), max(r.n_src for r in reqs)],
                        "n_freq": [min(r.n_freq for r in reqs), max(r.n_freq for r in reqs)],
                        "eps": sorted({r.eps for r in reqs})},
                "note": "plain_fifo: one blocking fv_simulate per request in arrival order on one stream; "
                        "plain_fifo_device: the same with fv_simulate_dev on inputs resident in HBM; "
                        "server_host: fv_submit with host buffers (PCIe in the latency); server_device: "
                        "fv_submit_dev with inputs resident in HBM; latency from scheduled arrival to "
                        "completion; saturation: all requests at t = 0"})
    return res


def print_serving(res: dict) -> None:
    for mode in ("trace", "saturation"):
        for k, v in res[mode].items():
            lat = v.get("latency_ms")
            print(f"bench: serving {mode} {k}: {v['pairs_per_s']:.3e} pairs/s, makespan {v['makespan_s']:.2f} s, "
                  f"GPU busy/makespan {v['gpu_busy_over_makespan']:.2f}"
                  + (f", p50 {lat['p50']:.1f} ms p99 {lat['p99']:.1f} ms" if lat else ""), file=sys.stderr,
                  flush=True)


def batch_device_leg(fv, probs, np, torch, stream, tune) -> dict:
    """The config4 batch (24 LSTs x 43 frequencies of the 127-antenna hex,
    uneven source counts) with its inputs resident in HBM: the GPU stage time
    from one call with stage events, then the wall time of calls whose launch
    sequence is captured once and replayed (FV_GRAPH), each call's planning
    scalars copied back once and the stream synchronised after it."""
    dev = torch.device("cuda:0")
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)

    def items(flags):
        return [{"ant_enu": d(q.ant_enu), "src_lmn": d(q.src_lmn), "freq_hz": d(q.freq_hz), "flux": d(q.flux),
                 "beam": None if q.beam is None else d(q.beam),
                 "vis": torch.empty((q.n_freq, q.n_pairs, 2), dtype=torch.float64, device=dev),
                 "eps": q.eps, "flags": flags} for q in probs]

    with fv.Context(0) as c:
        timed = items(tune | fv.TIMING)
        c.simulate_batch_dev(timed, stream=stream)  # warm
        stream.synchronize()
        rep = c.simulate_batch_dev(timed, stream=stream)
        stream.synchronize()
        gpu_ms = sum(rep["t_stage_ms"])
        cap = c.prepare_batch_dev(items(fv.GRAPH))
        c.run_batch_dev(cap, stream=stream)  # capture
        stream.synchronize()
        walls = []
        for _ in range(10):
            t0 = time.perf_counter()
            c.run_batch_dev(cap, stream=stream)
            stream.synchronize()
            walls.append((time.perf_counter() - t0) * 1e3)
    wall = _pct(walls, 0.5)
    return {"workload": f"hex{probs[0].n_ant}, {len(probs)} LSTs x {probs[0].n_freq} freqs, inputs in HBM",
            "ms": wall, "gpu_stage_ms": gpu_ms, "wall_over_gpu": wall / gpu_ms,
            "pairs_per_s": rep["src_pairs"] / (wall * 1e-3), "lattice": rep["lattice"],
            "launches": {n: rep["stage_launches"][i] for i, n in enumerate(fv.STAGES) if rep["stage_launches"][i]},
            "stages_ms": {n: round(rep["t_stage_ms"][i], 3) for i, n in enumerate(fv.STAGES)
                          if rep["stage_launches"][i] > 0},
            "walls_ms": [round(w, 3) for w in walls],
            "note": "wall = median of 10 calls of a prepared batch, captured launch sequence replayed; each call "
                    "checks the inputs on the device and waits once for the planning scalars"}


def fp64_leg(fv, synth, np, torch, stream) -> dict:
    """The 350-antenna workload at eps = 1e-10 (FP64 grids, the paper's own
    arithmetic), type-3 path and the library's default (type-1) path: inputs in
    HBM, best of two calls after a warm-up; rel l2 against the oracle's exact
    sum on 512 seeded pairs x 4 frequencies."""
    import oracle
    p = synth.config2()
    dev = torch.device("cuda:0")
    g = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
    args = (g(p.ant_enu), g(p.src_lmn), g(p.freq_hz), g(p.flux), g(p.beam))
    vis = torch.empty((p.n_freq, p.n_pairs, 2), dtype=torch.float64, device=dev)
    sub = synth.subset_pairs(p.n_ant, 512, 11)
    fsel = np.array([0, 21, 42, 63])
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    ref = oracle.direct_vis(p.ant_enu, p.src_lmn, p.freq_hz[fsel], p.flux[fsel], p.beam[fsel], pairs=sub,
                            threads=threads)
    pairs = float(p.n_src) * p.n_pairs * p.n_freq
    out = {}
    with fv.Context(0) as c:
        for name, fl in (("type3", fv.NO_LATTICE), ("default", 0)):
            c.simulate_dev(*args, vis, eps=1e-10, flags=fl, stream=stream)
            torch.cuda.synchronize()
            ts = []
            for _ in range(2):
                t0 = time.perf_counter()
                rep = c.simulate_dev(*args, vis, eps=1e-10, flags=fl | fv.TIMING, stream=stream)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            o = vis.cpu().numpy()
            got = o[fsel][:, sub, 0] + 1j * o[fsel][:, sub, 1]
            out[name] = {"ms": min(ts) * 1e3, "pairs_per_s": pairs / min(ts), "prec_bits": rep["prec_bits"],
                         "w": rep["w"], "lattice": rep["lattice"], "n1": rep["n1"],
                         "rel_l2_vs_oracle": oracle.rel_l2(got, ref),
                         "stages_ms": {n: round(rep["t_stage_ms"][i], 3) for i, n in enumerate(fv.STAGES)
                                       if rep["stage_launches"][i] > 0}}
    return {"workload": "hex350, 1e5 sources, 64 freqs 100-200 MHz, eps 1e-10 (FP64 grids), inputs in HBM",
            **out}


def disk3d_leg(fv, synth, np, torch, stream) -> dict:
    """1000 antennas in a 500 m disk (3-D), 393k pixels, 16 frequencies:
    inputs in HBM, two timed calls after one warm-up call."""
    p = synth.config3()
    dev = torch.device("cuda:0")
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
    args = (d(p.ant_enu), d(p.src_lmn), d(p.freq_hz), d(p.flux), None if p.beam is None else d(p.beam))
    vis = torch.empty((p.n_freq, p.n_pairs, 2), dtype=torch.float64, device=dev)
    with fv.Context(0) as c:
        c.simulate_dev(*args, vis, eps=p.eps, flags=0, stream=stream)
        torch.cuda.synchronize()
        ts = []
        for _ in range(2):
            t0 = time.perf_counter()
            rep = c.simulate_dev(*args, vis, eps=p.eps, flags=fv.TIMING, stream=stream)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
    pairs = float(p.n_src) * p.n_pairs * p.n_freq
    t = min(ts)
    return {"workload": f"{p.n_ant} antennas in a 500 m disk, heights +-5 m (3-D), {p.n_src} pixels, "
                        f"{p.n_freq} freqs 150-170 MHz, eps 1e-6, inputs in HBM",
            "ms": t * 1e3, "pairs_per_s": pairs / t, "n1": rep["n1"],
            "stages_ms": {n: round(rep["t_stage_ms"][i], 3) for i, n in enumerate(fv.STAGES)
                          if rep["stage_launches"][i] > 0}}


def drift_leg(fv, synth, np, torch, stream) -> dict:
    """The config4 drift scan (hex127, 24 hourly LSTs x 43 frequencies, a
    102k-source equatorial sky) through the device front end: sky resident in
    HBM, rotation, beam and horizon cut on the device; two timed calls after one
    warm-up call.  Pairs count the sources above the horizon."""
    d = synth.config4_drift()
    dev = torch.device("cuda:0")
    g = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
    src, flux = g(d.src_eq), g(d.flux)
    vis = torch.empty((len(d.lst), len(d.freq_hz), d.n_pairs, 2), dtype=torch.float64, device=dev)
    with fv.Context(0) as c:
        run = lambda fl: c.simulate_drift(d.ant_enu, src, d.freq_hz, flux, d.lst, d.latitude, d.beam_fwhm,
                                          d.beam_nu_ref, vis, eps=d.eps, flags=fl, stream=stream)
        run(0)
        torch.cuda.synchronize()
        ts = []
        for _ in range(2):
            t0 = time.perf_counter()
            rep = run(0)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        rep_t = run(fv.TIMING)
        torch.cuda.synchronize()
    t = min(ts)
    n_snap = len(d.lst) * len(d.freq_hz)
    return {"workload": f"hex{d.ant_enu.shape[0]}, {len(d.lst)} LSTs x {len(d.freq_hz)} freqs = {n_snap} snapshots, "
                        f"{d.src_eq.shape[0]}-source equatorial sky in HBM, rotation + beam + horizon cut on the "
                        f"device, eps {d.eps:g}",
            "ms": t * 1e3, "pairs_per_s": rep["src_pairs"] / t,
            "visible_sources_per_snapshot": rep["src_pairs"] / (n_snap * d.n_pairs),
            "lattice": rep["lattice"], "gpu_stage_ms": sum(rep_t["t_stage_ms"])}


def multivector_legs(fv, synth, np, torch, stream) -> dict:
    """The HERA-350 workload with per-antenna beams (3 amplitude patterns,
    6 pattern pairs, antennas assigned at random) and as polarised products
    (Stokes I, Q, U, V with ideal feeds: 4 transforms): inputs in HBM, best of
    two timed calls after one warm-up call."""
    p = synth.config2()
    dev = torch.device("cuda:0")
    g = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
    rng = np.random.default_rng(350)
    ant, src, freq = g(p.ant_enu), g(p.src_lmn), g(p.freq_hz)
    pats = g(np.sqrt(p.beam)[None] * rng.uniform(0.8, 1.0, (3, 1, p.n_src)))
    which = rng.integers(0, 3, p.n_ant)
    stokes = g(np.concatenate([p.flux[None], rng.uniform(-0.1, 0.1, (3, 1, 1)) * p.flux[None]]))
    flux = g(p.flux)
    vis_b = torch.empty((p.n_freq, p.n_pairs, 2), dtype=torch.float64, device=dev)
    vis_p = torch.empty((4, p.n_freq, p.n_pairs, 2), dtype=torch.float64, device=dev)
    out = {}
    with fv.Context(0) as c:
        calls = {"beams_3_patterns": lambda: c.simulate_beams(ant, src, freq, flux, pats, which, vis_b,
                                                             eps=p.eps, stream=stream),
                 "polarised_4_products": lambda: c.simulate_polar(ant, src, freq, stokes, None, vis_p, eps=p.eps,
                                                                  stream=stream)}
        for name, call in calls.items():
            call()
            torch.cuda.synchronize()
            ts = []
            for _ in range(2):
                t0 = time.perf_counter()
                rep = call()
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            t = min(ts)
            out[name] = {"ms": t * 1e3, "pairs_per_s": rep["src_pairs"] / t, "lattice": rep["lattice"],
                         "transforms": 6 if name.startswith("beams") else 4}
    return out


def basis_leg(fv, synth, np, torch, stream) -> dict:
    """The spectral-basis path against the per-frequency type-3 path on two
    workloads: the HERA-350 workload (64 frequencies over an octave, lattice
    path off so both are type 3) and the 3-D disk workload (16 frequencies,
    150-170 MHz).  Reports each path's time (best of two after a warm-up) and
    the relative l2 difference of the two outputs (which holds the basis's fit
    of the spectra)."""
    out = {}
    dev = torch.device("cuda:0")
    g = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
    for name, p, K in (("basis_hex350_type3", synth.config2(), 12), ("basis_disk1000_3d", synth.config3(), 6)):
        args = (g(p.ant_enu), g(p.src_lmn), g(p.freq_hz), g(p.flux), None if p.beam is None else g(p.beam))
        v_ref = torch.empty((p.n_freq, p.n_pairs, 2), dtype=torch.float64, device=dev)
        v_b = torch.empty_like(v_ref)
        with fv.Context(0) as c:
            runs = {"per_frequency": lambda: c.simulate_dev(*args, v_ref, eps=p.eps, flags=fv.NO_LATTICE,
                                                            stream=stream),
                    "basis": lambda: c.simulate_basis(*args, v_b, K, eps=p.eps, stream=stream)}
            res = {}
            for k, call in runs.items():
                call()
                torch.cuda.synchronize()
                ts = []
                for _ in range(2):
                    t0 = time.perf_counter()
                    call()
                    torch.cuda.synchronize()
                    ts.append(time.perf_counter() - t0)
                res[k] = min(ts) * 1e3
        diff = float(torch.linalg.vector_norm(v_b - v_ref) / torch.linalg.vector_norm(v_ref))
        out[name] = {"n_freq": p.n_freq, "n_basis": K, "ms_per_frequency_path": res["per_frequency"],
                     "ms_basis": res["basis"], "rel_l2_basis_vs_per_frequency": diff}
        del v_ref, v_b, args
        torch.cuda.empty_cache()
    return out


def make_roofline(p, dom, per_launch_ms, per_launch_bytes, lattice, w):
    """Roofline entry of the dominant stage from its event time per launch."""
    achieved = per_launch_bytes / (per_launch_ms * 1e-3) / 1e9
    kernels = KERNEL_OF_STAGE_T1 if lattice else KERNEL_OF_STAGE
    traffic = _traffic_from_profiles(dom, "type1" if lattice else "type3")
    if lattice and dom == "spread":
        # The type-1 spread is bound by LDS atomic adds, not HBM: its
        # algorithmic LDS bytes are one 8-byte read-modify-write per source,
        # frequency and footprint cell (n_freq n_src w^2), against the LDS
        # bandwidth of the chip; its HBM bytes per launch are kept beside.
        lds_bytes = float(p.n_freq) * p.n_src * w * w * 8.0
        lds_achieved = lds_bytes / (per_launch_ms * 1e-3) / 1e9
        return {"bound": "alu", "resource": "LDS (64-bit integer atomic adds)", "kernel": kernels[dom],
                "stage": dom, "achieved": lds_achieved, "peak": LDS_PEAK_GBS, "unit": "GB/s",
                "frac": lds_achieved / LDS_PEAK_GBS, "traffic": traffic, "avg_launch_ms": per_launch_ms,
                "lds_bytes_per_launch": lds_bytes, "hbm_bytes_per_launch": per_launch_bytes,
                "hbm_achieved": achieved}
    return {"bound": "hbm", "kernel": kernels.get(dom, dom), "stage": dom, "achieved": achieved,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "avg_launch_ms": per_launch_ms, "bytes_per_launch": per_launch_bytes}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=500,
                    help="untimed steps first (about a second on the type-3 path: a fresh GPU is still ramping up)")
    ap.add_argument("--n-src", type=int, default=100_000)
    ap.add_argument("--n-freq", type=int, default=64)
    ap.add_argument("--no-direct", action="store_true", help="skip the direct-sum comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline and parity sample")
    ap.add_argument("--profile", action="store_true", help="short run for a profiler: no direct, no CPU leg")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the steps, one device copy of this many MiB (reference for byte counters)")
    ap.add_argument("--autotune", action="store_true", help="tune the FFT launch shape on the first warm-up call")
    ap.add_argument("--no-extras", action="store_true", help="skip the graph-replay and batch legs")
    ap.add_argument("--serve-requests", type=int, default=500, help="requests of the serving mix leg")
    ap.add_argument("--only", choices=("serving", "basis", "fp64", "drift", "vectors", "disk3d"),
                    help="run one extra leg alone and print it")
    ap.add_argument("--overlap-md", metavar="KERNEL_TRACE_CSV",
                    help="no run: print how much of the serving slots' kernel time overlaps across streams, "
                         "from a rocprofv3 --kernel-trace CSV of a --only serving run")
    ap.add_argument("--path", choices=("type3", "auto"), default="type3",
                    help="type3: the type-3 NUFFT (every step of the hot path; the default); auto: the "
                         "library's choice, which is the type-1 path for this lattice array")
    ap.add_argument("--stats-md", metavar="KERNEL_STATS_CSV",
                    help="no run: print a markdown table of a rocprofv3 --stats kernel summary")
    ap.add_argument("--reduce-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="no run: reduce two counter-collection CSVs of a --profile --calib-copy-mib run")
    args = ap.parse_args()
    if args.stats_md:
        stats_md(args.stats_md)
        return
    if args.overlap_md:
        overlap_md(args.overlap_md)
        return
    if args.reduce_traffic:
        cmd = ("rocprofv3 --pmc COUNTER --output-format csv -d <out> -o run -- python3 bench.py --profile "
               f"--steps 2 --warmup 1 --calib-copy-mib {args.calib_copy_mib or 256}"
               + (" --path auto" if args.path == "auto" else ""))
        reduce_traffic(args.reduce_traffic[0], args.reduce_traffic[1], args.calib_copy_mib or 256, cmd,
                       "hex350 14.6 m, 1e5 sources, 64 frequencies, eps 1e-6")
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print("bench.py: this build measures one GPU; the multi-GPU sharding (snapshots across GPUs, or "
              "slab-decomposed FFT with one all-to-all) is a design only.  Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.profile:
        args.no_direct = True
        args.no_cpu = True
        args.no_extras = True

    import numpy as np
    import torch
    import paper_2506_02130_amd as fv
    import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.only == "serving":
        res = serving_leg(fv, synth, np, torch, args.serve_requests)
        print_serving(res)
        print(json.dumps({"serving": res}))
        return
    if args.only == "basis":
        print(json.dumps(basis_leg(fv, synth, np, torch, torch.cuda.Stream())))
        return
    if args.only == "fp64":
        print(json.dumps(fp64_leg(fv, synth, np, torch, torch.cuda.Stream())))
        return
    if args.only == "disk3d":
        print(json.dumps(disk3d_leg(fv, synth, np, torch, torch.cuda.Stream())))
        return
    if args.only == "drift":
        print(json.dumps(drift_leg(fv, synth, np, torch, torch.cuda.Stream())))
        return
    if args.only == "vectors":
        print(json.dumps(multivector_legs(fv, synth, np, torch, torch.cuda.Stream())))
        return
    dev = torch.device("cuda:0")
    p = synth.config2(n_src=args.n_src, n_freq=args.n_freq)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
    ant, src, freq, flux, beam = d(p.ant_enu), d(p.src_lmn), d(p.freq_hz), d(p.flux), d(p.beam)
    vis = torch.empty((p.n_freq, p.n_pairs, 2), dtype=torch.float64, device=dev)
    stream = torch.cuda.Stream(device=dev)
    ctx = fv.Context(0)
    pairs_per_step = float(p.n_src) * p.n_pairs * p.n_freq
    # with --autotune the FFT launch shape is tuned on the first warm-up call (cached after)
    tune = fv.AUTOTUNE if args.autotune else 0
    # stage events without waiting (TIMING_ACCUM), summed with ctx.stage_times()
    base = fv.TIMING_ACCUM | tune | (fv.NO_LATTICE if args.path == "type3" else 0)

    def step(fl=base):
        return ctx.simulate_dev(ant, src, freq, flux, beam, vis, eps=p.eps, flags=fl, stream=stream)

    def stage_table(t, rep):
        names = fv.STAGES
        ms = {n: t["ms"][i] / max(t["calls"], 1) for i, n in enumerate(names)}
        launches = {n: rep["stage_launches"][i] for i, n in enumerate(names)}
        nbytes = {n: rep["stage_bytes"][i] for i, n in enumerate(names)}
        return ms, launches, nbytes

    print(f"bench: workload {p.name}, pairs/step {pairs_per_step:.3e}", file=sys.stderr, flush=True)
    warm = [step() for _ in range(max(args.warmup, 1))]
    torch.cuda.synchronize()
    # the dominant stage, from the stage events of two more steps (the
    # warm-up's events, with first-call effects, are dropped)
    ctx.stage_times()
    warm += [step() for _ in range(2)]
    torch.cuda.synchronize()
    w_ms, w_launch, _ = stage_table(ctx.stage_times(), warm[-1])
    dom = max((n for n in fv.STAGES if w_launch[n] > 0), key=lambda n: w_ms[n])
    # in the timed steps only the dominant stage records events (two per launch
    # of it: the least the live measurement costs)
    flags = base | fv.timing_stage(dom)

    # ---------------------------------------------------------------- timed region
    reps = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        reps.append(step(flags))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timed = ctx.stage_times()  # the timed steps' events (the dominant kernel's)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = pairs_per_step / ((t1 - t0) / args.steps)
    print(f"bench: {ms_per_step:.3f} ms/step, {value:.3e} pairs/s", file=sys.stderr, flush=True)
    # every stage's event times, over as many steps again after the timed region
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    stage_ms, stage_launch, stage_bytes = stage_table(ctx.stage_times(), reps[0])
    # per-call latency (submit to completion), after the timed region
    lat = []
    for _ in range(2 if args.profile else max(20, min(args.steps, 50))):
        tl = time.perf_counter()
        step(fl=base & ~fv.TIMING_ACCUM)  # the same path, no timing
        stream.synchronize()
        lat.append((time.perf_counter() - tl) * 1e3)

    if args.calib_copy_mib:
        n = args.calib_copy_mib * (1 << 20) // 4
        xa = torch.ones(n, dtype=torch.float32, device=dev)
        xb = torch.empty_like(xa)
        torch.cuda.synchronize()
        xb.copy_(xa)
        torch.cuda.synchronize()
        del xa, xb

    # the dominant kernel's HIP-event time per launch, measured in the timed steps
    names = fv.STAGES
    live_ms, _, _ = stage_table(timed, reps[0])
    lattice = bool(reps[-1].get("lattice"))
    roofline = make_roofline(p, dom, live_ms[dom] / max(stage_launch[dom], 1),
                             stage_bytes[dom] / max(stage_launch[dom], 1), lattice, reps[-1]["w"])
    stages = {n: {"ms": round(stage_ms[n], 4), "launches": stage_launch[n],
                  "GBps": (stage_bytes[n] / max(stage_launch[n], 1)) / (stage_ms[n] / max(stage_launch[n], 1) * 1e-3)
                  / 1e9 if stage_ms[n] > 0 else None}
              for n in names if stage_launch[n] > 0}

    # ---------------------------------------------------------------- parity + CPU baseline
    rel_err = None
    cpu = None
    if not args.no_cpu:
        import oracle
        sub = synth.subset_pairs(p.n_ant, 4096, 7)
        fsel = np.linspace(0, p.n_freq - 1, min(16, p.n_freq)).round().astype(int)
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
        tc0 = time.perf_counter()
        ref = oracle.direct_vis(p.ant_enu, p.src_lmn, p.freq_hz[fsel], p.flux[fsel], p.beam[fsel], pairs=sub,
                                threads=threads)
        tc1 = time.perf_counter()
        cpu_pairs = float(p.n_src) * len(sub) * len(fsel)
        cpu = {"value": cpu_pairs / (tc1 - tc0), "unit": "src×baseline pairs/s", "cores": threads,
               "cpu_model": _cpu_model(), "kind": "oracle", "sample": f"{len(sub)} seeded pairs x {p.n_src} sources x {len(fsel)} of "
                                           f"{p.n_freq} frequencies ({cpu_pairs:.2e} pairs, {tc1 - tc0:.1f} s)"}
        out = vis.cpu().numpy()
        got = out[fsel][:, sub, 0] + 1j * out[fsel][:, sub, 1]
        rel_err = oracle.rel_l2(got, ref)
        print(f"bench: rel l2 vs oracle on the sample {rel_err:.3e}; oracle {cpu['value']:.3e} pairs/s",
              file=sys.stderr, flush=True)

    # ---------------------------------------------------------------- direct-sum kernels
    direct = {}
    if not args.no_direct:
        for name, method, fl in (("direct_valu", fv.METHOD_DIRECT, fv.TIMING | fv.METHOD_DIRECT),
                                 ("direct_mfma", fv.METHOD_MFMA, fv.TIMING | fv.METHOD_MFMA)):
            vis_d = torch.empty_like(vis)
            r = ctx.simulate_dev(ant, src, freq, flux, beam, vis_d, eps=p.eps, flags=fl, stream=stream)
            torch.cuda.synchronize()
            ts = []
            for _ in range(2):
                ta = time.perf_counter()
                ctx.simulate_dev(ant, src, freq, flux, beam, vis_d, eps=p.eps, flags=fl, stream=stream)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - ta)
            t = min(ts)
            a = vis.cpu().numpy()
            b = vis_d.cpu().numpy()
            import oracle as _o
            diff = _o.rel_l2(a[..., 0] + 1j * a[..., 1], b[..., 0] + 1j * b[..., 1])
            direct[name] = {"pairs_per_s": pairs_per_step / t, "ms": t * 1e3, "nufft_vs_direct_rel_l2": diff}
            if method == fv.METHOD_MFMA:
                # one complex multiply-add (8 real flops) per source, pair and frequency
                tf = 8.0 * pairs_per_step / t / 1e12
                direct[name].update({"alg_TFLOPs": tf, "peak_TFLOPs": FP32_MATRIX_PEAK_TFLOPS,
                                     "frac": tf / FP32_MATRIX_PEAK_TFLOPS})
            del vis_d
        best = max(v["pairs_per_s"] for v in direct.values())
        direct["nufft_speedup_over_best_direct"] = value / best

    # ---------------------------------------------------------------- graph replay and batched snapshots
    extras = {}
    n_extra = max(1, min(args.steps, 20))  # steps per leg outside the timed region
    if not args.no_extras:
        # the same workload on the other path: the library's choice (the type-1
        # path, as the hex array is a lattice) when the timed steps ran type 3,
        # else type 3; timed like the main steps (stage events summed after)
        other = "auto" if args.path == "type3" else "type3"
        ofl = fv.TIMING_ACCUM | tune | (fv.NO_LATTICE if other == "type3" else 0)
        n_other = args.steps
        # as the main path: the warm-up names the dominant stage, the timed steps
        # record only its events, every stage's events come from a pass after
        warm_o = [step(ofl) for _ in range(20)]
        torch.cuda.synchronize()
        w_ms, w_launch, _ = stage_table(ctx.stage_times(), warm_o[-1])
        o_dom = max((n for n in names if w_launch[n] > 0), key=lambda n: w_ms[n])
        t30 = time.perf_counter()
        r3 = [step(ofl | fv.timing_stage(o_dom)) for _ in range(n_other)]
        torch.cuda.synchronize()
        t3_ms = (time.perf_counter() - t30) * 1e3 / n_other
        live_o, _, _ = stage_table(ctx.stage_times(), r3[0])
        for _ in range(n_other):
            step(ofl)
        torch.cuda.synchronize()
        o_ms, o_launch, o_bytes = stage_table(ctx.stage_times(), r3[0])
        o_lat = bool(r3[-1].get("lattice"))
        key = "lattice_type1" if o_lat else "type3"
        extras[key] = {"path": "type-1 (lattice array; the library's default for this array)" if o_lat else "type-3",
                       "ms_per_step": t3_ms, "pairs_per_s": pairs_per_step / (t3_ms * 1e-3), "steps": n_other,
                       "stages_ms": {n: round(o_ms[n], 4) for n in names if o_launch[n] > 0},
                       "roofline": make_roofline(p, o_dom, live_o[o_dom] / max(o_launch[o_dom], 1),
                                                 o_bytes[o_dom] / max(o_launch[o_dom], 1), o_lat, r3[-1]["w"]),
                       "n1": r3[-1]["n1"][:2], "w": r3[-1]["w"]}
        print(f"bench: {extras[key]['path']} {t3_ms:.3f} ms/step", file=sys.stderr, flush=True)
        gfl = fv.GRAPH | fv.NO_LATTICE | tune
        for _ in range(2):
            step(gfl)
        torch.cuda.synchronize()
        tg0 = time.perf_counter()
        for _ in range(n_extra):
            step(gfl)
        torch.cuda.synchronize()
        g_ms = (time.perf_counter() - tg0) * 1e3 / n_extra
        # FV_DETERMINISTIC: records ranked by source index inside each sub-bin
        dfl = fv.DETERMINISTIC | fv.NO_LATTICE | tune | fv.TIMING
        for _ in range(2):
            step(dfl)
        torch.cuda.synchronize()
        td0 = time.perf_counter()
        for _ in range(n_extra):
            rd = step(dfl)
        torch.cuda.synchronize()
        d_ms = (time.perf_counter() - td0) * 1e3 / n_extra
        extras["deterministic"] = {"ms_per_step": d_ms, "pairs_per_s": pairs_per_step / (d_ms * 1e-3),
                                   "stages_ms": {n: round(rd["t_stage_ms"][i], 4) for i, n in enumerate(fv.STAGES)
                                                 if rd["stage_launches"][i] > 0},
                                   "note": "type-3 path with FV_DETERMINISTIC (bit-reproducible spread order), "
                                           "per-call stage events"}
        print(f"bench: deterministic {d_ms:.3f} ms/step", file=sys.stderr, flush=True)
        extras["graph_replay"] = {"ms_per_step": g_ms, "pairs_per_s": pairs_per_step / (g_ms * 1e-3),
                                  "note": "type-3 path of the same workload, launch sequence replayed as a HIP "
                                          "graph, no stage events"}
        probs = synth.config4()
        hps = [fv.HostProblem.of(q, flags=tune | fv.TIMING) for q in probs]
        ctx.simulate_batch(hps)  # warm: target tables, tuning
        tb0 = time.perf_counter()
        ctx.simulate_batch(hps)
        tb = time.perf_counter() - tb0
        rb = ctx.last_report
        extras["batch_config4"] = {
            "workload": f"hex{probs[0].n_ant}, {len(probs)} LSTs x {probs[0].n_freq} freqs = "
                        f"{len(probs) * probs[0].n_freq} snapshots, {min(q.n_src for q in probs)}-"
                        f"{max(q.n_src for q in probs)} sources, host buffers (PCIe included)",
            "pairs_per_s": rb["src_pairs"] / tb, "ms": tb * 1e3,
            "gpu_stage_ms": sum(rb["t_stage_ms"]), "gpu_pairs_per_s": rb["src_pairs"] / (sum(rb["t_stage_ms"]) * 1e-3)}
        extras["batch_config4_device"] = batch_device_leg(fv, probs, np, torch, stream, tune)
        print(f"bench: graph replay {g_ms:.3f} ms/step; batch of {len(probs)} x {probs[0].n_freq} snapshots "
              f"{tb * 1e3:.1f} ms (host buffers), {extras['batch_config4_device']['ms']:.2f} ms wall, "
              f"{extras['batch_config4_device']['gpu_stage_ms']:.2f} ms GPU stages (inputs in HBM, captured)",
              file=sys.stderr, flush=True)
        extras["serving"] = serving_leg(fv, synth, np, torch, args.serve_requests)
        print_serving(extras["serving"])
        extras["disk1000_3d"] = disk3d_leg(fv, synth, np, torch, stream)
        extras["hex350_fp64_eps1e-10"] = fp64_leg(fv, synth, np, torch, stream)
        x = extras["hex350_fp64_eps1e-10"]
        print(f"bench: eps 1e-10 (FP64) type-3 {x['type3']['ms']:.2f} ms (rel l2 {x['type3']['rel_l2_vs_oracle']:.1e}), "
              f"default path {x['default']['ms']:.2f} ms (rel l2 {x['default']['rel_l2_vs_oracle']:.1e})",
              file=sys.stderr, flush=True)
        extras["drift_config4"] = drift_leg(fv, synth, np, torch, stream)
        extras.update(multivector_legs(fv, synth, np, torch, stream))
        extras.update(basis_leg(fv, synth, np, torch, stream))
        print("bench: spectral basis " + ", ".join(
            f"{k}: {v['ms_basis']:.2f} ms vs {v['ms_per_frequency_path']:.2f} ms (diff {v['rel_l2_basis_vs_per_frequency']:.1e})"
            for k, v in extras.items() if k.startswith("basis_")), file=sys.stderr, flush=True)
        print(f"bench: per-antenna beams {extras['beams_3_patterns']['ms']:.2f} ms, polarised "
              f"{extras['polarised_4_products']['ms']:.2f} ms", file=sys.stderr, flush=True)
        print(f"bench: drift scan {extras['drift_config4']['ms']:.1f} ms "
              f"({extras['drift_config4']['pairs_per_s']:.3e} pairs/s)", file=sys.stderr, flush=True)

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "src×baseline pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"hex{p.n_ant} 14.6 m, {p.n_src} power-law sources, Gaussian beam, {p.n_freq} freqs "
                               f"100-200 MHz, eps 1e-6, 2-D, FP32 grids, inputs in HBM",
                   "path": "type-1 (lattice array)" if reps[-1].get("lattice") else "type-3 NUFFT (every hot-path step)",
                   "n_ant": p.n_ant, "n_pairs": p.n_pairs, "n_src": p.n_src, "n_freq": p.n_freq, "eps": p.eps,
                   "parallelism": "1 GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "rel_l2_vs_oracle": rel_err,
        "latency_ms": {"p50": _pct(lat, 0.5), "p99": _pct(lat, 0.99), "kind": "per call, submit to completion, host clock (after the timed region)"},
        "stages": stages,
        "stages_kind": (f"HIP-event ms per step of each stage over {args.steps} steps after the timed region; "
                        f"roofline.avg_launch_ms is the {dom} kernel's own events in the timed steps"),
        "direct": direct or None,
        "extras": extras or None,
        "report": {k: reps[-1][k] for k in ("dim", "prec_bits", "w", "fold_axis", "n1", "n2", "model_bytes",
                                            "lattice")},
    }
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
