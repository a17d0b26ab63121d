"""Host-side pieces of bench.py: the multi-GPU refusal, the reduction of two
byte-counter runs to per-stage traffic, and the rule that traffic figures are
dropped once the measured path's device sources change."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def _csv(path, rows):
    with open(path, "w") as f:
        f.write("Dispatch_Id,Kernel_Name,Counter_Value\n")
        for i, (name, v) in enumerate(rows):
            f.write(f'{i},"{name}",{v}\n')


def test_reduce_traffic_scales_by_the_copy_and_keeps_the_last_step(tmp_path, monkeypatch):
    step = [("fv::(anonymous namespace)::k_validate(double const*)", 100.0),
            ("fv::(anonymous namespace)::k_validate_reduce(double const*)", 1.0),
            ("void fv::(anonymous namespace)::k_t1_spread<float, 8>(fv::T1Params)", 50.0),
            ("fv::(anonymous namespace)::k_t1_rows(fv::T1Params)", 20.0),
            ("fv::(anonymous namespace)::k_t1_cols(fv::T1Params)", 5.0),
            ("fv::(anonymous namespace)::k_t1_out(fv::T1Params)", 2.0)]
    fetch = step + step + [("__amd_rocclr_copyBuffer", 131072.0)]
    write = [(n, v / 2) for n, v in step + step] + [("__amd_rocclr_copyBuffer", 262144.0)]
    _csv(tmp_path / "f.csv", fetch)
    _csv(tmp_path / "w.csv", write)
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    csrc = tmp_path / "paper_2506_02130_amd" / "csrc"
    csrc.mkdir(parents=True)
    for fn in bench.PATH_SOURCES["type1"]:
        (csrc / fn).write_text("kernel source " + fn)
    bench.reduce_traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), 256, "cmd", "w")
    d = json.load(open(prof / "traffic_c2_type1.json"))
    assert d["path"] == "type1"
    assert d["calibration"]["fetch_scale"] == pytest.approx(2.0)
    sp = d["stages"]["spread"]
    assert sp["launches"] == 1  # only the last step
    assert sp["fetch_bytes"] == pytest.approx(50.0 * 2.0 * 1024)
    assert sp["write_bytes"] == pytest.approx(25.0 * 1.0 * 1024)
    assert bench._traffic_from_profiles("spread", "type1") == pytest.approx(sp["bytes_per_launch"])
    assert bench._traffic_from_profiles("spread", "type3") is None  # other path
    (csrc / "lattice.hip").write_text("changed")
    assert bench._traffic_from_profiles("spread", "type1") is None  # stale after a source change
