"""The C-ABI library loads and exports every symbol include/fv.h declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"\b(fv_[a-z_]+)\s*\(", src))
    return sorted(names)


def test_header_declares_entry_points():
    d = _declared()
    for n in ("fv_create", "fv_destroy", "fv_simulate", "fv_simulate_dev", "fv_simulate_batch", "fv_server_start",
              "fv_submit", "fv_wait", "fv_server_stop", "fv_last_error", "fv_debug_stages"):
        assert n in d


def test_library_exports_every_declared_symbol():
    lib_path = os.path.join(ROOT, "paper_2506_02130_amd", "libfv.so")
    if not os.path.exists(lib_path):
        pytest.skip("libfv.so not built")
    lib = ctypes.CDLL(lib_path)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_the_header_symbols():
    lib_path = os.path.join(ROOT, "paper_2506_02130_amd", "libfv.so")
    if not os.path.exists(lib_path):
        pytest.skip("libfv.so not built")
    import paper_2506_02130_amd as fv
    assert sorted(fv.ABI_SYMBOLS) == _declared()


def test_product_does_not_import_oracle():
    for dirpath, _, files in os.walk(os.path.join(ROOT, "paper_2506_02130_amd")):
        for fn in files:
            if fn.endswith((".py", ".cpp", ".hip", ".h")):
                src = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in src and "from oracle" not in src and "oracle/" not in src, fn


def test_binding_flags_and_stage_indices_match_the_header():
    """The binding's flag constants and stage names follow include/fv.h."""
    import paper_2506_02130_amd as fv
    src = open(os.path.join(ROOT, "include", "fv.h")).read()
    defs = dict(re.findall(r"#define\s+(FV_[A-Z0-9_]+)\s+(0x[0-9A-Fa-f]+|\d+)u?\b", src))
    for name in ("TIMING", "AUTOTUNE", "GRAPH", "NO_LATTICE", "TIMING_ACCUM", "TIMING_ONE_STAGE"):
        assert getattr(fv, name) == int(defs["FV_" + name], 0), name
    for i, st in enumerate(fv.STAGES):
        assert int(defs["FV_STAGE_" + st.upper()], 0) == i, st
    assert "(FV_TIMING_ONE_STAGE | ((unsigned)(s) << 16))" in src
    assert fv.timing_stage("fft_x") == fv.TIMING_ONE_STAGE | (2 << 16)
    assert fv.timing_stage(1) == fv.timing_stage("spread")
    with pytest.raises(ValueError):
        fv.timing_stage("nope")
    with pytest.raises(ValueError):
        fv.timing_stage(len(fv.STAGES))
