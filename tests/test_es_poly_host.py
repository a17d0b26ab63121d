"""The FP32 kernel weights the spreading and interpolation kernels take from
piecewise polynomials (fitted on the host, in libfv.so) against the oracle's
ES kernel (paper section 2.2), evaluated in FP32 the way the kernels evaluate
them: for every FP32 width the weights stay within exp(-beta) (the size of the
kernel's own value at the edge of its support) or FP32 rounding, whichever is
larger.  Runs without a GPU (host code only)."""
import ctypes
import os

import numpy as np
import pytest

from oracle import es_kernel

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2506_02130_amd", "libfv.so")
MAXW, NC = 8, 11  # widths with polynomial tables; coefficients per piece (degree <= 10)


def _table(w):
    lib = ctypes.CDLL(LIB)
    try:
        f = getattr(lib, "_ZN2fv7es_polyEi")  # const EsPoly &fv::es_poly(int)
    except AttributeError:
        pytest.skip("host table not exported by this build")
    f.restype = ctypes.c_void_p
    f.argtypes = [ctypes.c_int]
    addr = f(w)
    return np.ctypeslib.as_array((ctypes.c_float * ((MAXW + 1) // 2 * NC)).from_address(addr)).reshape(-1, NC).copy()


def _weights_fp32(c, w, u):
    """All w weights at u = 2 offset - w + 1, in FP32, with the kernels' even/odd
    Horner scheme (piece w - 1 - i is piece i at -u)."""
    d = w + 2
    de, do = d - (d & 1), d - 1 + (d & 1)
    u = np.asarray(u, dtype=np.float32)
    v = u * u
    out = np.zeros((w,) + u.shape, dtype=np.float32)
    for i in range((w + 1) // 2):
        e = np.full_like(u, c[i, de])
        for k in range(de - 2, -1, -2):
            e = (e * v + np.float32(c[i, k])).astype(np.float32)
        od = np.full_like(u, c[i, do])
        for k in range(do - 2, 0, -2):
            od = (od * v + np.float32(c[i, k])).astype(np.float32)
        out[i] = u * od + e
        out[w - 1 - i] = -u * od + e
    return out


@pytest.mark.parametrize("w", [3, 4, 5, 6, 7, 8])
def test_polynomial_weights_follow_the_es_kernel(w):
    if not os.path.exists(LIB):
        pytest.skip("libfv.so not built")
    c = _table(w)
    beta = es_kernel.es_beta(w)
    u = np.linspace(-1.0, 1.0, 4001)
    off = (u + w - 1) / 2.0                          # the offset from the first cell, in (w/2 - 1, w/2]
    got = _weights_fp32(c, w, u).astype(np.float64)
    ref = np.stack([es_kernel.es_phi((i - off) * 2.0 / w, beta) for i in range(w)])
    err = np.abs(got - ref).max()
    # the fit's error (about exp(-beta)) or FP32 rounding, whichever is larger; a
    # wrong piece order, mirror or sign would be an error of order one
    tol = max(np.exp(-beta), 2 * np.finfo(np.float32).eps)
    assert err <= tol, (w, err, tol)


def test_no_table_beyond_the_fp32_widths():
    if not os.path.exists(LIB):
        pytest.skip("libfv.so not built")
    assert not np.any(_table(MAXW + 1))
