"""Oracle: plain, slow, obviously-correct CPU reference for the visibility sum.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import it; the product library neither
imports nor links anything here, and nothing here imports the product.

Contents
  * ``direct_vis``  -- FP64 direct sum in plain C (``direct.c``), the
    definition the type-3 NUFFT approximates (paper section 2.2, the
    point-source sum and the type-3 form it is rewritten as; pair
    orientation from the phasor factorisation of section 5.1).
  * ``es_kernel``   -- the ES kernel and its Fourier transform by quadrature.
  * ``type3``       -- the type-3 transform taken step by step in numpy FP64
    (spread, oversampled FFT, deconvolve + interpolate), for per-stage checks.
  * ``type1``       -- lattice detection and the type-1 steps for gridded
    arrays (section 2.2.1).
  * ``beams``       -- the direct sum with per-antenna beam patterns
    (section 2.2.3), pair by pair.
  * ``polar``       -- polarised feed products, the Jones-form sum of
    section 2.1 with a shared beam, source by source.
  * ``basis``       -- spectral-basis evaluation (appendix A): projection,
    structure constants, one transform per basis function, expansion.
  * ``frontend``    -- drift-scan front end: rotation of equatorial directions
    to ENU per sidereal time (section 2.3) and an analytic Gaussian power beam
    (section 2.4).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_build", "liboracle_direct.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile direct.c into a shared library with gcc (-O2, OpenMP, IEEE math)."""
    if force or not os.path.exists(_LIB_PATH):
        os.makedirs(os.path.dirname(_LIB_PATH), exist_ok=True)
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-D_GNU_SOURCE", os.path.join(_HERE, "direct.c"), "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.oracle_direct_vis.restype = ctypes.c_int
        lib.oracle_direct_vis.argtypes = [
            ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int64,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def direct_vis(ant_enu, src_lmn, freq_hz, flux, beam=None, pairs=None, drop_up: bool = False,
               threads: int = 0) -> np.ndarray:
    """V[f, k] = sum_s beam*flux * exp(-2 pi i nu_f/c (x_i - x_j) . s_hat_s), complex128.

    ``pairs``: optional subset of (i<=j) row-major pair indices (else all).
    ``drop_up``: evaluate u*l + v*m only (the coplanar form)."""
    lib = _load()
    ant = np.ascontiguousarray(ant_enu, dtype=np.float64)
    src = np.ascontiguousarray(src_lmn, dtype=np.float64).reshape(-1, 3)
    freq = np.ascontiguousarray(freq_hz, dtype=np.float64).reshape(-1)
    n_ant, n_src, n_freq = ant.shape[0], src.shape[0], freq.shape[0]
    fl = np.ascontiguousarray(flux, dtype=np.float64).reshape(n_freq, n_src)
    bm = None if beam is None else np.ascontiguousarray(beam, dtype=np.float64).reshape(n_freq, n_src)
    n_pairs = n_ant * (n_ant + 1) // 2
    pr = None if pairs is None else np.ascontiguousarray(pairs, dtype=np.int64)
    n_out = n_pairs if pr is None else pr.shape[0]
    out = np.zeros((n_freq, n_out, 2), dtype=np.float64)
    rc = lib.oracle_direct_vis(n_ant, _ptr(ant), n_src, _ptr(src), n_freq, _ptr(freq), _ptr(fl),
                               _ptr(bm), 1 if drop_up else 0, n_out, _ptr(pr), _ptr(out), int(threads))
    if rc != 0:
        raise ValueError("oracle_direct_vis rejected its arguments")
    return out[..., 0] + 1j * out[..., 1]


def direct_problem(problem, pairs=None, drop_up: bool = False, threads: int = 0) -> np.ndarray:
    """direct_vis on a synth.Problem."""
    return direct_vis(problem.ant_enu, problem.src_lmn, problem.freq_hz, problem.flux, problem.beam,
                      pairs=pairs, drop_up=drop_up, threads=threads)


def rel_l2(a: np.ndarray, ref: np.ndarray) -> float:
    """Relative l2 error ||a - ref|| / ||ref|| over the whole array (the
    error measure every result is held to)."""
    den = float(np.linalg.norm(ref))
    num = float(np.linalg.norm(np.asarray(a) - ref))
    if den == 0.0:
        return 0.0 if num == 0.0 else float("inf")
    return num / den
