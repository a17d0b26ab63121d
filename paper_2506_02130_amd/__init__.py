"""Python binding of libfv.so, the MI355X type-3 NUFFT visibility simulator.

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI declared in ``include/fv.h``.  There is no CPU
fallback; importing this package raises if the library has not been built.

    import paper_2506_02130_amd as fv
    ctx = fv.Context()
    vis = ctx.simulate(ant_enu, src_lmn, freq_hz, flux, beam, eps=1e-6)   # [n_freq, n_pairs] complex128
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfv.so")

OK, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED, EBUSY, ECANCELLED, ETIMEOUT = 0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "EUNSUPPORTED", -5: "EBUSY",
                -6: "ECANCELLED", -7: "ETIMEOUT"}

DIM_AUTO, DIM_2D, DIM_3D = 0x0, 0x1, 0x2
PREC_AUTO, PREC_FP32, PREC_FP64 = 0x0, 0x4, 0x8
METHOD_NUFFT, METHOD_DIRECT, METHOD_MFMA = 0x00, 0x10, 0x20
NO_FOLD = 0x100
TIMING = 0x200
AUTOTUNE = 0x400
GRAPH = 0x800
NO_LATTICE = 0x1000
TIMING_ACCUM = 0x2000  # stage events without waiting; sums from Context.stage_times()
DETERMINISTIC = 0x8000  # bitwise reproducible type-3 spread order
TIMING_ONE_STAGE = 0x4000  # with TIMING or TIMING_ACCUM: only one stage (flag bits 16-19) records events
STAGES = ("sort", "spread", "fft_x", "fft_y", "fft_z", "interp", "direct", "other")


def timing_stage(stage) -> int:
    """Flags that restrict event recording to one stage (a name of STAGES or
    its index), as FV_TIMING_STAGE(s); combine with TIMING or TIMING_ACCUM."""
    s = STAGES.index(stage) if isinstance(stage, str) else int(stage)
    if not 0 <= s < len(STAGES):
        raise ValueError(f"no stage {stage!r}")
    return TIMING_ONE_STAGE | (s << 16)

ABI_SYMBOLS = ("fv_create", "fv_destroy", "fv_last_error", "fv_simulate", "fv_simulate_dev", "fv_simulate_batch",
               "fv_server_start", "fv_submit", "fv_wait", "fv_server_stop", "fv_set_tune_cache", "fv_debug_stages",
               "fv_simulate_drift", "fv_simulate_beams", "fv_simulate_polar", "fv_simulate_basis",
               "fv_stage_times", "fv_simulate_mfma_noalloc", "fv_simulate_batch_dev", "fv_submit_dev")



def _dev_problem(ant_enu, src_lmn, freq_hz, flux, beam, vis, eps, flags) -> "Problem":
    """The C struct of one problem whose arrays are torch device tensors;
    every size is checked here, since the C ABI takes bare device pointers."""
    import torch
    for name, t in (("ant_enu", ant_enu), ("src_lmn", src_lmn), ("freq_hz", freq_hz), ("flux", flux),
                    ("vis", vis)):
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous float64 device tensor")
    if beam is not None and not (beam.is_cuda and beam.dtype == torch.float64 and beam.is_contiguous()):
        raise ValueError("beam must be a contiguous float64 device tensor")
    n_ant, n_src, n_freq = ant_enu.shape[0], src_lmn.shape[0], freq_hz.shape[0]
    sizes = (("ant_enu", ant_enu, 3 * n_ant), ("src_lmn", src_lmn, 3 * n_src), ("freq_hz", freq_hz, n_freq),
             ("flux", flux, n_freq * n_src), ("vis", vis, 2 * n_freq * n_ant * (n_ant + 1) // 2))
    if beam is not None:
        sizes += (("beam", beam, n_freq * n_src),)
    for name, t, want in sizes:
        if t.numel() != want:
            raise ValueError(f"{name} has {t.numel()} elements, expected {want}")
    return Problem(n_ant, ant_enu.data_ptr(), n_src, src_lmn.data_ptr() if n_src else None, n_freq,
                   freq_hz.data_ptr(), flux.data_ptr() if n_src else None,
                   None if beam is None else beam.data_ptr(), float(eps), int(flags))


class DevBatch:
    """A batch of device-tensor problems marshalled for fv_simulate_batch_dev."""

    def __init__(self, problems):
        self.n = len(problems)
        self.items = list(problems)  # keeps the tensors alive
        cs = [_dev_problem(q["ant_enu"], q["src_lmn"], q["freq_hz"], q["flux"], q.get("beam"), q["vis"],
                           q.get("eps", 1e-6), q.get("flags", 0)) for q in problems]
        self.arr = (Problem * self.n)(*cs)
        self.ptrs = (ctypes.c_void_p * self.n)(*[q["vis"].data_ptr() for q in problems])


class FvError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Problem(ctypes.Structure):
    _fields_ = [("n_ant", ctypes.c_int), ("ant_enu", ctypes.c_void_p),
                ("n_src", ctypes.c_int), ("src_lmn", ctypes.c_void_p),
                ("n_freq", ctypes.c_int), ("freq_hz", ctypes.c_void_p),
                ("flux", ctypes.c_void_p), ("beam", ctypes.c_void_p),
                ("eps", ctypes.c_double), ("flags", ctypes.c_uint)]


class Drift(ctypes.Structure):
    """fv_drift: drift scan with the rotation and beam on the device."""
    _fields_ = [("n_ant", ctypes.c_int), ("ant_enu", ctypes.c_void_p), ("n_src", ctypes.c_int),
                ("src_eq", ctypes.c_void_p), ("n_freq", ctypes.c_int), ("freq_hz", ctypes.c_void_p),
                ("flux", ctypes.c_void_p), ("n_time", ctypes.c_int), ("lst", ctypes.c_void_p),
                ("latitude", ctypes.c_double), ("beam_fwhm", ctypes.c_double), ("beam_nu_ref", ctypes.c_double),
                ("eps", ctypes.c_double), ("flags", ctypes.c_uint)]


class Beams(ctypes.Structure):
    """fv_beams: per-antenna beam patterns."""
    _fields_ = [("n_ant", ctypes.c_int), ("ant_enu", ctypes.c_void_p), ("n_src", ctypes.c_int),
                ("src_lmn", ctypes.c_void_p), ("n_freq", ctypes.c_int), ("freq_hz", ctypes.c_void_p),
                ("flux", ctypes.c_void_p), ("n_beam", ctypes.c_int), ("beams", ctypes.c_void_p),
                ("beam_of_ant", ctypes.c_void_p), ("eps", ctypes.c_double), ("flags", ctypes.c_uint)]


class Polar(ctypes.Structure):
    """fv_polar: polarised feed products with a shared beam."""
    _fields_ = [("n_ant", ctypes.c_int), ("ant_enu", ctypes.c_void_p), ("n_src", ctypes.c_int),
                ("src_lmn", ctypes.c_void_p), ("n_freq", ctypes.c_int), ("freq_hz", ctypes.c_void_p),
                ("stokes", ctypes.c_void_p), ("jones", ctypes.c_void_p), ("eps", ctypes.c_double),
                ("flags", ctypes.c_uint)]


class Report(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("prec_bits", ctypes.c_int), ("method", ctypes.c_int), ("w", ctypes.c_int),
                ("fold_axis", ctypes.c_int), ("n1", ctypes.c_int * 3), ("n2", ctypes.c_int * 3),
                ("t_total_ms", ctypes.c_double), ("model_bytes", ctypes.c_double), ("src_pairs", ctypes.c_double),
                ("t_stage_ms", ctypes.c_double * 8), ("stage_bytes", ctypes.c_double * 8),
                ("stage_launches", ctypes.c_int * 8), ("lattice", ctypes.c_int), ("reserved", ctypes.c_int)]

    def as_dict(self) -> dict:
        return {"dim": self.dim, "prec_bits": self.prec_bits, "method": self.method, "w": self.w,
                "fold_axis": self.fold_axis, "n1": list(self.n1), "n2": list(self.n2),
                "t_total_ms": self.t_total_ms, "model_bytes": self.model_bytes, "src_pairs": self.src_pairs,
                "t_stage_ms": list(self.t_stage_ms), "stage_bytes": list(self.stage_bytes),
                "stage_launches": list(self.stage_launches), "lattice": self.lattice}


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
                          "(hipcc for gfx950); there is no CPU fallback")
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    vp, dp = ctypes.c_void_p, P(ctypes.c_double)
    lib.fv_create.argtypes = [ctypes.c_int, ctypes.c_size_t, P(vp)]
    lib.fv_destroy.argtypes = [vp]
    lib.fv_destroy.restype = None
    lib.fv_last_error.restype = ctypes.c_char_p
    lib.fv_last_error.argtypes = []
    lib.fv_simulate.argtypes = [vp, P(Problem), vp, P(Report)]
    lib.fv_simulate_dev.argtypes = [vp, P(Problem), vp, vp, P(Report)]
    lib.fv_simulate_batch.argtypes = [vp, ctypes.c_int, P(Problem), P(vp), P(Report)]
    lib.fv_simulate_batch_dev.argtypes = [vp, ctypes.c_int, P(Problem), P(vp), vp, P(Report)]
    lib.fv_submit_dev.argtypes = [vp, P(Problem), vp, P(ctypes.c_uint64)]
    lib.fv_server_start.argtypes = [vp, ctypes.c_int]
    lib.fv_submit.argtypes = [vp, P(Problem), vp, P(ctypes.c_uint64)]
    lib.fv_wait.argtypes = [vp, ctypes.c_uint64, ctypes.c_double, P(Report)]
    lib.fv_server_stop.argtypes = [vp]
    lib.fv_debug_stages.argtypes = [vp, P(Problem), ctypes.c_int, dp, vp, ctypes.c_size_t, vp, ctypes.c_size_t]
    lib.fv_set_tune_cache.argtypes = [vp, ctypes.c_char_p]
    lib.fv_simulate_drift.argtypes = [vp, P(Drift), vp, vp, P(Report)]
    lib.fv_simulate_beams.argtypes = [vp, P(Beams), vp, vp, P(Report)]
    lib.fv_simulate_polar.argtypes = [vp, P(Polar), vp, vp, P(Report)]
    lib.fv_simulate_basis.argtypes = [vp, P(Problem), ctypes.c_int, vp, vp, P(Report)]
    lib.fv_stage_times.argtypes = [vp, dp, P(ctypes.c_int), P(ctypes.c_int)]
    lib.fv_simulate_mfma_noalloc.argtypes = [P(Problem), vp, vp]
    lib.fv_simulate_mfma_noalloc.restype = ctypes.c_int
    for name in ("fv_create", "fv_simulate", "fv_simulate_dev", "fv_simulate_batch", "fv_simulate_batch_dev",
                 "fv_submit_dev", "fv_server_start",
                 "fv_submit", "fv_wait", "fv_server_stop", "fv_set_tune_cache", "fv_debug_stages"):
        getattr(lib, name).restype = ctypes.c_int
    return lib


_lib = load_library()


def _check(status: int):
    if status != OK:
        raise FvError(status, (_lib.fv_last_error() or b"").decode())


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def simulate_mfma_noalloc(ant_enu, src_lmn, freq_hz, flux, beam, vis, eps: float = 1e-6, flags: int = 0,
                          stream=None) -> None:
    """The allocation-free matrix-core direct sum (fv_simulate_mfma_noalloc):
    torch float64 device tensors as for Context.simulate_dev, on the current
    device; FV_METHOD_MFMA is added to ``flags``.  No context is needed."""
    import torch
    for name, t in (("ant_enu", ant_enu), ("src_lmn", src_lmn), ("freq_hz", freq_hz), ("flux", flux),
                    ("vis", vis)):
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous float64 device tensor")
    if beam is not None and not (beam.is_cuda and beam.dtype == torch.float64 and beam.is_contiguous()):
        raise ValueError("beam must be a contiguous float64 device tensor")
    n_ant, n_src, n_freq = ant_enu.shape[0], src_lmn.shape[0], freq_hz.shape[0]
    sizes = (("ant_enu", ant_enu, 3 * n_ant), ("src_lmn", src_lmn, 3 * n_src), ("freq_hz", freq_hz, n_freq),
             ("flux", flux, n_freq * n_src), ("vis", vis, 2 * n_freq * n_ant * (n_ant + 1) // 2))
    if beam is not None:
        sizes += (("beam", beam, n_freq * n_src),)
    for name, t, want in sizes:
        if t.numel() != want:
            raise ValueError(f"{name} has {t.numel()} elements, expected {want}")
    st = stream if stream is not None else torch.cuda.current_stream()
    c = Problem(n_ant, ant_enu.data_ptr(), n_src, src_lmn.data_ptr() if n_src else None, n_freq,
                freq_hz.data_ptr(), flux.data_ptr() if n_src else None,
                None if beam is None else beam.data_ptr(), float(eps), int(flags) | METHOD_MFMA)
    _check(_lib.fv_simulate_mfma_noalloc(ctypes.byref(c), vis.data_ptr(), ctypes.c_void_p(st.cuda_stream)))


class HostProblem:
    """Keeps the contiguous FP64 copies alive while the C struct points at them."""

    def __init__(self, ant_enu, src_lmn, freq_hz, flux, beam=None, eps: float = 1e-6, flags: int = 0):
        self.ant = _f64(ant_enu).reshape(-1, 3)
        self.src = _f64(src_lmn).reshape(-1, 3)
        self.freq = _f64(freq_hz).reshape(-1)
        n_freq, n_src = self.freq.shape[0], self.src.shape[0]
        self.flux = _f64(flux).reshape(n_freq, n_src)
        self.beam = None if beam is None else _f64(beam).reshape(n_freq, n_src)
        self.n_pairs = self.ant.shape[0] * (self.ant.shape[0] + 1) // 2
        ptr = lambda a: None if a is None or a.size == 0 else a.ctypes.data
        self.c = Problem(self.ant.shape[0], ptr(self.ant), n_src, ptr(self.src), n_freq, ptr(self.freq),
                         ptr(self.flux), ptr(self.beam), float(eps), int(flags))

    @classmethod
    def of(cls, p, eps: Optional[float] = None, flags: int = 0) -> "HostProblem":
        """From any object with ant_enu, src_lmn, freq_hz, flux, beam, eps attributes."""
        return cls(p.ant_enu, p.src_lmn, p.freq_hz, p.flux, p.beam, p.eps if eps is None else eps, flags)


class Context:
    """One fv_ctx on a HIP device; owns its device memory and caches."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        h = ctypes.c_void_p()
        _check(_lib.fv_create(int(device), int(hbm_budget_bytes), ctypes.byref(h)))
        self._h = h
        self.last_report: Optional[dict] = None

    def close(self):
        if getattr(self, "_h", None):
            _lib.fv_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ------------------------------------------------------------------ host API
    def simulate(self, ant_enu, src_lmn, freq_hz, flux, beam=None, eps: float = 1e-6, flags: int = 0) -> np.ndarray:
        hp = HostProblem(ant_enu, src_lmn, freq_hz, flux, beam, eps, flags)
        return self.simulate_problem(hp)

    def simulate_into(self, hp: HostProblem, out: np.ndarray) -> dict:
        """fv_simulate into a caller's float64 [n_freq, n_pairs, 2] array;
        returns the report."""
        if out.dtype != np.float64 or not out.flags.c_contiguous or out.size != 2 * hp.freq.shape[0] * hp.n_pairs:
            raise ValueError("out must be a contiguous float64 [n_freq, n_pairs, 2] array")
        rep = Report()
        _check(_lib.fv_simulate(self._h, ctypes.byref(hp.c), out.ctypes.data, ctypes.byref(rep)))
        self.last_report = rep.as_dict()
        return self.last_report

    def simulate_problem(self, hp: HostProblem) -> np.ndarray:
        out = np.empty((hp.freq.shape[0], hp.n_pairs, 2), dtype=np.float64)
        rep = Report()
        _check(_lib.fv_simulate(self._h, ctypes.byref(hp.c), out.ctypes.data, ctypes.byref(rep)))
        self.last_report = rep.as_dict()
        return out[..., 0] + 1j * out[..., 1]

    # ------------------------------------------------------------------ device API
    def simulate_dev(self, ant_enu, src_lmn, freq_hz, flux, beam, vis, eps: float = 1e-6, flags: int = 0,
                     stream=None) -> dict:
        """All arguments are torch tensors on this context's device (float64,
        contiguous); ``vis`` is float64 [n_freq, n_pairs, 2].  The work is
        enqueued on ``stream`` (a torch.cuda.Stream, default: torch's current
        stream); returns the report."""
        import torch
        st = stream if stream is not None else torch.cuda.current_stream()
        c = _dev_problem(ant_enu, src_lmn, freq_hz, flux, beam, vis, eps, flags)
        rep = Report()
        _check(_lib.fv_simulate_dev(self._h, ctypes.byref(c), vis.data_ptr(), ctypes.c_void_p(st.cuda_stream),
                                    ctypes.byref(rep)))
        self.last_report = rep.as_dict()
        return self.last_report

    def simulate_drift(self, ant_enu, src_eq, freq_hz, flux, lst, latitude: float, beam_fwhm: float,
                       beam_nu_ref: float, vis, eps: float = 1e-6, flags: int = 0, stream=None) -> dict:
        """Drift scan with the front end on the device.  ``ant_enu`` [n_ant, 3],
        ``freq_hz`` [n_freq] and ``lst`` [n_time] are host arrays; ``src_eq``
        [n_src, 3] (equatorial unit vectors), ``flux`` [n_freq, n_src] and
        ``vis`` [n_time, n_freq, n_pairs, 2] are contiguous float64 torch
        tensors on this context's device.  Returns the report (summed over
        times)."""
        import torch
        ant = np.ascontiguousarray(ant_enu, dtype=np.float64).reshape(-1, 3)
        freq = np.ascontiguousarray(freq_hz, dtype=np.float64).reshape(-1)
        lsts = np.ascontiguousarray(lst, dtype=np.float64).reshape(-1)
        for name, t in (("src_eq", src_eq), ("flux", flux), ("vis", vis)):
            if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous float64 device tensor")
        n_ant, n_freq, n_time = ant.shape[0], freq.shape[0], lsts.shape[0]
        n_src = src_eq.shape[0] if src_eq.dim() == 2 else src_eq.numel() // 3
        n_pairs = n_ant * (n_ant + 1) // 2
        for name, t, want in (("src_eq", src_eq, 3 * n_src), ("flux", flux, n_freq * n_src),
                              ("vis", vis, 2 * n_time * n_freq * n_pairs)):
            if t.numel() != want:
                raise ValueError(f"{name} has {t.numel()} elements, expected {want}")
        st = stream if stream is not None else torch.cuda.current_stream()
        d = Drift(n_ant, ant.ctypes.data, n_src, src_eq.data_ptr() if n_src else None, n_freq, freq.ctypes.data,
                  flux.data_ptr() if n_src else None, n_time, lsts.ctypes.data, float(latitude), float(beam_fwhm),
                  float(beam_nu_ref), float(eps), int(flags))
        rep = Report()
        _check(_lib.fv_simulate_drift(self._h, ctypes.byref(d), vis.data_ptr(), ctypes.c_void_p(st.cuda_stream),
                                      ctypes.byref(rep)))
        self.last_report = rep.as_dict()
        return self.last_report

    def simulate_beams(self, ant_enu, src_lmn, freq_hz, flux, beams, beam_of_ant, vis, eps: float = 1e-6,
                       flags: int = 0, stream=None) -> dict:
        """Per-antenna beam patterns.  ``ant_enu``, ``src_lmn``, ``freq_hz``,
        ``flux`` [n_freq, n_src], ``beams`` [n_beam, n_freq, n_src] and ``vis``
        [n_freq, n_pairs, 2] are contiguous float64 torch tensors on this
        context's device; ``beam_of_ant`` [n_ant] is a host integer array."""
        import torch
        for name, t in (("ant_enu", ant_enu), ("src_lmn", src_lmn), ("freq_hz", freq_hz), ("flux", flux),
                        ("beams", beams), ("vis", vis)):
            if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous float64 device tensor")
        which = np.ascontiguousarray(beam_of_ant, dtype=np.int32).reshape(-1)
        n_ant, n_src, n_freq = ant_enu.shape[0], src_lmn.shape[0], freq_hz.shape[0]
        n_beam = beams.shape[0] if beams.dim() == 3 else 1
        for name, t, want in (("ant_enu", ant_enu, 3 * n_ant), ("src_lmn", src_lmn, 3 * n_src),
                              ("freq_hz", freq_hz, n_freq), ("flux", flux, n_freq * n_src),
                              ("beams", beams, n_beam * n_freq * n_src),
                              ("vis", vis, 2 * n_freq * n_ant * (n_ant + 1) // 2)):
            if t.numel() != want:
                raise ValueError(f"{name} has {t.numel()} elements, expected {want}")
        if which.shape[0] != n_ant:
            raise ValueError(f"beam_of_ant has {which.shape[0]} entries, expected {n_ant}")
        st = stream if stream is not None else torch.cuda.current_stream()
        b = Beams(n_ant, ant_enu.data_ptr(), n_src, src_lmn.data_ptr() if n_src else None, n_freq,
                  freq_hz.data_ptr(), flux.data_ptr() if n_src else None, n_beam,
                  beams.data_ptr() if n_src else None, which.ctypes.data, float(eps), int(flags))
        rep = Report()
        _check(_lib.fv_simulate_beams(self._h, ctypes.byref(b), vis.data_ptr(), ctypes.c_void_p(st.cuda_stream),
                                      ctypes.byref(rep)))
        self.last_report = rep.as_dict()
        return self.last_report

    def simulate_polar(self, ant_enu, src_lmn, freq_hz, stokes, jones, vis, eps: float = 1e-6, flags: int = 0,
                       stream=None) -> dict:
        """Polarised feed products.  ``ant_enu``, ``src_lmn``, ``freq_hz``,
        ``stokes`` [4, n_freq, n_src], ``jones`` ([n_freq, n_src, 2, 2, 2] real
        view of the complex feed response, or None for ideal feeds) and ``vis``
        [4, n_freq, n_pairs, 2] (xx, xy, yx, yy) are contiguous float64 torch
        tensors on this context's device."""
        import torch
        named = [("ant_enu", ant_enu), ("src_lmn", src_lmn), ("freq_hz", freq_hz), ("stokes", stokes), ("vis", vis)]
        if jones is not None:
            named.append(("jones", jones))
        for name, t in named:
            if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous float64 device tensor")
        n_ant, n_src, n_freq = ant_enu.shape[0], src_lmn.shape[0], freq_hz.shape[0]
        want = [("ant_enu", ant_enu, 3 * n_ant), ("src_lmn", src_lmn, 3 * n_src), ("freq_hz", freq_hz, n_freq),
                ("stokes", stokes, 4 * n_freq * n_src), ("vis", vis, 8 * n_freq * n_ant * (n_ant + 1) // 2)]
        if jones is not None:
            want.append(("jones", jones, 8 * n_freq * n_src))
        for name, t, n in want:
            if t.numel() != n:
                raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
        st = stream if stream is not None else torch.cuda.current_stream()
        q = Polar(n_ant, ant_enu.data_ptr(), n_src, src_lmn.data_ptr() if n_src else None, n_freq,
                  freq_hz.data_ptr(), stokes.data_ptr() if n_src else None,
                  None if jones is None or not n_src else jones.data_ptr(), float(eps), int(flags))
        rep = Report()
        _check(_lib.fv_simulate_polar(self._h, ctypes.byref(q), vis.data_ptr(), ctypes.c_void_p(st.cuda_stream),
                                      ctypes.byref(rep)))
        self.last_report = rep.as_dict()
        return self.last_report

    def simulate_basis(self, ant_enu, src_lmn, freq_hz, flux, beam, vis, n_basis: int, eps: float = 1e-6,
                       flags: int = 0, stream=None) -> dict:
        """Spectral-basis evaluation: arguments as for simulate_dev, plus the
        number of basis functions."""
        import torch
        for name, t in (("ant_enu", ant_enu), ("src_lmn", src_lmn), ("freq_hz", freq_hz), ("flux", flux),
                        ("vis", vis)):
            if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous float64 device tensor")
        if beam is not None and not (beam.is_cuda and beam.dtype == torch.float64 and beam.is_contiguous()):
            raise ValueError("beam must be a contiguous float64 device tensor")
        n_ant, n_src, n_freq = ant_enu.shape[0], src_lmn.shape[0], freq_hz.shape[0]
        sizes = (("ant_enu", ant_enu, 3 * n_ant), ("src_lmn", src_lmn, 3 * n_src), ("freq_hz", freq_hz, n_freq),
                 ("flux", flux, n_freq * n_src), ("vis", vis, 2 * n_freq * n_ant * (n_ant + 1) // 2))
        if beam is not None:
            sizes += (("beam", beam, n_freq * n_src),)
        for name, t, want in sizes:
            if t.numel() != want:
                raise ValueError(f"{name} has {t.numel()} elements, expected {want}")
        st = stream if stream is not None else torch.cuda.current_stream()
        c = Problem(n_ant, ant_enu.data_ptr(), n_src, src_lmn.data_ptr() if n_src else None, n_freq,
                    freq_hz.data_ptr(), flux.data_ptr() if n_src else None,
                    None if beam is None else beam.data_ptr(), float(eps), int(flags))
        rep = Report()
        _check(_lib.fv_simulate_basis(self._h, ctypes.byref(c), int(n_basis), vis.data_ptr(),
                                      ctypes.c_void_p(st.cuda_stream), ctypes.byref(rep)))
        self.last_report = rep.as_dict()
        return self.last_report

    def stage_times(self) -> dict:
        """Summed stage event times of the TIMING_ACCUM calls since the last
        query (waits for them): {"ms": [...], "launches": [...], "calls": n}."""
        ms = np.zeros(len(STAGES), dtype=np.float64)
        launches = (ctypes.c_int * len(STAGES))()
        calls = ctypes.c_int(0)
        _check(_lib.fv_stage_times(self._h, ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), launches,
                                   ctypes.byref(calls)))
        return {"ms": ms.tolist(), "launches": list(launches), "calls": calls.value}

    def set_tune_cache(self, path: Optional[str]):
        """Autotuner cache file (JSON); None keeps the cache in memory only."""
        _check(_lib.fv_set_tune_cache(self._h, None if path is None else str(path).encode()))

    # ------------------------------------------------------------------ batch API
    def simulate_batch(self, problems: Sequence[HostProblem]) -> list:
        n = len(problems)
        arr = (Problem * n)(*[p.c for p in problems])
        outs = [np.empty((p.freq.shape[0], p.n_pairs, 2), dtype=np.float64) for p in problems]
        ptrs = (ctypes.c_void_p * n)(*[o.ctypes.data for o in outs])
        rep = Report()
        _check(_lib.fv_simulate_batch(self._h, n, arr, ptrs, ctypes.byref(rep)))
        self.last_report = rep.as_dict()
        return [o[..., 0] + 1j * o[..., 1] for o in outs]

    def prepare_batch_dev(self, problems: Sequence[dict]) -> "DevBatch":
        """Checks and marshals a batch of problems whose arrays are torch
        device tensors: each item is a dict with the keys of simulate_dev
        (ant_enu, src_lmn, freq_hz, flux, beam, vis, eps, flags).  The result
        can be run many times (run_batch_dev); it keeps the tensors alive."""
        return DevBatch(problems)

    def run_batch_dev(self, batch: "DevBatch", stream=None) -> dict:
        """Enqueues a prepared batch on ``stream`` (default: torch's current
        stream); returns the batch report."""
        import torch
        st = stream if stream is not None else torch.cuda.current_stream()
        rep = Report()
        _check(_lib.fv_simulate_batch_dev(self._h, batch.n, batch.arr, batch.ptrs, ctypes.c_void_p(st.cuda_stream),
                                          ctypes.byref(rep)))
        self.last_report = rep.as_dict()
        return self.last_report

    def simulate_batch_dev(self, problems: Sequence[dict], stream=None) -> dict:
        """prepare_batch_dev and run_batch_dev in one call."""
        return self.run_batch_dev(self.prepare_batch_dev(problems), stream)

    # ------------------------------------------------------------------ serving
    def server_start(self, max_slots: int = 4):
        _check(_lib.fv_server_start(self._h, int(max_slots)))

    def submit_dev(self, ant_enu, src_lmn, freq_hz, flux, beam, vis, eps: float = 1e-6, flags: int = 0) -> int:
        """Submits a request whose arrays are torch device tensors (as for
        simulate_dev); the tensors must stay alive until wait() returns."""
        c = _dev_problem(ant_enu, src_lmn, freq_hz, flux, beam, vis, eps, flags)
        t = ctypes.c_uint64()
        _check(_lib.fv_submit_dev(self._h, ctypes.byref(c), vis.data_ptr(), ctypes.byref(t)))
        return int(t.value)

    def submit(self, hp: HostProblem, out: np.ndarray) -> int:
        t = ctypes.c_uint64()
        _check(_lib.fv_submit(self._h, ctypes.byref(hp.c), out.ctypes.data, ctypes.byref(t)))
        return int(t.value)

    def wait(self, ticket: int, timeout_s: float = -1.0):
        rep = Report()
        st = _lib.fv_wait(self._h, ctypes.c_uint64(ticket), float(timeout_s), ctypes.byref(rep))
        return st, rep.as_dict()

    def server_stop(self):
        _check(_lib.fv_server_stop(self._h))

    # ------------------------------------------------------------------ diagnostics
    def debug_stages(self, hp: HostProblem, f: int = 0):
        """Plan scalars, the deconvolved spreading grid and the pruned FFT
        output of frequency ``f`` (complex128, axes ordered z, y, x)."""
        plan = np.zeros(31, dtype=np.float64)
        _check(_lib.fv_debug_stages(self._h, ctypes.byref(hp.c), int(f),
                                    plan.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None, 0, None, 0))
        n1 = plan[3:6].astype(int)
        M = plan[9:12].astype(int)
        spread = np.empty((int(np.prod(n1)), 2))
        fft = np.empty((int(np.prod(M)), 2))
        _check(_lib.fv_debug_stages(self._h, ctypes.byref(hp.c), int(f),
                                    plan.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), spread.ctypes.data,
                                    spread.shape[0], fft.ctypes.data, fft.shape[0]))
        dim = int(plan[0])
        info = {"dim": dim, "w": int(plan[1]), "fold_axis": int(plan[2]), "n1": n1[:dim].tolist(),
                "n2": plan[6:9].astype(int)[:dim].tolist(), "M": M[:dim].tolist(),
                "P": plan[12:15].astype(int)[:dim].tolist(), "s_c": plan[15:18][:dim].copy(),
                "S": plan[18:21][:dim].copy(), "b_c": plan[21:24][:dim].copy(), "B": plan[24:27][:dim].copy(),
                "prec_bits": int(plan[27]), "X": plan[28:31][:dim].copy()}
        shape1 = tuple(int(v) for v in n1[:dim][::-1])
        shapeM = tuple(int(v) for v in M[:dim][::-1])
        return info, (spread[:, 0] + 1j * spread[:, 1]).reshape(shape1), (fft[:, 0] + 1j * fft[:, 1]).reshape(shapeM)
