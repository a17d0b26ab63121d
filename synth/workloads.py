"""Seeded workload generators (inputs only; no visibility arithmetic).

Every generator draws from ``numpy.random.Generator(PCG64(SEED_BASE + k))`` so
that the oracle side and the GPU side see bit-identical inputs.

Conventions shared with the library's C ABI:
  * antenna positions ``ant_enu[n_ant][3]`` in metres (East, North, Up);
  * source directions ``src_lmn[n_src][3]`` unit vectors (l=E, m=N, n=Up);
  * ``flux[n_freq][n_src]`` Stokes-I in Jy and ``beam[n_freq][n_src]`` the
    real beam weight applied as-is (the source strength is beam*flux);
  * output pairs are (i <= j) in row-major order, baseline b_ij = x_i - x_j.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

C_LIGHT = 299792458.0
SEED_BASE = 2506021300
HERA_SPACING = 14.6
HERA_LAT_DEG = -30.72


@dataclasses.dataclass
class Problem:
    name: str
    ant_enu: np.ndarray            # [n_ant, 3] float64
    src_lmn: np.ndarray            # [n_src, 3] float64
    freq_hz: np.ndarray            # [n_freq] float64
    flux: np.ndarray               # [n_freq, n_src] float64
    beam: Optional[np.ndarray]     # [n_freq, n_src] float64 or None (=1)
    eps: float

    @property
    def n_ant(self) -> int:
        return int(self.ant_enu.shape[0])

    @property
    def n_src(self) -> int:
        return int(self.src_lmn.shape[0])

    @property
    def n_freq(self) -> int:
        return int(self.freq_hz.shape[0])

    @property
    def n_pairs(self) -> int:
        return self.n_ant * (self.n_ant + 1) // 2

    @property
    def n_src_pairs(self) -> int:
        """Source x baseline pairs of one call: n_src * n_pairs * n_freq."""
        return self.n_src * self.n_pairs * self.n_freq

    def strengths(self) -> np.ndarray:
        return self.flux if self.beam is None else self.flux * self.beam


# --------------------------------------------------------------------------
# arrays
# --------------------------------------------------------------------------
def hex_array(n_ant: int, spacing: float = HERA_SPACING) -> np.ndarray:
    """First ``n_ant`` points of a centred triangular lattice (basis (s,0) and
    (s/2, s*sqrt(3)/2), z=0), ordered by radius (rounded to 1e-9 m) then by
    azimuth atan2(y, x)."""
    R = 0
    while 3 * R * (R + 1) + 1 < n_ant:
        R += 1
    pts = []
    for a in range(-R, R + 1):
        for b in range(-R, R + 1):
            if abs(a + b) <= R:
                pts.append((a * spacing + b * spacing / 2.0, b * spacing * math.sqrt(3.0) / 2.0))
    p = np.asarray(pts, dtype=np.float64)
    r = np.round(np.hypot(p[:, 0], p[:, 1]), 9)
    ang = np.arctan2(p[:, 1], p[:, 0])
    order = np.lexsort((ang, r))
    p = p[order][:n_ant]
    return np.column_stack([p, np.zeros(len(p))])


def disk_array(rng: np.random.Generator, n_ant: int, radius: float, zhalf: float) -> np.ndarray:
    """Antennas uniform in a disk of ``radius`` metres with heights U(-zhalf, zhalf)."""
    r = radius * np.sqrt(rng.random(n_ant))
    ph = 2 * np.pi * rng.random(n_ant)
    z = rng.uniform(-zhalf, zhalf, n_ant)
    return np.column_stack([r * np.cos(ph), r * np.sin(ph), z])


# --------------------------------------------------------------------------
# skies
# --------------------------------------------------------------------------
def unit_disk_lm(rng: np.random.Generator, n: int) -> np.ndarray:
    """(l, m) uniform over the unit disk, n = sqrt(1 - l^2 - m^2) (above horizon)."""
    r = np.sqrt(rng.random(n))
    ph = 2 * np.pi * rng.random(n)
    l, m = r * np.cos(ph), r * np.sin(ph)
    return np.column_stack([l, m, np.sqrt(np.maximum(0.0, 1 - l * l - m * m))])


def isotropic_hemisphere(rng: np.random.Generator, n: int) -> np.ndarray:
    """Directions isotropic over the upper hemisphere: n ~ U(0, 1], azimuth U(0, 2pi)."""
    up = 1.0 - rng.random(n)
    ph = 2 * np.pi * rng.random(n)
    rho = np.sqrt(np.maximum(0.0, 1 - up * up))
    return np.column_stack([rho * np.cos(ph), rho * np.sin(ph), up])


def fibonacci_sphere(npix: int) -> np.ndarray:
    """Equal-area Fibonacci lattice of ``npix`` unit vectors (HEALPix-like pixelisation)."""
    i = np.arange(npix, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / npix
    ga = math.pi * (3.0 - math.sqrt(5.0))
    ph = np.mod(i * ga, 2 * np.pi)
    rho = np.sqrt(np.maximum(0.0, 1 - z * z))
    return np.column_stack([rho * np.cos(ph), rho * np.sin(ph), z])


def powerlaw_fluxes(rng: np.random.Generator, n: int, smin: float = 0.01, smax: float = 100.0,
                    slope: float = -1.8) -> np.ndarray:
    """Fluxes with dN/dS proportional to S**slope on [smin, smax] (inverse CDF)."""
    a = slope + 1.0
    u = rng.random(n)
    return (smin ** a + u * (smax ** a - smin ** a)) ** (1.0 / a)


def gaussian_beam(src_lmn: np.ndarray, freq_hz: np.ndarray, fwhm150_deg: float = 10.0) -> np.ndarray:
    """Gaussian power beam exp(-theta^2 / 2 sigma_b^2), theta = arccos(n), with
    FWHM = fwhm150 * (150 MHz / nu); zero at and below the horizon.  [n_freq, n_src]."""
    n = np.clip(src_lmn[:, 2], -1.0, 1.0)
    theta = np.arccos(n)
    fwhm = np.radians(fwhm150_deg) * (150e6 / np.asarray(freq_hz))
    sig = fwhm / math.sqrt(8 * math.log(2))
    b = np.exp(-theta[None, :] ** 2 / (2 * sig[:, None] ** 2))
    b[:, n <= 0] = 0.0
    return b


def equatorial_to_enu(ra: np.ndarray, dec: np.ndarray, lst: float, lat: float) -> np.ndarray:
    """Rigid rotation of equatorial directions to local (E, N, Up) at local
    sidereal time ``lst`` and latitude ``lat`` (radians), hour angle H = lst - ra."""
    H = lst - ra
    cd, sd = np.cos(dec), np.sin(dec)
    cl, sl = math.cos(lat), math.sin(lat)
    l = -cd * np.sin(H)
    m = cl * sd - sl * cd * np.cos(H)
    n = sl * sd + cl * cd * np.cos(H)
    return np.column_stack([l, m, n])


def _spectral(rng, s150, freq_hz, mean=-0.8, sd=0.2):
    alpha = rng.normal(mean, sd, s150.shape[0])
    return s150[None, :] * (np.asarray(freq_hz)[:, None] / 150e6) ** alpha[None, :]


def _renorm(lmn: np.ndarray) -> np.ndarray:
    return lmn / np.linalg.norm(lmn, axis=1, keepdims=True)


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------
def config1() -> Problem:
    """37-antenna hex, 100 sources uniform over the unit disk, fluxes
    log-uniform 0.1-10 Jy, Gaussian beam FWHM 10 deg at 150 MHz, one
    frequency (150 MHz), eps 1e-10 (FP64)."""
    rng = np.random.default_rng(np.random.PCG64(SEED_BASE + 1))
    ant = hex_array(37)
    src = _renorm(unit_disk_lm(rng, 100))
    freq = np.array([150e6])
    flux = (10.0 ** rng.uniform(-1.0, 1.0, 100))[None, :]
    return Problem("hex37_src100_f1_eps1e-10", ant, src, freq, flux, gaussian_beam(src, freq), 1e-10)


def config2(n_src: int = 100_000, n_freq: int = 64, n_ant: int = 350) -> Problem:
    """350-antenna hex, 1e5 isotropic point sources, power-law counts
    (0.01-100 Jy, slope -1.8), spectral index N(-0.8, 0.2), Gaussian beam
    scaled with frequency, 64 frequencies in 100-200 MHz, eps 1e-6 (FP32 grids)."""
    rng = np.random.default_rng(np.random.PCG64(SEED_BASE + 2))
    ant = hex_array(n_ant)
    src = _renorm(isotropic_hemisphere(rng, n_src))
    freq = np.linspace(100e6, 200e6, n_freq)
    flux = _spectral(rng, powerlaw_fluxes(rng, n_src), freq)
    return Problem(f"hex{n_ant}_src{n_src}_f{n_freq}_eps1e-6", ant, src, freq, flux,
                   gaussian_beam(src, freq), 1e-6)


def config3(n_ant: int = 1000, npix: int = 786_432, n_freq: int = 16, radius: float = 500.0) -> Problem:
    """1000 antennas uniform in a disk of radius 500 m with heights +-5 m (3-D),
    diffuse sky of npix equal-area pixels (horizon-cut), Gaussian-random
    amplitudes times the pixel solid angle with spectrum (nu/160 MHz)^-2.5,
    beam 1 above the horizon, 16 frequencies in 150-170 MHz, eps 1e-6."""
    rng = np.random.default_rng(np.random.PCG64(SEED_BASE + 3))
    ant = disk_array(rng, n_ant, radius, 5.0)
    pix = fibonacci_sphere(npix)
    src = _renorm(pix[pix[:, 2] > 0])
    freq = np.linspace(150e6, 170e6, n_freq)
    amp = rng.normal(0.0, 1.0, src.shape[0]) * (4 * math.pi / npix)
    flux = amp[None, :] * (freq[:, None] / 160e6) ** -2.5
    return Problem(f"disk{n_ant}_pix{npix}_f{n_freq}_3d_eps1e-6", ant, src, freq, flux, None, 1e-6)


def config4(n_lst: int = 24, n_freq: int = 43, n_cap: int = 100_000, n_iso: int = 2000,
            n_ant: int = 127) -> List[Problem]:
    """127-antenna hex observed at ``n_lst`` hourly LSTs x ``n_freq`` frequencies
    (100-200 MHz): a 25-degree cap of power-law sources centred at (RA 0,
    Dec -30.72 deg) plus isotropic sources, rotated to ENU per LST and cut at
    the horizon, so per-snapshot source counts vary by two orders of
    magnitude.  One Problem per LST (all frequencies share its sources)."""
    rng = np.random.default_rng(np.random.PCG64(SEED_BASE + 4))
    lat = math.radians(HERA_LAT_DEG)
    # cap around (ra0, dec0)
    ra0, dec0 = 0.0, lat
    c = np.array([math.cos(dec0) * math.cos(ra0), math.cos(dec0) * math.sin(ra0), math.sin(dec0)])
    e1 = np.cross([0.0, 0.0, 1.0], c); e1 /= np.linalg.norm(e1)
    e2 = np.cross(c, e1)
    ct = rng.uniform(math.cos(math.radians(25.0)), 1.0, n_cap)
    st = np.sqrt(1 - ct * ct)
    psi = 2 * np.pi * rng.random(n_cap)
    p = ct[:, None] * c + st[:, None] * (np.cos(psi)[:, None] * e1 + np.sin(psi)[:, None] * e2)
    ra = np.concatenate([np.arctan2(p[:, 1], p[:, 0]), 2 * np.pi * rng.random(n_iso)])
    dec = np.concatenate([np.arcsin(np.clip(p[:, 2], -1, 1)), np.arcsin(rng.uniform(-1, 1, n_iso))])
    s150 = powerlaw_fluxes(rng, n_cap + n_iso)
    alpha = rng.normal(-0.8, 0.2, n_cap + n_iso)
    freq = np.linspace(100e6, 200e6, n_freq)
    ant = hex_array(n_ant)
    out = []
    for t in range(n_lst):
        lst = 2 * np.pi * t / n_lst
        lmn = equatorial_to_enu(ra, dec, lst, lat)
        keep = lmn[:, 2] > 0
        src = _renorm(lmn[keep])
        flux = s150[keep][None, :] * (freq[:, None] / 150e6) ** alpha[keep][None, :]
        out.append(Problem(f"hex{n_ant}_lst{t}_src{src.shape[0]}_f{n_freq}", ant, src, freq, flux,
                           gaussian_beam(src, freq), 1e-6))
    return out


@dataclasses.dataclass
class DriftScan:
    """A drift scan: the array, an equatorial sky (unit vectors, x towards RA 0
    on the equator, z to the north pole), fluxes per frequency, sidereal times,
    the latitude and a Gaussian power beam's FWHM at a reference frequency."""
    name: str
    ant_enu: np.ndarray     # [n_ant, 3]
    src_eq: np.ndarray      # [n_src, 3]
    freq_hz: np.ndarray     # [n_freq]
    flux: np.ndarray        # [n_freq, n_src]
    lst: np.ndarray         # [n_time] radians
    latitude: float         # radians
    beam_fwhm: float        # radians at beam_nu_ref
    beam_nu_ref: float
    eps: float

    @property
    def n_pairs(self) -> int:
        n = self.ant_enu.shape[0]
        return n * (n + 1) // 2


def _eq_unit(ra: np.ndarray, dec: np.ndarray) -> np.ndarray:
    return np.stack([np.cos(dec) * np.cos(ra), np.cos(dec) * np.sin(ra), np.sin(dec)], axis=1)


def config4_drift(n_lst: int = 24, n_freq: int = 43, n_cap: int = 100_000, n_iso: int = 2000,
                  n_ant: int = 127) -> DriftScan:
    """The sky of config4 (25-degree power-law cap at Dec -30.72 deg plus
    isotropic sources, spectral index N(-0.8, 0.2), 100-200 MHz) left in
    equatorial form with the hourly sidereal times, for the device front end;
    beam FWHM 10 degrees at 150 MHz."""
    rng = np.random.default_rng(np.random.PCG64(SEED_BASE + 40))
    lat = math.radians(HERA_LAT_DEG)
    c = _eq_unit(np.array([0.0]), np.array([lat]))[0]
    e1 = np.cross([0.0, 0.0, 1.0], c); e1 /= np.linalg.norm(e1)
    e2 = np.cross(c, e1)
    ct = rng.uniform(math.cos(math.radians(25.0)), 1.0, n_cap)
    st = np.sqrt(1 - ct * ct)
    psi = 2 * np.pi * rng.random(n_cap)
    cap = ct[:, None] * c + st[:, None] * (np.cos(psi)[:, None] * e1 + np.sin(psi)[:, None] * e2)
    iso = _eq_unit(2 * np.pi * rng.random(n_iso), np.arcsin(rng.uniform(-1, 1, n_iso)))
    src = _renorm(np.concatenate([cap, iso]))
    s150 = powerlaw_fluxes(rng, n_cap + n_iso)
    alpha = rng.normal(-0.8, 0.2, n_cap + n_iso)
    freq = np.linspace(100e6, 200e6, n_freq)
    flux = s150[None, :] * (freq[:, None] / 150e6) ** alpha[None, :]
    lst = 2 * np.pi * np.arange(n_lst) / n_lst
    return DriftScan(f"hex{n_ant}_drift{n_lst}x{n_freq}_src{n_cap + n_iso}", hex_array(n_ant), src, freq, flux, lst,
                     lat, math.radians(10.0), 150e6, 1e-6)


def small_drift(seed: int, n_ant: int = 19, n_src: int = 300, n_freq: int = 2, n_time: int = 3,
                hex_layout: bool = True, three_d: bool = False, eps: float = 1e-6) -> DriftScan:
    """A small drift scan for tests: isotropic equatorial sky, power-law fluxes."""
    rng = np.random.default_rng(np.random.PCG64(SEED_BASE + 500 + seed))
    ant = hex_array(n_ant) if hex_layout else disk_array(rng, n_ant, 60.0, 2.0 if three_d else 0.0)
    src = _renorm(_eq_unit(2 * np.pi * rng.random(n_src), np.arcsin(rng.uniform(-1, 1, n_src)))) if n_src else \
        np.zeros((0, 3))
    freq = np.linspace(110e6, 190e6, n_freq)
    flux = _spectral(rng, powerlaw_fluxes(rng, n_src), freq) if n_src else np.zeros((n_freq, 0))
    lst = np.sort(rng.uniform(0, 2 * np.pi, n_time))
    return DriftScan(f"drift{seed}", ant, src, freq, flux, lst, math.radians(HERA_LAT_DEG), math.radians(12.0),
                     150e6, eps)


@dataclasses.dataclass
class Request:
    rid: int
    arrival_s: float
    n_ant: int
    n_src: int
    n_freq: int
    eps: float
    seed: int

    def materialize(self) -> Problem:
        rng = np.random.default_rng(np.random.PCG64(self.seed))
        ant = hex_array(self.n_ant)
        src = _renorm(isotropic_hemisphere(rng, self.n_src))
        freq = np.linspace(100e6, 200e6, self.n_freq) if self.n_freq > 1 else np.array([150e6])
        flux = _spectral(rng, powerlaw_fluxes(rng, self.n_src), freq)
        return Problem(f"req{self.rid}", ant, src, freq, flux, gaussian_beam(src, freq), self.eps)


    def materialize_torch(self, device):
        """The same request drawn on a torch device (for large serving runs):
        the distributions of materialize(), from a torch generator seeded with
        the request's seed, so the values differ from materialize()'s.
        Returns (ant, src, freq, flux, beam) float64 tensors."""
        import torch
        g = torch.Generator(device=device)
        g.manual_seed(self.seed)
        f64 = dict(dtype=torch.float64, device=device)
        ant = torch.from_numpy(hex_array(self.n_ant)).to(device)
        up = 1.0 - torch.rand(self.n_src, generator=g, **f64)
        ph = 2 * math.pi * torch.rand(self.n_src, generator=g, **f64)
        rho = torch.sqrt(torch.clamp(1 - up * up, min=0.0))
        src = torch.stack([rho * torch.cos(ph), rho * torch.sin(ph), up], dim=1)
        src = src / torch.linalg.norm(src, dim=1, keepdim=True)
        freq = (torch.linspace(100e6, 200e6, self.n_freq, **f64) if self.n_freq > 1
                else torch.full((1,), 150e6, **f64))
        a, smin, smax = -0.8, 0.01, 100.0  # slope -1.8 power law by inverse CDF
        u = torch.rand(self.n_src, generator=g, **f64)
        s150 = (smin ** a + u * (smax ** a - smin ** a)) ** (1.0 / a)
        alpha = -0.8 + 0.2 * torch.randn(self.n_src, generator=g, **f64)
        flux = s150[None, :] * (freq[:, None] / 150e6) ** alpha[None, :]
        theta = torch.arccos(torch.clamp(src[:, 2], -1.0, 1.0))
        sig = math.radians(10.0) * (150e6 / freq) / math.sqrt(8 * math.log(2))
        beam = torch.exp(-theta[None, :] ** 2 / (2 * sig[:, None] ** 2))
        beam[:, src[:, 2] <= 0] = 0.0
        return ant, src.contiguous(), freq, flux.contiguous(), beam.contiguous()


SERVING_ARRAYS = (37, 61, 91, 127, 169, 217, 271, 331, 350)


def config5_requests(n_req: int = 2000, rate_hz: float = 100.0, src_lo: float = 1e3, src_hi: float = 1e6,
                     max_freq: int = 64, eps_choices=(1e-4, 1e-6, 1e-10)) -> List[Request]:
    """Poisson arrivals (seeded) of requests mixing hex arrays of 37-350
    antennas, log-uniform 1e3-1e6 sources, 1-64 frequencies and eps in
    {1e-4, 1e-6, 1e-10}."""
    rng = np.random.default_rng(np.random.PCG64(SEED_BASE + 5))
    gaps = rng.exponential(1.0 / rate_hz, n_req)
    t = np.cumsum(gaps) - gaps[0]
    reqs = []
    for k in range(n_req):
        reqs.append(Request(
            rid=k, arrival_s=float(t[k]),
            n_ant=int(rng.choice(SERVING_ARRAYS)),
            n_src=int(round(10 ** rng.uniform(math.log10(src_lo), math.log10(src_hi)))),
            n_freq=int(rng.integers(1, max_freq + 1)),
            eps=float(rng.choice(eps_choices)),
            seed=SEED_BASE + 1000 + k))
    return reqs


def small_problem(seed: int, n_ant: int = 12, n_src: int = 40, n_freq: int = 2, eps: float = 1e-6,
                  three_d: bool = False, hex_layout: bool = False, beam: bool = True,
                  sky: str = "hemisphere", f_lo: float = 100e6, f_hi: float = 200e6,
                  radius: float = 60.0, zhalf: float = 2.0) -> Problem:
    """A small random problem for tests: a random (or hex) array, isotropic
    (or unit-disk) sources, power-law fluxes, optional Gaussian beam."""
    rng = np.random.default_rng(np.random.PCG64(SEED_BASE + 100 + seed))
    if hex_layout:
        ant = hex_array(n_ant)
    else:
        ant = disk_array(rng, n_ant, radius, zhalf if three_d else 0.0)
    if sky == "disk":
        src = unit_disk_lm(rng, n_src)
    else:
        src = isotropic_hemisphere(rng, n_src)
    src = _renorm(src) if n_src else src.reshape(0, 3)
    freq = np.linspace(f_lo, f_hi, n_freq) if n_freq > 1 else np.array([0.5 * (f_lo + f_hi)])
    flux = _spectral(rng, powerlaw_fluxes(rng, n_src), freq)
    bm = gaussian_beam(src, freq, 30.0) if beam else None
    return Problem(f"small{seed}", ant, src, freq, flux, bm, eps)


def subset_pairs(n_ant: int, k: int, seed: int) -> np.ndarray:
    """Seeded, sorted subset of ``k`` pair indices of the (i<=j) row-major layout."""
    n = n_ant * (n_ant + 1) // 2
    rng = np.random.default_rng(np.random.PCG64(SEED_BASE + 9000 + seed))
    if k >= n:
        return np.arange(n, dtype=np.int64)
    return np.sort(rng.choice(n, k, replace=False)).astype(np.int64)
