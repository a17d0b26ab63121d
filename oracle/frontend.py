"""Drift-scan front end in FP64 numpy: equatorial directions to local
East-North-Up at each local sidereal time, and an analytic Gaussian power beam.

TEST INFRASTRUCTURE ONLY (oracle side; the product never imports this).

Section 2.3 of the paper (coordinate rotation): between astrometric
pre-corrections, a rigid rotation that depends only on the local sidereal time
and the latitude takes pre-corrected equatorial positions to the horizontal
(ENU) frame at each time step.  Written here in the hour-angle form of
spherical astronomy, from right ascension alpha and declination delta:

    H = LST - alpha
    E = -cos(delta) sin(H)
    N =  cos(lat) sin(delta) - sin(lat) cos(delta) cos(H)
    U =  sin(lat) sin(delta) + cos(lat) cos(delta) cos(H)

Section 2.4 (beams): analytic beam models are evaluated in closed form at the
source positions.  The model here is a Gaussian power beam in zenith angle
theta = arccos(U) whose full width at half maximum scales as 1/nu,

    A(theta, nu) = 2^(-(2 theta / F(nu))^2),   F(nu) = F_ref nu_ref / nu,

zero at and below the horizon (U <= 0); F_ref = 0 means a unit beam above
the horizon.

Equatorial inputs are unit vectors (x towards alpha = 0 on the equator,
z towards the north celestial pole).
"""
from __future__ import annotations

import numpy as np

from . import direct_vis


def radec(src_eq: np.ndarray):
    """(alpha, delta) of equatorial unit vectors [n, 3]."""
    x, y, z = src_eq[:, 0], src_eq[:, 1], src_eq[:, 2]
    return np.arctan2(y, x), np.arcsin(np.clip(z, -1.0, 1.0))


def enu(alpha: np.ndarray, delta: np.ndarray, lst: float, lat: float) -> np.ndarray:
    """[n, 3] local (E, N, U) directions at sidereal time lst (radians)."""
    H = lst - alpha
    e = -np.cos(delta) * np.sin(H)
    n = np.cos(lat) * np.sin(delta) - np.sin(lat) * np.cos(delta) * np.cos(H)
    u = np.sin(lat) * np.sin(delta) + np.cos(lat) * np.cos(delta) * np.cos(H)
    return np.stack([e, n, u], axis=1)


def gaussian_beam(dirs_enu: np.ndarray, freq_hz: np.ndarray, fwhm_ref: float, nu_ref: float) -> np.ndarray:
    """[n_freq, n_src] power beam at the given ENU directions."""
    u = dirs_enu[:, 2]
    out = np.zeros((len(freq_hz), dirs_enu.shape[0]))
    up = u > 0.0
    if fwhm_ref == 0.0:
        out[:, up] = 1.0
        return out
    theta = np.arccos(np.clip(u[up], -1.0, 1.0))
    for f, nu in enumerate(freq_hz):
        F = fwhm_ref * nu_ref / nu
        out[f, up] = 2.0 ** (-(2.0 * theta / F) ** 2)
    return out


def drift_vis(ant_enu, src_eq, freq_hz, flux, lst, lat, fwhm_ref, nu_ref, pairs=None) -> np.ndarray:
    """V[t, f, pair]: the exact sum of every snapshot of a drift scan (sources
    rotated to ENU at each LST, strengths flux times the beam)."""
    alpha, delta = radec(np.asarray(src_eq, dtype=np.float64))
    out = []
    for t in lst:
        d = enu(alpha, delta, float(t), float(lat))
        b = gaussian_beam(d, np.asarray(freq_hz), fwhm_ref, nu_ref)
        out.append(direct_vis(ant_enu, d, freq_hz, flux, b, pairs=pairs))
    return np.stack(out)
