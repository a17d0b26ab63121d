"""Step-by-step FP64 type-1 path for arrays whose antennas lie on a lattice.

TEST INFRASTRUCTURE ONLY (oracle side; the product never imports this).

Section 2.2.1 of the paper (evaluating the measurement equation for gridded
arrays): when every physical baseline is an integer combination of lattice
vectors, b = A k with A = [a1 a2] and k integer, the phase is
b.s = k.(A^T s).  The visibilities are then a type-1 transform from the
non-uniform points A^T s (scaled by nu/c, in turns) onto the uniform integer
modes k.  The paper's map L, with L b_phys = b_gridded, is A^-1, and its
(L^T)^-1 s is A^T s.  Since k is integer, only the fractional part of each
point matters.

Lattice detection follows the paper's description of it: find a common
fundamental spacing of the baselines within a tolerance, build the lattice
vectors, else fall back to type 3.  Here the candidate basis is the shortest
baseline and the shortest one not parallel to it, Gauss-reduced.  Every
antenna offset must be an integer combination of the basis within `tol`
metres.

Type-1 steps (the published algorithm the paper cites), per frequency, with
sigma = 2, beta = 2.3 w and the paper's width rule w = ceil(log10(1/eps)) + 1
(one kernel application, unlike type 3):
  u_s = (nu / c) A^T s (turns), x_s = 2 pi frac(u_s) in [0, 2 pi)^2;
  N_a = 2 K_a + 1 modes per axis, fine periodic grid n_a = smallest even
  {2,3,5}-smooth size >= max(sigma N_a, 2 w), h_a = 2 pi / n_a,
  alpha_a = w h_a / 2;
  spread   b_l = sum_s c_s prod_a phi((x_s,a - l_a h_a) / alpha_a), periodic in l;
  transform B_k = sum_l b_l exp(-i k . l h);
  correct  f_k = prod_a [h_a / (alpha_a phihat(alpha_a k_a))] B_k;
and V(i, j) = f at k = k_i - k_j.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional

import numpy as np

from .es_kernel import es_beta, es_phi, es_phihat
from .type3 import C_LIGHT, SIGMA, next_smooth_even


@dataclass
class Lattice:
    A: np.ndarray      # [2, 2], columns are the lattice vectors (metres, East/North)
    k: np.ndarray      # [n_ant, 2] integer lattice coordinates of each antenna (antenna 0 at 0)
    K: np.ndarray      # [2] largest |k_i - k_j| per axis


def find_lattice(ant: np.ndarray, tol: float) -> Optional[Lattice]:
    """Lattice of the antennas' East/North positions, or None."""
    x = np.asarray(ant, dtype=np.float64)[:, :2]
    n = x.shape[0]
    if n < 2:
        return None
    d = (x[:, None, :] - x[None, :, :]).reshape(-1, 2)
    ln = np.hypot(d[:, 0], d[:, 1])
    keep = ln > tol
    if not keep.any():
        return None
    d, ln = d[keep], ln[keep]
    order = np.argsort(ln, kind="stable")
    b1 = d[order[0]]
    cross = np.abs(b1[0] * d[:, 1] - b1[1] * d[:, 0])
    ok = cross > 1e-6 * np.linalg.norm(b1) * ln
    if not ok.any():
        return None  # collinear
    b2 = d[order[np.argmax(ok[order])]]
    # Gauss (Lagrange) reduction of the pair
    while True:
        if np.dot(b2, b2) < np.dot(b1, b1):
            b1, b2 = b2, b1
        mu = round(float(np.dot(b1, b2) / np.dot(b1, b1)))
        if mu == 0:
            break
        b2 = b2 - mu * b1
    A = np.column_stack([b1, b2])
    kr = np.linalg.solve(A, (x - x[0]).T).T
    k = np.rint(kr)
    if np.abs(k @ A.T - (x - x[0])).max() > tol:
        return None
    k = k.astype(np.int64)
    K = k.max(0) - k.min(0)
    return Lattice(A, k, K)


def lattice_tolerance(eps: float, freq_hz: np.ndarray) -> float:
    """Position tolerance (metres) that keeps the phase error below eps / 10."""
    return eps * C_LIGHT / (20.0 * math.pi * float(np.max(freq_hz)))


def kernel_width_type1(eps: float) -> int:
    """The paper's rule w = ceil(log10(1/eps)) + 1 (section 2.2), at least 3.
    Type 1 applies the kernel once (one spread, no interpolation), so the rule
    holds the error below eps without the extra point type 3 needs."""
    return max(3, int(math.ceil(-math.log10(eps) - 1e-9)) + 1)


def grid_sizes(lat: Lattice, w: int) -> np.ndarray:
    N = 2 * lat.K + 1
    return np.array([next_smooth_even(max(int(math.ceil(SIGMA * N[a])), 2 * w)) for a in range(2)])


def spread(lat: Lattice, nf: np.ndarray, w: int, freq_hz: float, src: np.ndarray, c: np.ndarray) -> np.ndarray:
    """Periodic fine grid b[l1, l0] (axis 0 fastest) of one frequency."""
    beta = es_beta(w)
    u = (freq_hz / C_LIGHT) * (src[:, :2] @ lat.A)          # turns, [n_src, 2]
    t = u - np.floor(u)                                     # [0, 1)
    b = np.zeros((nf[1], nf[0]), dtype=np.complex128)
    cells = []
    wts = []
    for a in range(2):
        g = t[:, a] * nf[a]                                 # grid coordinate in cells
        l0 = np.ceil(g - 0.5 * w).astype(np.int64)
        ii = l0[:, None] + np.arange(w)[None, :]
        z = (ii - g[:, None]) / (0.5 * w)
        cells.append(np.mod(ii, nf[a]))
        wts.append(es_phi(z, beta))
    for s in range(src.shape[0]):
        np.add.at(b, (cells[1][s][:, None], cells[0][s][None, :]), c[s] * np.outer(wts[1][s], wts[0][s]))
    return b


def modes(lat: Lattice, nf: np.ndarray, w: int, b: np.ndarray) -> np.ndarray:
    """f[k1 + K1, k0 + K0] for k in [-K, K]^2 (axis 0 fastest)."""
    beta = es_beta(w)
    h = 2 * math.pi / nf
    out = b
    fac = []
    for a in (0, 1):
        k = np.arange(-lat.K[a], lat.K[a] + 1)
        l = np.arange(nf[a])
        E = np.exp(-1j * np.outer(k, l) * h[a])             # [N_a, n_a]
        alpha = w * h[a] / 2
        fac.append(h[a] / (alpha * es_phihat(alpha * k, beta)))
        if a == 0:
            out = out @ E.T                                 # [n1, N0]
        else:
            out = E @ out                                   # [N1, N0]
    return out * np.outer(fac[1], fac[0])


def type1_vis(ant: np.ndarray, src: np.ndarray, freq: np.ndarray, c: np.ndarray, eps: float,
              lat: Optional[Lattice] = None) -> np.ndarray:
    """V[f, pair] for pairs i <= j in row-major order; c is [n_freq, n_src]."""
    if lat is None:
        lat = find_lattice(ant, lattice_tolerance(eps, freq))
        if lat is None:
            raise ValueError("antennas are not on a lattice")
    w = kernel_width_type1(eps)
    nf = grid_sizes(lat, w)
    n = ant.shape[0]
    iu, ju = np.triu_indices(n)
    dk = lat.k[iu] - lat.k[ju]                              # k_i - k_j
    out = np.empty((len(freq), len(iu)), dtype=np.complex128)
    for f, nu in enumerate(freq):
        fk = modes(lat, nf, w, spread(lat, nf, w, nu, src, c[f]))
        out[f] = fk[dk[:, 1] + lat.K[1], dk[:, 0] + lat.K[0]]
    return out
