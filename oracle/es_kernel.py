"""ES ("exponential of semicircle") spreading kernel and its Fourier transform.

TEST INFRASTRUCTURE ONLY (oracle side; the product never imports this).

Paper section 2.2, step 1: the spreading kernel is
    phi(z) = exp(beta * (sqrt(1 - z^2) - 1))   on [-1, 1], zero outside,
with beta = 2.3 w for a kernel touching w grid points per dimension.
Step 3 divides by the kernel's Fourier transform.  phi has no elementary
transform, so

    phihat(xi) = int_{-1}^{1} phi(z) cos(xi z) dz

is evaluated by Gauss-Legendre quadrature after the substitution
z = sin(theta), which turns the square-root endpoint behaviour into a smooth
periodic integrand:  int_{-pi/2}^{pi/2} exp(beta (cos t - 1)) cos(xi sin t) cos t dt.
The node count is doubled from 32 until two successive estimates agree to
2e-15 relative (at most 256 nodes, where the numpy node tables are still
accurate); pinned in the tests against mpmath adaptive quadrature.
"""
from __future__ import annotations

import numpy as np


def es_beta(w: int) -> float:
    """Shape parameter for a kernel of w points (paper section 2.2: beta = 2.3 w)."""
    return 2.3 * float(w)


def es_phi(z, beta: float):
    """phi(z) = exp(beta (sqrt(1 - z^2) - 1)) for |z| <= 1, else 0 (FP64)."""
    z = np.asarray(z, dtype=np.float64)
    out = np.zeros_like(z)
    m = np.abs(z) <= 1.0
    out[m] = np.exp(beta * (np.sqrt(1.0 - z[m] * z[m]) - 1.0))
    return out


_NODES: dict = {}


def _gl(n: int):
    if n not in _NODES:
        x, w = np.polynomial.legendre.leggauss(n)
        _NODES[n] = (x * (np.pi / 2.0), w * (np.pi / 2.0))
    return _NODES[n]


def _phihat_n(xi: np.ndarray, beta: float, n: int) -> np.ndarray:
    t, wt = _gl(n)
    g = wt * np.exp(beta * (np.cos(t) - 1.0)) * np.cos(t)
    return np.cos(np.outer(xi, np.sin(t))) @ g


def es_phihat(xi, beta: float) -> np.ndarray:
    """int_{-1}^{1} phi(z) cos(xi z) dz for each xi (FP64)."""
    xi = np.atleast_1d(np.asarray(xi, dtype=np.float64))
    n = 32
    prev = _phihat_n(xi, beta, n)
    while True:
        n *= 2
        cur = _phihat_n(xi, beta, n)
        scale = np.max(np.abs(cur)) if cur.size else 1.0
        if cur.size == 0 or np.max(np.abs(cur - prev)) <= 2e-15 * max(scale, 1e-300) or n >= 256:
            return cur
        prev = cur
