"""Spectral-basis evaluation of the visibility sum, step by step in FP64 numpy.

TEST INFRASTRUCTURE ONLY (oracle side; the product never imports this).

Appendix A of the paper: sky and beam spectra are projected per source onto a
compact spectral basis M (n_freq x K),

    s_hat = (M^T M)^-1 M^T s,     b_hat = (M^T M)^-1 M^T b,

their product is expanded with the basis's structure constants

    d^k_ij = sum_q M_qi M_qj M_qk,     v_k = sum_ij s_hat_i b_hat_j d^k_ij,

one transform per basis function k takes v_k to the uv-plane, and the result
is expanded back to the frequencies and evaluated at the baselines:

    V(b, nu_q) = sum_k M_qk F_k(b nu_q / c),
    F_k(u) = sum_s v_{k,s} exp(-2 pi i u . s_hat_s).

The structure constants give the projection of the product only for a basis
with orthonormal columns, so the basis here is the discrete orthonormal
polynomial basis of the frequencies: the first K columns of the QR
factorisation of the Vandermonde matrix in x = (nu - nu_mid) / half-width,
with the signs making R's diagonal positive.  F_k is evaluated here by the
exact direct sum at each frequency's baselines.
"""
from __future__ import annotations

import numpy as np

from . import direct_vis


def spectral_basis(freq_hz: np.ndarray, K: int) -> np.ndarray:
    """[n_freq, K] orthonormal columns (discrete orthonormal polynomials)."""
    nu = np.asarray(freq_hz, dtype=np.float64)
    half = 0.5 * (nu.max() - nu.min())
    x = (nu - 0.5 * (nu.max() + nu.min())) / (half if half > 0 else 1.0)
    V = np.vander(x, K, increasing=True)
    Q, R = np.linalg.qr(V)
    return Q * np.sign(np.diag(R))[None, :]


def project(M: np.ndarray, y: np.ndarray) -> np.ndarray:
    """(M^T M)^-1 M^T y for y [n_freq, n_src] -> [K, n_src]."""
    return np.linalg.solve(M.T @ M, M.T @ y)


def structure_constants(M: np.ndarray) -> np.ndarray:
    """d[i, j, k] = sum_q M_qi M_qj M_qk."""
    return np.einsum("qi,qj,qk->ijk", M, M, M)


def product_coeffs(s_hat: np.ndarray, b_hat: np.ndarray, d: np.ndarray) -> np.ndarray:
    """v[k, s] = sum_ij s_hat[i, s] b_hat[j, s] d[i, j, k]."""
    return np.einsum("is,js,ijk->ks", s_hat, b_hat, d)


def basis_vis(ant_enu, src_lmn, freq_hz, flux, beam, K: int, pairs=None) -> np.ndarray:
    """V[f, pair] through a K-function spectral basis (beam None = 1)."""
    freq = np.asarray(freq_hz, dtype=np.float64)
    fl = np.asarray(flux, dtype=np.float64)
    bm = np.ones_like(fl) if beam is None else np.asarray(beam, dtype=np.float64)
    M = spectral_basis(freq, K)
    v = product_coeffs(project(M, fl), project(M, bm), structure_constants(M))
    out = None
    for q, nu in enumerate(freq):
        # F_k at this frequency's baselines, for every k at once (one strength row per k)
        Fk = direct_vis(ant_enu, src_lmn, np.full(K, nu), v, pairs=pairs)     # [K, n_pairs]
        row = M[q] @ Fk
        out = row[None] if out is None else np.concatenate([out, row[None]])
    return out
