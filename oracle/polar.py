"""Polarised visibilities (2 x 2 feed products), summed directly in FP64 numpy.

TEST INFRASTRUCTURE ONLY (oracle side; the product never imports this).

Section 2.1 of the paper (the measurement equation in Jones form): with
point sources and one beam shared by every antenna,

    V_ij = sum_s A(s) C(s) A(s)^H exp(-2 pi i (nu / c) (x_i - x_j) . s_hat_s)

where A(s) is the 2 x 2 complex voltage response of the feeds and the
coherency matrix C = [[I + Q, U + i V], [U - i V, I - Q]] holds the Stokes
parameters.  V_ij is a 2 x 2 matrix per pair and frequency; it is written out
here source by source with full matrix products (no split into real
strengths).
"""
from __future__ import annotations

import numpy as np

from .type3 import C_LIGHT


def coherency(I, Q, U, V) -> np.ndarray:
    """[..., 2, 2] coherency matrices from Stokes arrays."""
    C = np.empty(np.shape(I) + (2, 2), dtype=np.complex128)
    C[..., 0, 0] = I + Q
    C[..., 0, 1] = U + 1j * V
    C[..., 1, 0] = U - 1j * V
    C[..., 1, 1] = I - Q
    return C


def polar_vis(ant_enu, src_lmn, freq_hz, stokes, jones=None, pairs=None) -> np.ndarray:
    """V[f, pair, 2, 2] for pairs i <= j in row-major order.  stokes:
    [4, n_freq, n_src] (I, Q, U, V); jones: [n_freq, n_src, 2, 2] complex, or
    None for the identity."""
    ant = np.asarray(ant_enu, dtype=np.float64)
    src = np.asarray(src_lmn, dtype=np.float64).reshape(-1, 3)
    freq = np.asarray(freq_hz, dtype=np.float64).reshape(-1)
    st = np.asarray(stokes, dtype=np.float64).reshape(4, len(freq), src.shape[0])
    iu, ju = np.triu_indices(ant.shape[0])
    if pairs is not None:
        iu, ju = iu[pairs], ju[pairs]
    out = np.zeros((len(freq), len(iu), 2, 2), dtype=np.complex128)
    for f, nu in enumerate(freq):
        C = coherency(st[0, f], st[1, f], st[2, f], st[3, f])          # [n_src, 2, 2]
        if jones is not None:
            A = np.asarray(jones[f], dtype=np.complex128)               # [n_src, 2, 2]
            C = A @ C @ np.conj(np.transpose(A, (0, 2, 1)))
        for k, (i, j) in enumerate(zip(iu, ju)):
            ph = np.exp(-2j * np.pi * nu / C_LIGHT * (src @ (ant[i] - ant[j])))
            out[f, k] = np.einsum("s,sab->ab", ph, C)
    return out
