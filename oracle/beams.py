"""Visibilities with per-antenna beams, summed directly in FP64 numpy.

TEST INFRASTRUCTURE ONLY (oracle side; the product never imports this).

Section 2.2.3 of the paper: when antennas carry different beam patterns the
direction-dependent response of a baseline depends on the pair of patterns
of its two antennas, so one snapshot needs one transform per unordered pair of
patterns, N_beam (N_beam + 1) / 2 of them.  For scalar (unpolarised) real
amplitude beams a_p the strength of source s on baseline (i, j) is
a_{p(i)}(s) a_{p(j)}(s) flux(s), and

    V_ij = sum_s a_{p(i)}(s) a_{p(j)}(s) flux(s) exp(-2 pi i (nu / c) (x_i - x_j) . s_hat_s)

written out here pair by pair (no grouping by pattern pair).
"""
from __future__ import annotations

import numpy as np

from .type3 import C_LIGHT


def beams_vis(ant_enu, src_lmn, freq_hz, flux, beams, beam_of_ant, pairs=None) -> np.ndarray:
    """V[f, pair] for pairs i <= j in row-major order.  beams: [n_beam, n_freq,
    n_src] amplitude patterns; beam_of_ant: [n_ant] pattern index."""
    ant = np.asarray(ant_enu, dtype=np.float64)
    src = np.asarray(src_lmn, dtype=np.float64).reshape(-1, 3)
    freq = np.asarray(freq_hz, dtype=np.float64).reshape(-1)
    fl = np.asarray(flux, dtype=np.float64).reshape(len(freq), src.shape[0])
    bm = np.asarray(beams, dtype=np.float64).reshape(-1, len(freq), src.shape[0])
    pat = np.asarray(beam_of_ant, dtype=np.int64)
    iu, ju = np.triu_indices(ant.shape[0])
    if pairs is not None:
        iu, ju = iu[pairs], ju[pairs]
    out = np.zeros((len(freq), len(iu)), dtype=np.complex128)
    for f, nu in enumerate(freq):
        for k, (i, j) in enumerate(zip(iu, ju)):
            c = bm[pat[i], f] * bm[pat[j], f] * fl[f]
            ph = -2.0 * np.pi * nu / C_LIGHT * (src @ (ant[i] - ant[j]))
            out[f, k] = np.sum(c * np.exp(1j * ph))
    return out
