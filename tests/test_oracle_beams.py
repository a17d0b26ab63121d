"""Pins of the oracle's per-antenna-beam sum (no GPU): one pattern reduces to
the direct sum with the squared pattern as power beam, the zenith closed form,
a dead antenna, and the symmetry of the pattern pair."""
import numpy as np

import oracle
import synth
from oracle import beams


def _setup(seed, n_ant=9, n_src=40, n_freq=2, n_beam=3):
    rng = np.random.default_rng(seed)
    ant = synth.hex_array(n_ant)
    src = synth.workloads.isotropic_hemisphere(rng, n_src)
    freq = np.linspace(120e6, 180e6, n_freq)
    flux = rng.uniform(0.1, 2.0, (n_freq, n_src))
    pats = rng.uniform(0.2, 1.0, (n_beam, n_freq, n_src))
    which = rng.integers(0, n_beam, n_ant)
    return ant, src, freq, flux, pats, which


def test_one_pattern_is_the_direct_sum_with_its_power_beam():
    ant, src, freq, flux, pats, _ = _setup(1, n_beam=1)
    v = beams.beams_vis(ant, src, freq, flux, pats, np.zeros(len(ant), dtype=int))
    ref = oracle.direct_vis(ant, src, freq, flux, pats[0] ** 2)
    assert oracle.rel_l2(v, ref) < 1e-13


def test_zenith_source_gives_the_pattern_product():
    ant, _, freq, _, _, which = _setup(2)
    src = np.array([[0.0, 0.0, 1.0]])
    pats = np.array([[[0.5], [0.6]], [[0.8], [0.9]], [[1.0], [0.3]]])
    flux = np.array([[2.0], [4.0]])
    v = beams.beams_vis(ant, src, freq, flux, pats, which)
    iu, ju = np.triu_indices(len(ant))
    want = pats[which[iu], :, 0].T * pats[which[ju], :, 0].T * flux
    assert np.allclose(v, want, atol=1e-14)


def test_dead_antenna_and_hermitian_pairs():
    ant, src, freq, flux, pats, which = _setup(3, n_beam=2)
    pats = np.concatenate([pats, np.zeros((1,) + pats.shape[1:])])  # pattern 2 is dead
    which[4] = 2
    v = beams.beams_vis(ant, src, freq, flux, pats, which)
    iu, ju = np.triu_indices(len(ant))
    dead = (iu == 4) | (ju == 4)
    assert np.all(v[:, dead] == 0) and np.all(np.abs(v[:, ~dead]) > 0)
    # swapping the antennas of a pair (i > j) conjugates, as for one shared beam
    sw = beams.beams_vis(ant[::-1], src, freq, flux, pats, which[::-1])
    n = len(ant)
    k_rev = {(i, j): k for k, (i, j) in enumerate(zip(iu, ju))}
    for k, (i, j) in enumerate(zip(iu, ju)):
        a, b = n - 1 - j, n - 1 - i   # (i, j) in the reversed order is the pair (n-1-j, n-1-i)
        assert np.allclose(sw[:, k_rev[(a, b)]], np.conj(v[:, k]), atol=1e-12)


def test_grouping_by_pattern_pair_matches():
    # the sum of each pair depends only on its unordered pattern pair: pairs with
    # the same patterns equal the direct sum with the product pattern
    ant, src, freq, flux, pats, which = _setup(4, n_ant=12)
    v = beams.beams_vis(ant, src, freq, flux, pats, which)
    iu, ju = np.triu_indices(len(ant))
    for p in range(pats.shape[0]):
        for q in range(p, pats.shape[0]):
            sel = np.where(((which[iu] == p) & (which[ju] == q)) | ((which[iu] == q) & (which[ju] == p)))[0]
            if len(sel) == 0:
                continue
            ref = oracle.direct_vis(ant, src, freq, flux, pats[p] * pats[q], pairs=sel)
            assert oracle.rel_l2(v[:, sel], ref) < 1e-12
