"""Pins of the oracle's lattice detection and type-1 path (no GPU)."""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import type1


@pytest.mark.parametrize("n", [7, 37, 127, 350])
def test_hex_array_is_a_lattice_with_the_spacing_cell(n):
    ant = synth.hex_array(n)
    lat = type1.find_lattice(ant, 1e-9)
    assert lat is not None
    s = synth.workloads.HERA_SPACING
    # unit cell of the triangular lattice of spacing s
    assert abs(abs(np.linalg.det(lat.A)) - s * s * math.sqrt(3) / 2) < 1e-9
    assert np.allclose(np.linalg.norm(lat.A, axis=0), s)
    # positions reproduced exactly by the integer coordinates
    assert np.abs(lat.k @ lat.A.T - (ant[:, :2] - ant[0, :2])).max() < 1e-9


def test_square_grid_is_a_lattice():
    d = 3.5
    ant = np.array([[i * d, j * d, 0.0] for i in range(5) for j in range(4)])
    lat = type1.find_lattice(ant, 1e-9)
    assert lat is not None and abs(abs(np.linalg.det(lat.A)) - d * d) < 1e-12
    assert sorted(lat.K.tolist()) == [3, 4]


def test_random_collinear_and_jittered_arrays_are_not_lattices():
    rng = np.random.default_rng(5)
    assert type1.find_lattice(synth.disk_array(rng, 30, 100.0, 0.0), 1e-6) is None
    line = np.array([[i * 2.0, i * 1.0, 0.0] for i in range(10)])
    assert type1.find_lattice(line, 1e-9) is None
    ant = synth.hex_array(37)
    jit = ant + np.concatenate([rng.normal(0, 1e-2, (37, 2)), np.zeros((37, 1))], 1)
    assert type1.find_lattice(jit, 1e-6) is None
    tiny = ant + np.concatenate([rng.normal(0, 1e-13, (37, 2)), np.zeros((37, 1))], 1)
    assert type1.find_lattice(tiny, 1e-9) is not None


def test_type1_kernel_width_is_the_papers_rule():
    # w = ceil(log10(1/eps)) + 1, at least 3
    assert [type1.kernel_width_type1(e) for e in (1e-1, 1e-2, 1e-3, 1e-6, 1e-12)] == [3, 3, 4, 7, 13]


@pytest.mark.parametrize("eps", [1e-4, 1e-6, 1e-8, 1e-10, 1e-12])
def test_type1_within_eps_of_direct_sum(eps):
    p = synth.small_problem(120, n_ant=37, n_src=150, n_freq=2, hex_layout=True)
    c = p.strengths()
    got = type1.type1_vis(p.ant_enu, p.src_lmn, p.freq_hz, c, eps)
    ref = oracle.direct_problem(p)
    assert oracle.rel_l2(got, ref) <= eps


def test_type1_error_falls_with_eps():
    p = synth.small_problem(121, n_ant=19, n_src=80, n_freq=1, hex_layout=True)
    ref = oracle.direct_problem(p)
    c = p.strengths()
    errs = [oracle.rel_l2(type1.type1_vis(p.ant_enu, p.src_lmn, p.freq_hz, c, e), ref)
            for e in (1e-3, 1e-5, 1e-7, 1e-9, 1e-11)]
    assert all(b < a for a, b in zip(errs, errs[1:])), errs


def test_type1_zenith_source_is_constant():
    ant = synth.hex_array(19)
    src = np.array([[0.0, 0.0, 1.0]])
    v = type1.type1_vis(ant, src, np.array([150e6]), np.array([[3.0]]), 1e-10)
    assert np.allclose(v, 3.0, rtol=1e-10, atol=1e-10)


def test_rotated_hex_array_is_a_lattice_and_modes_reproduce_every_baseline():
    # a joint rotation of the array keeps it a lattice (the basis rotates with
    # it), and A (k_i - k_j) is the baseline of every pair i <= j
    th = 0.37
    R = np.array([[math.cos(th), -math.sin(th), 0.0], [math.sin(th), math.cos(th), 0.0], [0.0, 0.0, 1.0]])
    ant = synth.hex_array(61) @ R.T + np.array([3.0, -7.0, 0.0])
    lat = type1.find_lattice(ant, 1e-9)
    assert lat is not None
    iu, ju = np.triu_indices(ant.shape[0])
    b = ant[iu, :2] - ant[ju, :2]
    dk = lat.k[iu] - lat.k[ju]
    assert np.abs(dk @ lat.A.T - b).max() < 1e-9
    assert np.all(np.abs(dk) <= lat.K[None, :])


def test_type1_on_rotated_array_matches_direct_sum():
    th = 1.1
    R = np.array([[math.cos(th), -math.sin(th), 0.0], [math.sin(th), math.cos(th), 0.0], [0.0, 0.0, 1.0]])
    p = synth.small_problem(122, n_ant=19, n_src=60, n_freq=2, hex_layout=True)
    ant = p.ant_enu @ R.T
    got = type1.type1_vis(ant, p.src_lmn, p.freq_hz, p.strengths(), 1e-8)
    ref = oracle.direct_vis(ant, p.src_lmn, p.freq_hz, p.flux, p.beam)
    assert oracle.rel_l2(got, ref) <= 1e-8
