"""Pins of the oracle's drift-scan front end (rotation to ENU, analytic beam):
fixed points of the sky, rigidity, periodicity, the beam's half-power width
and horizon, and a closed form of the resulting visibilities (no GPU)."""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import frontend

LAT = math.radians(-30.7215)


def _unit(alpha, delta):
    return np.stack([np.cos(delta) * np.cos(alpha), np.cos(delta) * np.sin(alpha), np.sin(delta)], axis=1)


def test_radec_round_trip():
    rng = np.random.default_rng(1)
    a = rng.uniform(-math.pi, math.pi, 50)
    d = rng.uniform(-1.5, 1.5, 50)
    a2, d2 = frontend.radec(_unit(a, d))
    assert np.allclose(a2, a, atol=1e-12) and np.allclose(d2, d, atol=1e-12)


@pytest.mark.parametrize("lst", [0.0, 1.3, 4.0])
def test_fixed_points_zenith_pole_east_west_meridian(lst):
    # the source transiting at declination = latitude is at the zenith
    assert np.allclose(frontend.enu(np.array([lst]), np.array([LAT]), lst, LAT), [[0, 0, 1]], atol=1e-12)
    # the north celestial pole sits at altitude = latitude due north, at any time
    assert np.allclose(frontend.enu(np.array([2.0]), np.array([math.pi / 2]), lst, LAT),
                       [[0, math.cos(LAT), math.sin(LAT)]], atol=1e-12)
    # on the celestial equator six hours east of the meridian is due east on the horizon
    assert np.allclose(frontend.enu(np.array([lst + math.pi / 2]), np.array([0.0]), lst, LAT), [[1, 0, 0]],
                       atol=1e-12)
    assert np.allclose(frontend.enu(np.array([lst - math.pi / 2]), np.array([0.0]), lst, LAT), [[-1, 0, 0]],
                       atol=1e-12)
    # on the meridian 30 degrees south of the zenith
    z = math.radians(30)
    assert np.allclose(frontend.enu(np.array([lst]), np.array([LAT - z]), lst, LAT),
                       [[0, -math.sin(z), math.cos(z)]], atol=1e-12)


def test_rotation_is_rigid_and_sidereal_periodic():
    rng = np.random.default_rng(2)
    a = rng.uniform(0, 2 * math.pi, 40)
    d = np.arcsin(rng.uniform(-1, 1, 40))
    eq = _unit(a, d)
    e = frontend.enu(a, d, 0.7, LAT)
    assert np.allclose(np.linalg.norm(e, axis=1), 1.0, atol=1e-14)
    assert np.allclose(e @ e.T, eq @ eq.T, atol=1e-13)           # angles preserved
    # handedness preserved (a rotation, not a reflection)
    assert np.allclose(np.linalg.det(e[:3]), np.linalg.det(eq[:3]), atol=1e-12)
    assert np.allclose(frontend.enu(a, d, 0.7 + 2 * math.pi, LAT), e, atol=1e-12)
    # the sky turns westward: an hour later a source's hour angle grows
    e1 = frontend.enu(np.array([0.0]), np.array([0.0]), -0.1, 0.0)
    e2 = frontend.enu(np.array([0.0]), np.array([0.0]), 0.1, 0.0)
    assert e1[0, 0] > 0 > e2[0, 0]


def test_beam_half_power_width_scaling_and_horizon():
    F, nu0 = math.radians(10.0), 150e6
    th = np.array([0.0, F / 2, F / 4, math.pi / 2 + 1e-9, 2.0])
    dirs = np.stack([np.sin(th), np.zeros(5), np.cos(th)], axis=1)
    b = frontend.gaussian_beam(dirs, np.array([nu0, 2 * nu0]), F, nu0)
    assert b[0, 0] == 1.0 and abs(b[0, 1] - 0.5) < 1e-12
    assert abs(b[1, 2] - 0.5) < 1e-12                             # half the width at twice the frequency
    assert np.all(b[:, 3:] == 0.0)                                 # below the horizon
    assert np.all(frontend.gaussian_beam(dirs, np.array([nu0]), 0.0, nu0)[0] == [1, 1, 1, 0, 0])


def test_drift_of_a_transiting_source_is_its_flux_on_every_baseline():
    ant = synth.hex_array(7)
    lsts = np.array([0.3, 1.0])
    eq = _unit(lsts, np.array([LAT, LAT]))                         # each transits at one of the LSTs
    flux = np.array([[2.0, 0.0]])
    v = frontend.drift_vis(ant, eq, np.array([150e6]), flux, lsts[:1], LAT, math.radians(10), 150e6)
    assert np.allclose(v, 2.0, atol=1e-12)
    # an hour later the source has moved off the zenith: the beam drops and phases appear
    v2 = frontend.drift_vis(ant, eq, np.array([150e6]), flux, lsts[:1] + 0.26, LAT, math.radians(10), 150e6)
    assert np.all(np.abs(v2) < 2.0) and np.abs(v2.imag).max() > 1e-3


def test_drift_matches_the_direct_sum_of_each_rotated_snapshot():
    rng = np.random.default_rng(4)
    a = rng.uniform(0, 2 * math.pi, 30)
    d = np.arcsin(rng.uniform(-1, 0.3, 30))
    ant = synth.hex_array(12)
    freq = np.array([120e6, 180e6])
    flux = rng.uniform(0.1, 2.0, (2, 30))
    v = frontend.drift_vis(ant, _unit(a, d), freq, flux, [0.5], LAT, math.radians(15), 150e6)
    e = frontend.enu(a, d, 0.5, LAT)
    b = frontend.gaussian_beam(e, freq, math.radians(15), 150e6)
    assert np.allclose(v[0], oracle.direct_vis(ant, e, freq, flux, b), atol=1e-12)
