"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only *generates inputs*: antenna layouts, source directions, fluxes,
beam weights and frequencies.  It holds none of the visibility arithmetic
(no phases, no transforms): both the oracle and the HIP path consume what it
returns, and neither is imported here.

Recipes follow the workloads of the paper's sections 4 and 5 (hexagonal
HERA-like arrays of 14.6 m spacing, power-law point-source counts, Gaussian
beams scaled with frequency, an equal-area Nside-256-like diffuse sky); the
public catalogues and layout files the paper used are not available, so
seeded stand-ins of the same shape are drawn here.

The rotation and beam here only build the ENU inputs of per-snapshot
problems.  Drift scans (``DriftScan``) are handed over in equatorial form: the
device front end and the oracle's own rotation and beam (``oracle.frontend``)
each turn them into snapshots, and neither uses this module's versions.
"""
from .workloads import (  # noqa: F401
    C_LIGHT, SEED_BASE, Problem, hex_array, disk_array, gaussian_beam,
    powerlaw_fluxes, isotropic_hemisphere, unit_disk_lm, fibonacci_sphere,
    equatorial_to_enu, config1, config2, config3, config4, config5_requests,
    small_problem, subset_pairs, DriftScan, config4_drift, small_drift,
)
