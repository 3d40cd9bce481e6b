"""Seeded synthetic particle sets shared by the tests, the benchmark and the smoke check.

This package only draws inputs (positions, velocities, masses, smoothing lengths,
energies).  It holds none of the SPH or tree arithmetic: the reference implementation
lives in ``oracle/`` and the GPU implementation in ``paper_2007_03097_amd/``.
"""
from .generators import (  # noqa: F401
    ParticleSet,
    lattice_box,
    sod_tube,
    polytrope_n1,
    ensemble,
    evrard,
    uniform_random,
    fig1_points,
)
