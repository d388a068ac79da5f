"""Seeded synthetic inputs shared by the CPU oracle, the tests and the bench.

Nothing here performs the solver's own arithmetic: this package only builds
permeability fields, face transmissibilities, boundary/well connections,
sources and request streams.
"""
from .grids import (  # noqa: F401
    Problem,
    rng_for,
    make_config0,
    make_config1,
    make_config2,
    make_config3_member,
    make_lognormal_box,
    make_homogeneous,
    pressure_increment_pair,
)
