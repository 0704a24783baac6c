"""Seeded synthetic inputs (initial states) shared by the HIP path's tests/bench and the oracle.

This package holds input generation only: Gaussian random fields, string loops and
plane waves used as initial states.  It contains none of the time-stepping, ghost,
interpolation, tagging or energy arithmetic of the method, so both sides can take
their inputs from here without sharing any of the computation that is compared.
"""
from .ic import (  # noqa: F401
    gaussian_random_pair,
    random_state,
    string_loop_state,
    straight_strings,
    plane_wave,
    quadratic_field,
    state_from_psi,
)
