"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

Holds none of the method's arithmetic: it draws random band-limited fields
on the sphere, evaluates them on a tensor grid of points and stores them as
modal coefficients in the state layout q[E][3][N].
"""
from .fields import (band_limited_state, ensemble_members, gaussian_bump_plane,
                     lake_at_rest_state, random_plane_state, sine_square, StateInfo)

__all__ = ["band_limited_state", "ensemble_members", "gaussian_bump_plane", "lake_at_rest_state",
           "random_plane_state", "sine_square", "StateInfo"]
