"""Seeded synthetic inputs for the Mobius domain-wall solver.

This module only draws random numbers and lays them out in the host
layouts that both the HIP library and the FP64 oracle accept.  It holds
none of the solver's arithmetic: no hopping term, no fifth-dimension
operator, no Krylov step.  Both sides receive its arrays as plain data.

Host layouts (FP64, complex interleaved):

* gauge field  ``U[T][Z][Y][X][mu][3][3]``; ``U[x][mu]`` is the SU(3) link
  from site ``x`` to ``x + mu_hat``, ``mu = 0, 1, 2, 3`` for ``x, y, z, t``;
* single-parity 5D field ``psi[Ls][V/2][4][3]`` (spin, colour) on the sites of
  one checkerboard parity, ordered by ``lex // 2`` with
  ``lex = x + X*(y + Y*(z + Z*t))``.
"""
from .fields import (
    gauge_field,
    unit_gauge_field,
    gaussian_source,
    point_smeared_sources,
    random_gauge_transform,
    gauge_transform_links,
)
from .configs import CONFIGS, Config

__all__ = [
    "gauge_field",
    "unit_gauge_field",
    "gaussian_source",
    "point_smeared_sources",
    "random_gauge_transform",
    "gauge_transform_links",
    "CONFIGS",
    "Config",
]
