"""Seeded synthetic inputs for the D3(BJ) path.

This package only draws inputs: a synthetic D3 reference table, periodic
cells of bilayer graphene and MOF-like composition, and MD start velocities.
It holds none of the dispersion arithmetic, so both the FP64 oracle and the
GPU path can consume its output without sharing any of the method's code.
"""

from .table import make_table, ELEMENTS, MASSES_AMU, MAX_REF  # noqa: F401
from .structures import (  # noqa: F401
    bilayer_graphene,
    mof_like,
    mof_counts,
    maxwell_velocities,
    cluster,
    simple_lattice,
)
