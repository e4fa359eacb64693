"""Seeded synthetic polymer-melt inputs for the TILD particle-mesh step.

This package only *generates inputs* (bead positions, species, bond lists and
the run parameters of the five reference workloads).  It contains none of the
method's arithmetic: no assignment weights, transforms, forces or updates.
Both the FP64 oracle and the GPU library consume what it produces.
"""

from .melts import (  # noqa: F401
    CONFIGS,
    Melt,
    config,
    make_custom,
    make_melt,
    make_replicas,
    snap_to_lattice,
)
