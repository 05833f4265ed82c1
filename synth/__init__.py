"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package only draws random numbers and shapes them into the canonical
layouts (gauge links, fermion fields, test directions).  It contains none of
the domain-wall operator's arithmetic, so it can serve both the CPU oracle and
the HIP path without coupling them.
"""

from .fields import (  # noqa: F401
    WORKLOADS,
    gauge_field,
    fermion_full,
    fermion_cb,
    su3_directions,
    random_su3_field,
    unit_gauge,
    lattice_volume,
)
