"""Seeded synthetic scene generators shared by the GPU library's tests and the oracle.

This package holds geometry and motion only: triangle meshes of box-shaped
buildings, vehicles and a ground plane, transmitter and receiver positions and
per-frame rigid transforms.  It contains none of the propagation method's
arithmetic (no ray tracing, no path search, no field evaluation).
"""

from .city import (  # noqa: F401
    Scene,
    Frame,
    WorkloadConfig,
    make_city,
    workload,
    WORKLOADS,
    tiny_ground,
    tiny_ground_wall,
    tiny_canyon,
    tiny_wedge,
)
