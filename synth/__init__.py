"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package holds graphs, lattices, leg structures of site tensors, raw
random numbers and the contraction-path planner. It contains none of the
method's arithmetic: it never enumerates symmetry blocks, never computes a
fermionic sign and never contracts anything. Each side takes the dense random
arrays drawn here and extracts the allowed blocks with its own code.
"""

from .graphs import square_lattice, random_regular_graph, diamond_lattice
from .peps import (LegSpec, SiteSpec, PepsSpec, z2_leg, u1u1_leg, make_peps,
                   site_values, occupation_samples)
from .paths import greedy_path, path_stats
from . import workloads

__all__ = [
    "square_lattice", "random_regular_graph", "diamond_lattice",
    "LegSpec", "SiteSpec", "PepsSpec", "z2_leg", "u1u1_leg", "make_peps",
    "site_values", "occupation_samples", "greedy_path", "path_stats",
    "workloads",
]
