"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds geometry and random draws only: a geodesic sphere mesh, a
trihedral corner reflector mesh, complex Gaussian vectors, random directions (and the
plane waves travelling along them) and random Tucker factors of given shapes.  It
contains none of the method's arithmetic (no far-field quadrature, no basis
functions, no decomposition, no tensor products), so that the CPU oracle and the
GPU library can both be fed from it without sharing any code path.

Workload parameters (sphere size, mesh frequency, box edge, angular grid, tolerance,
seeds) live in :mod:`synth.workloads`.
"""
from .mesh import icosphere, trihedral
from .draws import (complex_normal, unit_vectors, planewaves, synthetic_tucker,
                    synthetic_ranks, rng)

__all__ = ["icosphere", "trihedral", "complex_normal", "unit_vectors", "planewaves", "synthetic_tucker",
           "synthetic_ranks", "rng"]
