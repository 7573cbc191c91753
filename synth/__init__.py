"""Seeded synthetic inputs for the SVLF per-ray render path.

This package only *generates inputs*: occupied-leaf coordinates of analytic
scenes, per-vertex feature tables, MLP initial weights, camera rays and
analytic ground-truth targets.  It contains none of the method's arithmetic
(no octree traversal, no interpolation, no MLP evaluation, no compositing),
so both the FP64 oracle and the HIP path can consume the arrays it returns
without sharing any computation.

Random draws use ``numpy.random.Generator(PCG64)`` streams derived from one
``SeedSequence(seed)`` per workload, one child stream per purpose, in the order
scene -> features -> MLP -> cameras -> batch (see ``configs.streams``).
"""

from .configs import WORKLOADS, Workload, get_workload, streams  # noqa: F401
