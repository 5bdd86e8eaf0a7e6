"""Seeded synthetic inputs shared by the tests, the bench and the oracle checks.

This package holds input construction only (random orthogonal bases,
prescribed spectra, perturbation sequences, arrival times).  It computes no
part of the projection method and imports neither the GPU library nor the
oracle.
"""
from .generators import *  # noqa: F401,F403
from .generators import __all__  # noqa: F401
from .sdp import (Sdp, complete_graph, cycle_graph, dual_infeasible, maxcut,  # noqa: F401
                  primal_infeasible, random_graph, theta, trace_min)
