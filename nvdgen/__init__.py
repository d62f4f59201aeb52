"""Seeded synthetic inputs (graphs, node-vector pairs, edge weights).

This package holds input construction only; it computes nothing of the
distance method itself.  It is the one piece shared by the CPU oracle and the
GPU library's tests and benchmarks.
"""
from .graphs import *  # noqa: F401,F403
from .vectors import *  # noqa: F401,F403
from .configs import (Workload, workload, ws_connected, seeds, density_graph,  # noqa: F401
                      DENSITY_MODELS, DENSITY_DEGREES, DENSITY_N)
