"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle checks.

This package only draws random graphs and query parameters.  It holds none of
the influence-maximization arithmetic: no RR sampling, no coding, no seed
selection.  Both the GPU path and the CPU oracle consume what it produces.
"""

from .graphs import (  # noqa: F401
    Graph,
    erdos_renyi,
    rmat,
    lt_weights,
    chung_lu,
    tiny_graph,
    config_graph,
    batched_instances,
)
