"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws random graphs, weights and starting factors.  It holds
none of the method's arithmetic: it does not build cost matrices, constraint
maps or anything the solver computes.  Both the CPU oracle and the HIP path
take their inputs from here, so that the two see exactly the same data.

All randomness is NumPy's PCG64 (``numpy.random.default_rng(seed)``).
"""

from .graphs import (  # noqa: F401
    Graph,
    er_graph,
    torus_graph,
    cycle_graph,
    complete_graph,
    complete_bipartite_graph,
    edgeless_graph,
    rmat_graph,
    batch_instances,
    init_factor,
    draw_weights,
)
from .completion import Completion, completion_instance, sample_count  # noqa: F401
