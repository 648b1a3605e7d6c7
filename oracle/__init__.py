"""CPU oracle for the sliced QAOA amplitude contraction.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, links or
executes anything here; only the test-suite, the smoke check and the
benchmark's CPU-baseline leg do.  The oracle shares no code with the HIP path:
it rebuilds every tensor, order and cost from the instance data by itself.
"""
from .qaoa import (  # noqa: F401
    variable_id, qaoa_factors, statevector, statevector_amplitude,
    brute_force_amplitude, restrict_factors, eliminate, ve_amplitude,
    slice_partial, neumaier_sum, sliced_amplitude, interaction_graph,
    min_degree_order, min_fill_order, elimination_cost, bags_from_order,
    check_tree_decomposition, exact_treewidth, closed_form_amplitude,
)
from .search import splitmix64, SplitMix64, ga_cut_search, ga_min_k  # noqa: F401
from .mlp import MLP64  # noqa: F401
