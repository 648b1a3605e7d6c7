"""MI355X-native sliced tensor-network contraction of QAOA single amplitudes.

Host planner + HIP kernels live in libqtn.so (C ABI, include/qtn.h); this
package only binds it.  Build with paper_2010_14962_amd.build.build().
"""
from .qtn import (  # noqa: F401
    Plan, QtnError, QtnPartial, qtn_plan, qtn_partial_combine, plan_instance, lib,
    QTN_FP64, QTN_FP32, QTN_3XBF16, COST_FEATURES, CostMLP, cost_exact, cost_features,
    cut_search, batch_contract,
)
