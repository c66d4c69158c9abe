"""MI355X-native IFGF-accelerated N-Mueller boundary-integral operator.

The compute lives in the HIP/C++ library libifgf.so (C-ABI in include/ifgf.h);
`binding` marshals torch/numpy arguments to it.
"""
from .binding import (IFGFError, IFGFEval, IFGFPlan, NMullerOperator, nmuller_apply, nmuller_plan,
                      nmuller_rhs, nmuller_destroy, ifgf_apply, ifgf_destroy, ifgf_plan,
                      ifgf_plan_counts, ifgf_plan_table, ifgf_stats, lib, MLP, MLP_BF16, MLP_FP32,
                      NMullerGraph)

__all__ = ["IFGFError", "IFGFEval", "IFGFPlan", "NMullerOperator", "nmuller_apply", "nmuller_plan",
           "nmuller_rhs", "nmuller_destroy", "ifgf_apply", "ifgf_destroy", "ifgf_plan",
           "ifgf_plan_counts", "ifgf_plan_table", "ifgf_stats", "lib", "MLP", "MLP_BF16", "MLP_FP32",
           "NMullerGraph"]
