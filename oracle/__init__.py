"""FP64 CPU oracle for the MSPCG hot path (arxiv 2104.05615).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``, never by the HIP library or its
Python binding.  It shares no code with them.

Parity unpinned: none of the functions here is left without an independent
check; the checks live in ``tests/test_oracle_*.py``.
"""
from .dwf import (  # noqa: F401
    GAMMA, GAMMA5, P_PLUS, P_MINUS,
    parity_coords, wilson_hop, build_hop_library,
    ptilde, m5_matrix, mphi_matrix, inverse5, adjoint5, apply5, norm2,
    MobiusDWF, Tiling, tiling_ok, local_operator, padded_operator, truncated_local_operator,
    local_operator_stored, inner_cg_stored, stored_links,
    inner_cg, precondition,
    pcg, mspcg, cg, SolveInfo, stored, STORAGE_FORMATS,
    transform, transform_dag, local_op_full, reduced_precondition, outer_sum, chi2,
    line_quartic, quartic_min, train_transform,
)
