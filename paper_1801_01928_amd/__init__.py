"""MI355X-native TT-completion hot path (gather, adjoint, Riemannian step,
Gram matrices, batched plans) and the TT-matrix layer.

The compute lives in libttgfx.so (hand-written HIP kernels for gfx950 behind
the C ABI of include/ttgfx.h); this package marshals arguments only.
"""
from ._lib import load, TTError, last_error, TT_LR, TT_RL  # noqa: F401
from .tt import (  # noqa: F401
    TT,
    check_indices,
    gather,
    gather_backward,
    gather_halves,
    halves_split,
    halves_tables,
    gather_mse_backward,
    gather_mse_workspace,
    tt_gather,
    KernelTimer,
    orthogonalize,
    orthogonalize_both,
    project_sparse,
    round_tt,
    riemannian_step,
    line_search_terms,
    project_tt,
    project_sum,
    tangent_combine,
    completion_iteration,
    cg_iteration,
    riemannian_cg,
    tangent_inner,
    tangent_gram,
    tangent_axpby,
    riemannian_completion,
    gram,
    BatchedPlan,
    TTMatrix,
    ttm_matmul,
    tt_matvec,
    tt_matmat,
    ttm_matmul_backward,
    tt_linear,
)
