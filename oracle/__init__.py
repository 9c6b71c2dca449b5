"""Plain FP64 CPU oracle for the TT-completion hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import, call
or link anything in this directory; only the test suite, the smoke check and
the CPU-baseline leg of the benchmark do.  The oracle shares no code with the
HIP path (no kernels, headers, helpers or constant tables); the only thing the
two sides have in common is the seeded input generator in ``workloads``,
which holds none of the method's arithmetic.

Every function follows a definition stated in the T3F paper (arXiv 1801.01928)
or, where the paper only names an operation, the standard TT-format
algorithm of the literature it cites (Oseledets 2011 for the format and
rounding; Steinlechner 2016 for the tangent-space geometry).  Each function's
docstring names the passage it follows.  Arithmetic is float64 throughout.

Conventions (shared reading of the paper's index order, Introduction, entry
formula): a TT tensor is a list of cores ``G[k]`` with shape
``(r_k, n_k, r_{k+1})`` and ``r_0 = r_d = 1``; multi-indices are C-ordered
(``i_1`` slowest); observed index sets are stored structure-of-arrays as an
integer array ``idx`` of shape ``(d, M)``.
"""
from .core import (  # noqa: F401
    storage_count,
    ranks_of,
    full,
    gather,
    sparse_adjoint,
    gather_backward,
    mse_loss_and_grad,
    inner,
    gram,
    norm,
    add,
    scale,
    pad_ranks,
)
from .riemannian import (  # noqa: F401
    qr_pos,
    orthogonalize_lr,
    orthogonalize_rl,
    project_sparse_cores,
    tangent_cores,
    tangent_tt,
    project_sparse,
    round_tt,
    completion_step,
    left_interface,
    right_interface,
    dense_projector,
    observed_loss,
    riemannian_grad_dense,
)
from .ttmatrix import (  # noqa: F401
    ttm_full,
    ttm_forward,
    ttm_backward,
    tt_matvec,
    tt_matmat,
)
