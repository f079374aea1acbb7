"""PISCO subspace sensitivity-map estimation on MI355X (gfx950).

The computation lives in libpisco.so (HIP kernels behind the C ABI of
include/pisco.h); this package is its Python binding plus a small pipeline
helper that allocates device buffers with torch.
"""
from ._lib import (  # noqa: F401
    Handle, Opts, PiscoError, Problem, lib, make_opts, make_problem, pisco_eig,
    pisco_eig_checked, pisco_eig_from, pisco_eig_sets, pisco_eig_sets_workspace_size, pisco_espirit_operator, pisco_estimate, pisco_gram, pisco_gram_static,
    pisco_gram_static_bytes, pisco_gx, pisco_llr_svd, pisco_maps, pisco_nullspace, pisco_nullspace_block,
    pisco_support, pisco_support_mask, pisco_status_string, pisco_trace_enable, pisco_trace_read,
    pisco_workspace_size, pisco_ws_forward, pisco_ws_init, pisco_ws_neighbor,
    pisco_ws_param_count, pisco_ws_train_step, pisco_ws_workspace_size)
from .pipeline import Estimator  # noqa: F401
from .warmstart import WarmStart, coarse_grid  # noqa: F401
from .batch import Batch  # noqa: F401
