"""MI355X (gfx950) Jacobi-PCG for the 3D seven-point Poisson operator.

The computation lives in libpcgmi.so (hand-written HIP, C ABI in
include/pcgmi.h); this package is its thin Python binding. Importing it
requires the built library and raises otherwise.
"""
from ._binding import (  # noqa: F401
    Batch, pcg_batch_create, pcg_batch_destroy, pcg_batch_set_barrier, pcg_batch_set_restarts, pcg_batch_solve,
    Cnn, cnn_adam_step, cnn_create, cnn_forward, cnn_get_adam, cnn_get_weights, cnn_set_adam, cnn_loss_grad, cnn_num_weights, cnn_set_operator, cnn_set_loss_norm, cnn_set_weights,
    cnn_train_step,
    DT_TORCH, LIBPATH, PCG_BF16, PCG_E_ARG, PCG_E_BREAKDOWN, PCG_E_HIP, PCG_E_NOCONV, PCG_E_NOMEM,
    PCG_E_TRUE_RESIDUAL, PCG_E_UNSUPPORTED, PCG_F16, SOLVE_OUTCOMES, STATUS_NAMES, PCG_F32, PCG_F64, PCG_OK, Context, PcgError, PcgInfo, PcgOptions, axpy,
    dot, dot_f64, dot_noalloc, dtype_code, lib, pcg_create, pcg_destroy, pcg_get_history, pcg_last_error,
    pcg_options_default, pcg_make_pairs, pcg_refine_history, pcg_set_coefficients, pcg_solve, pcg_solve_flexible, pcg_solve_refined,
    pcg_solve_snapshots, stencil_apply, pcg_set_multigrid, pcg_mg_levels, pcg_mg_apply, pcg_solve_mg,
    REFINE_RTOL_INNER, Sell, pcg_sell_build, pcg_sell_create, pcg_sell_destroy, pcg_sell_set_graph, pcg_sell_set_restarts, pcg_sell_solve, pcg_sell_spmv)
