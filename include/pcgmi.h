/*
 * pcgmi.h -- C ABI of the MI355X (gfx950) Jacobi-PCG library.
 *
 * The method (paper Sec. VII): preconditioned conjugate gradients for the 3D
 * seven-point finite-difference operator with zero Dirichlet boundaries,
 *   (A x)_{i,j,k} = 6 x_{i,j,k} - x_{i+-1,j,k} - x_{i,j+-1,k} - x_{i,j,k+-1},
 * neighbours outside the grid reading as 0 (no h^2 scaling), applied
 * matrix-free (Sec. VI), with the Jacobi preconditioner D = diag(A) applied
 * as element-wise scaling. PCG is composed of the element-wise update
 * (Sec. IV), the global dot-product reduction (Sec. V) and the stencil
 * (Sec. VI); here they are fused into two kernels per iteration, or into one
 * kernel with one grid reduction on small grids (pcg_options.single_reduction).
 *
 * Conventions for every entry point:
 *  - Grids are contiguous C-order [nz][ny][nx] arrays, x fastest.
 *  - Every data pointer is a DEVICE pointer on the context's device, owned
 *    by the caller, 16-byte aligned (PCG_E_ARG otherwise). The library owns
 *    only its workspace (allocated in *_create, freed in *_destroy).
 *  - Work is enqueued on the HIP stream given at creation (NULL = the
 *    default stream). stencil_apply, axpy and dot are asynchronous;
 *    pcg_solve returns after the solve has finished.
 *  - Calls return a status and never abort; the message of the last failure
 *    on the calling thread is available from pcg_last_error().
 *  - Calls on one context must not overlap (the workspace is shared).
 */
#ifndef PCGMI_H
#define PCGMI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pcg_ctx_s *pcg_ctx;

typedef enum {
    PCG_OK = 0,
    PCG_E_ARG = 1,         /* invalid argument: null/misaligned pointer, bad size, aliasing */
    PCG_E_HIP = 2,         /* a HIP runtime call failed */
    PCG_E_NOCONV = 3,      /* maxit reached; the last iterate is left in x */
    PCG_E_BREAKDOWN = 4,   /* p.Ap <= 0 or a non-finite scalar (e.g. NaN in b) */
    PCG_E_NOMEM = 5,       /* workspace allocation failed */
    PCG_E_UNSUPPORTED = 6, /* combination not implemented (e.g. dtype for an op) */
    PCG_E_TRUE_RESIDUAL = 7 /* the recursion met ||r|| <= rtol ||b||, but the FP64 true residual
                              ||b - A x|| / ||b|| of the returned x is still above rtol after the
                              allowed restarts; x holds that last iterate */
} pcg_status;

/* Storage type of the vectors. Arithmetic is FP32 for F32/BF16/F16 (values
 * widened on load, rounded to nearest-even on store) and FP64 for F64. */
typedef enum { PCG_F32 = 0, PCG_BF16 = 1, PCG_F16 = 2, PCG_F64 = 3 } pcg_dtype;

typedef struct {
    int chunk_iters;   /* iterations per captured HIP graph chunk (default 16, even) */
    int x_accum;       /* type of the x accumulator in the workspace: PCG_F64 (default,
                          -1 selects it), PCG_F32, or the storage type */
    int x_dtype;       /* type of the caller's x in pcg_solve: PCG_F32 (default for F32
                          storage) or PCG_F64; for BF16/F16 storage x is that type or F64 */
    int use_x0;        /* 0 (default): x0 = 0; 1: x holds the initial guess on entry */
    int use_graph;     /* 1 (default): replay captured graph chunks; 0: eager launches */
    int kernel_timing; /* 1: eager launches with HIP events around every iteration
                          kernel; sums are returned in pcg_info */
    int tile_x;        /* stencil tile in x (points); 0 = autotuned default */
    int tile_y;        /* stencil tile in y (rows); 0 = default */
    int zchunk;        /* z planes per work-group; 0 = default */
    int stag_window;   /* refinement's inner solves stop when the best ||r|| so far has
                          not improved by 10% for this many iterations; 0 = never;
                          -1 = default (100) */
    int max_restarts;  /* pcg_solve: when the recursion has converged but the FP64 true
                          residual ||b - A x|| > rtol ||b||, restart from x with r = b - A x
                          (computed in FP64, stored in the storage type) and beta = 0, at
                          most this many times; 0 = never; -1 = default (3) */
    int single_reduction; /* iteration form of pcg_solve / pcg_solve_refined with constant
                          coefficients: 0 = two kernels and two grid reductions per
                          iteration (Hestenes-Stiefel PCG); 1 = one fused kernel and one
                          reduction per iteration (Chronopoulos-Gear single-reduction
                          PCG, the same iterates in exact arithmetic; moves 48 instead of
                          40 bytes per point); -1 = default (chosen by grid size) */
    int zchunk_update;  /* z planes per work-group of the two-kernel form's update kernel
                          when it adds to x (every second iteration with x_defer = 1; the
                          other updates take the direction kernel's plan):
                          0 = default (twice the direction kernel's when r, p, p' and x
                          exceed the 256 MiB last-level cache and the launch keeps at least
                          256 work-groups, else the direction kernel's; the direction
                          kernel's when zchunk is given); -1 = the direction kernel's;
                          > 0 = this many */
    int x_defer;        /* two-kernel form: 1 (default) = the x accumulator advances every
                          second iteration (an odd iteration's update leaves x, the next
                          adds alpha_{k-1} p_{k-1} + alpha_k p_k; nothing in the recursion
                          reads x), so the update moves 12 and 32 bytes per point in turn
                          instead of 28 each time (FP32 storage, FP64 x); same bits of x
                          for an FP64 accumulator. 0 = x current after every iteration
                          (the same kernels plus one x += alpha p pass per iteration) */
} pcg_options;

typedef struct {
    int iters;               /* A p products of the solve (inner iterations for refinement) */
    int outer_iters;         /* refinement steps (pcg_solve_refined) */
    int fallback_used;       /* reserved for the flexible solver */
    int status;              /* pcg_status of the solve */
    double rel_res_recursive;/* ||r_k|| / ||b|| from the recursion */
    double rel_res_true_fp64;/* ||b - A x|| / ||b|| recomputed in FP64 on the GPU */
    double seconds;          /* host wall time of the call */
    double t_1e6;            /* refinement: seconds until the true residual <= 1e-6 */
    double t_1e10;           /* refinement: seconds until the true residual <= 1e-10 */
    double k1_ms, k2_ms;     /* kernel_timing: summed event time of the two iteration kernels
                                (pcg_solve; the inner solves of pcg_solve_refined) */
    int k1_launches, k2_launches;
    int restarts;            /* pcg_solve: FP64 residual restarts taken (max_restarts) */
    double k2_even_ms;       /* kernel_timing: the part of k2_ms spent in the updates of even
                                iterations (those that advance x; x_defer = 1) */
    int k2_even_launches;
} pcg_info;

/* Fill *opt with the defaults listed above. */
pcg_status pcg_options_default(pcg_options *opt);

/* Create a context for an nx*ny*nz grid whose vectors are stored as
 * `storage`. hip_stream is a hipStream_t (NULL = default stream). opt may be
 * NULL (defaults). Allocates the workspace: 3 vectors of the storage type
 * (r, p twice) plus the x accumulator (opt->x_accum), plus reduction
 * partials and a small scalar block. Errors: PCG_E_ARG (dims < 1 or
 * nx*ny*nz > 2^33), PCG_E_NOMEM, PCG_E_HIP. */
pcg_status pcg_create(pcg_ctx *out, int nx, int ny, int nz, pcg_dtype storage, void *hip_stream,
                      const pcg_options *opt);

/* Release the context and its workspace (waits for its stream). NULL is a no-op. */
pcg_status pcg_destroy(pcg_ctx ctx);

/* y = A x on the context's grid (paper Sec. VI), x and y of the storage type,
 * x != y (PCG_E_ARG when they overlap). FP32 math for F32/BF16/F16 storage,
 * FP64 for F64. */
pcg_status stencil_apply(pcg_ctx ctx, const void *x, void *y);

/* z = alpha x + y over n elements of the storage type (paper Sec. IV). alpha
 * is rounded once to the arithmetic type (FP32 for F32/BF16/F16 storage, kept
 * FP64 for F64). z may equal x or y; other partial overlaps are PCG_E_ARG.
 * n >= 0. */
pcg_status axpy(pcg_ctx ctx, int64_t n, double alpha, const void *x, const void *y, void *z);

/* *out_dev = sum_i x_i y_i over n elements of the storage type (paper Sec. V):
 * per-lane FP32 accumulation (FP64 for F64 storage), wavefront and
 * work-group reduction, then an FP64 sum of the work-group partials in a
 * fixed order by the last work-group to finish (deterministic). out_dev is a
 * DEVICE pointer to one float. n = 0 gives 0. */
pcg_status dot(pcg_ctx ctx, int64_t n, const void *x, const void *y, float *out_dev);

/* Same as dot with an FP64 device result. */
pcg_status dot_f64(pcg_ctx ctx, int64_t n, const void *x, const void *y, double *out_dev);

/* Allocation-free dot product, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the result of dot / dot_f64 (the same kernels and the same
 * summation order, so the same bits) over n elements of type `storage`, with
 * no context. x, y: DEVICE arrays, 16-byte aligned; out_f32 (DEVICE float) and
 * out_f64 (DEVICE double) receive the sum, either may be NULL but not both.
 * hip_stream: the stream to enqueue on (NULL = default stream), on the current
 * device. Asynchronous.
 * The work-group partials live in a fixed library-owned device array of 1024
 * doubles (8 KiB) per device, held until the process ends, instead of a
 * context's workspace; no hipMalloc, hipFree or other allocating call is made.
 * Limit: n <= PCG_DOT_NOALLOC_MAX_N (2^40), else PCG_E_ARG.
 * Calls that overlap on one device (on different streams or host threads)
 * share that array and race: serialize them. */
#define PCG_DOT_NOALLOC_MAX_N ((int64_t)1 << 40)
pcg_status dot_noalloc(pcg_dtype storage, int64_t n, const void *x, const void *y, float *out_f32, double *out_f64,
                       void *hip_stream);

/* Solve A x = b with Jacobi-PCG (paper Sec. VII): b of the storage type, x
 * of opt->x_dtype. Stops when the recursive residual satisfies
 * ||r|| <= rtol ||b|| or after maxit iterations (in total, restarts
 * included); then recomputes the true residual ||b - A x|| / ||b|| in FP64
 * and, while it exceeds rtol, restarts from x (opt->max_restarts).
 * b = 0 gives x = 0, iters = 0.
 * Returns PCG_OK only when that FP64 true residual is <= rtol;
 * PCG_E_TRUE_RESIDUAL when the recursion converged but the true residual is
 * still above rtol; PCG_E_NOCONV (maxit reached) or PCG_E_BREAKDOWN. In every
 * case the last iterate is left in x and info is filled.
 * info may be NULL. Blocks until the solve is finished. */
pcg_status pcg_solve(pcg_ctx ctx, const void *b, void *x, double rtol, int maxit, pcg_info *info);

/* Mixed-precision iterative refinement (Wilkinson 1963; Moler 1967) around
 * the paper's Jacobi-PCG (Sec. VII): b64 and x64 are FP64 device vectors on
 * the context's grid; the context's storage type (F32, BF16 or F16) is the
 * inner solver's. From x = 0:
 *   loop: r = b - A x in FP64 (GPU); stop when ||r|| / ||b|| <= rtol_outer
 *         or after max_outer corrections;
 *         s = 1 / max|r|; rhat = storage(s r) (FP64 -> FP32 -> storage,
 *         nearest even); inner Jacobi-PCG A d = rhat in the storage type with
 *         FP32 arithmetic, stopped at ||r_in|| <= rtol_inner ||rhat||, at
 *         maxit_inner, or when the best ||r_in|| has not improved by 10%
 *         for the context's stag_window iterations; d accumulates in the context's x_accum type (FP32
 *         keeps the correction accurate at large grids, where rounding d to
 *         16 bits costs about kappa(A) times its unit roundoff); x += d / s
 *         in FP64.
 * info: iters = total inner iterations, outer_iters, rel_res_true_fp64 (the
 * last FP64 residual), t_1e6 / t_1e10 = seconds until the FP64 residual
 * first reached 1e-6 / 1e-10 (-1 if never). Returns PCG_OK when the
 * tolerance was met, PCG_E_NOCONV otherwise (x holds the last iterate),
 * PCG_E_UNSUPPORTED for F64 storage. Blocks until done. */
pcg_status pcg_solve_refined(pcg_ctx ctx, const double *b64, double *x64, double rtol_outer, double rtol_inner,
                             int max_outer, int maxit_inner, pcg_info *info);

/* The last pcg_solve_refined's FP64 relative residual before each outer
 * step (relres, may be NULL) and the inner iterations of each step
 * (inner_iters, may be NULL), n entries at most; *count = entries written. */
pcg_status pcg_refine_history(pcg_ctx ctx, double *relres, int *inner_iters, int n, int *count);

/* Switch the context's operator to the variable-coefficient form
 * (A_k u)_p = sum over the six faces f of k_f (u_p - u_nb), with the face
 * coefficient k_f = 2 k_p k_q / (k_p + k_q) (harmonic mean of the two cell
 * values), k_f = k_p on a boundary face and u = 0 outside the grid; the
 * Jacobi preconditioner becomes D^-1 with D_p = sum_f k_f. This is the
 * paper's operator (Sec. VII) with k = 1 and the learned-preconditioner
 * workload's operator in general. k_cell: DEVICE array of nx*ny*nz FP32
 * cell values > 0, owned by the caller and read by later calls (keep it
 * alive and unchanged); NULL restores constant coefficients. Computes and
 * stores D^-1 in the workspace. Needs F32 or F64 storage
 * (PCG_E_UNSUPPORTED otherwise). Affects stencil_apply, pcg_solve and
 * pcg_solve_refined on this context. */
pcg_status pcg_set_coefficients(pcg_ctx ctx, const float *k_cell);

/* ------------------------------------------------------------------------
 * Geometric multigrid V-cycle preconditioner (the paper names multigrid as
 * future work for its solver, Sec. VIII); FP32 storage. The textbook
 * cell-centred V-cycle (Trottenberg, Oosterlee and Schueller, "Multigrid",
 * 2001; Wesseling 1992):
 *  - hierarchy: level l+1 halves every dimension of level l (a coarse cell
 *    is 2 x 2 x 2 fine cells) while all three are even and level l has more
 *    than coarse_max points; the coarsest grid may hold at most 1024 points
 *    (PCG_E_UNSUPPORTED otherwise);
 *  - coarse operators by rediscretisation: the seven-point operator of the
 *    coarse grid, 4^-l A[k_l] (the unscaled operator's h^2 factor follows
 *    the doubled spacing), with k_l the mean of the children's k (constant
 *    coefficients stay constant);
 *  - prolongation P: per dimension 3/4 of the coarse cell holding a fine cell
 *    and 1/4 of the coarse cell on its other side (0 outside the grid),
 *    restriction R = P^T / 8;
 *  - smoother: damped Jacobi u += omega D^-1 (f - A u), nu sweeps before and
 *    nu after the coarse correction, from u = 0; coarsest level: exact solve
 *    (dense inverse, formed once in FP64 on the host).
 * With equal sweeps before and after, the V-cycle is symmetric positive
 * definite.
 * ------------------------------------------------------------------------ */

/* Build the hierarchy for the context's current operator (constant, or the
 * coefficients of pcg_set_coefficients, which rebuilds it when they change).
 * nu in 1..8 (sweeps on each side), omega in (0, 1] (0 = default 6/7, the best
 * damping of the 3-D seven-point operator's high frequencies), coarse_max >= 0
 * (0 = default 512). Allocates per level: the fine level 2-3 vectors, every
 * coarser one 4-5 of its size, plus the coarsest inverse. Needs F32 storage. */
pcg_status pcg_set_multigrid(pcg_ctx ctx, int nu, double omega, int coarse_max);

/* Levels of the hierarchy (*nlev) and their dims (dims: host int[3 * nlev],
 * {nx, ny, nz} finest first; may be NULL). */
pcg_status pcg_mg_levels(pcg_ctx ctx, int *nlev, int *dims);

/* u = V-cycle(g) on the context's grid: g and u DEVICE FP32 arrays of nx*ny*nz
 * values, not overlapping; asynchronous on the context's stream. */
pcg_status pcg_mg_apply(pcg_ctx ctx, const float *g, float *u);

/* PCG with the V-cycle as preconditioner: pcg_solve_flexible's iteration
 * (Notay's flexible CG with one stored direction, which equals PCG for a
 * fixed symmetric preconditioner) with M(r) = V-cycle(r); b FP32, x of
 * opt->x_dtype, FP64 x accumulator; stops on ||r|| <= rtol ||b||, then the
 * FP64 true residual judges: while it is above rtol the same method restarts
 * from x with r = fl32(b - A x) computed in FP64 (at most opt->max_restarts
 * times; info.restarts); PCG_OK only when it is <= rtol, else
 * PCG_E_TRUE_RESIDUAL; PCG_E_NOCONV, PCG_E_BREAKDOWN. A V-cycle output with
 * z.r <= 0 (not expected) switches to Jacobi as in pcg_solve_flexible
 * (info.fallback_used). PCG_E_ARG without pcg_set_multigrid. */
pcg_status pcg_solve_mg(pcg_ctx ctx, const void *b, void *x, double rtol, int maxit, pcg_info *info);

/* Copy the recursive relative residuals ||r_k||/||b||, k = 0..iters of the
 * last pcg_solve on this context, to the host array hist (n entries at most).
 * *count receives the number written. */
pcg_status pcg_get_history(pcg_ctx ctx, double *hist, int n, int *count);

/* ------------------------------------------------------------------------
 * Learned preconditioner (not in the paper): a 3D CNN z = rms(r) N(r / rms(r), g)
 * with four 3x3x3 convolution layers 2 -> 16 -> 16 -> 16 -> 1, zero
 * padding, ReLU after the first three, no bias. Input channels: the scaled
 * residual and g (the standardised log-coefficient field). Weights: FP32
 * master copy, packed as W1[27][2][16], W2[27][16][16], W3[27][16][16],
 * W4[27][16][1] (tap t = 9 dz + 3 dy + dx, offsets -1..1), 15120 floats;
 * computed with BF16 weights and activations and FP32 accumulation on the
 * matrix cores. Activations live in the network object, sized for the last
 * grid used.
 * ------------------------------------------------------------------------ */
typedef struct cnn_s *cnn_net;

/* Create a network (weights zero) whose work is enqueued on hip_stream. */
pcg_status cnn_create(cnn_net *out, void *hip_stream);
/* Release the network (waits for its stream). NULL is a no-op. */
pcg_status cnn_destroy(cnn_net net);
/* Number of weights (15120). */
int cnn_num_weights(void);
/* Copy the 15120 FP32 master weights from / to a DEVICE buffer. Setting
 * weights resets the Adam moments and step count. */
pcg_status cnn_set_weights(cnn_net net, const float *w_dev);
pcg_status cnn_get_weights(cnn_net net, float *w_dev);
/* Training checkpoint: Adam's state (Kingma & Ba 2015), the first and second
 * moment estimates (15120 FP32 values each, DEVICE buffers) and the step
 * count. cnn_get_adam copies them out (step may be NULL); cnn_set_adam
 * restores them (call it after cnn_set_weights, which resets them), so that
 * training resumes exactly where the checkpoint was taken. Errors: PCG_E_ARG
 * for a null network or buffer or a step outside [0, 2^31). Both enqueue on
 * the network's stream. */
pcg_status cnn_get_adam(cnn_net net, float *m_dev, float *v_dev, int64_t *step);
pcg_status cnn_set_adam(cnn_net net, const float *m_dev, const float *v_dev, int64_t step);
/* z = s N(r / s, g) on an nx*ny*nz grid: r of type rdt (F32, F64 or BF16),
 * g FP32 (NULL: zero channel), z FP32, all DEVICE arrays of nx*ny*nz
 * values. rr_dev: DEVICE pointer to ||r||^2 (FP64) giving s = rms(r) =
 * sqrt(rr / (nx ny nz)); NULL means s = 1 (the raw network). */
pcg_status cnn_forward(cnn_net net, int nx, int ny, int nz, pcg_dtype rdt, const void *r, const float *g,
                       const double *rr_dev, float *z);
/* Mean loss over a batch of training pairs and its gradient with respect to
 * the master weights. pairs: DEVICE BF16 array [batch][2][nx*ny*nz] holding,
 * per pair, the network input channel (the scaled residual rh) and the
 * target (the scaled error eh); g as in cnn_forward. Loss per pair:
 *  - no operator set (cnn_set_operator): relative MSE ||N - eh||^2 / ||eh||^2;
 *  - operator A with Jacobi scale D^-1 set: the A-norm error of the
 *    preconditioner D^-1 rh + N (the form pcg_solve_flexible applies),
 *    u = N + D^-1 rh - eh, loss u.A u / (rh.D^-1 rh); the normaliser makes
 *    every residual count alike, whatever its smoothness.
 * grad_dev: DEVICE FP32[15120] (NULL: the network's own gradient buffer);
 * loss_dev: DEVICE double (may be NULL). */
pcg_status cnn_loss_grad(cnn_net net, int nx, int ny, int nz, const void *pairs, const float *g, int batch,
                         float *grad_dev, double *loss_dev);
/* Use the A-norm loss with ctx's operator (an F32 context on the training
 * grid, on the network's stream, with the coefficients of the problem the
 * pairs come from); NULL restores the relative-MSE loss. The context must
 * outlive its use here. */
pcg_status cnn_set_operator(cnn_net net, pcg_ctx ctx);
/* Normaliser of the A-norm loss: mode 0 (default) rh.D^-1 rh; mode 1 rh.eh,
 * which is the error's energy eh.A eh when rh = A eh (pairs from a solve:
 * r = b - A x and e = x* - x), so every pair counts by its relative A-norm
 * error whatever its smoothness. PCG_E_ARG for another mode. */
pcg_status cnn_set_loss_norm(cnn_net net, int mode);
/* One Adam step (lr, beta = (0.9, 0.999), eps = 1e-8, bias-corrected) on the
 * master weights with gradient grad_dev (NULL: the network's own). */
pcg_status cnn_adam_step(cnn_net net, const float *grad_dev, float lr);
/* cnn_loss_grad followed by cnn_adam_step. */
pcg_status cnn_train_step(cnn_net net, int nx, int ny, int nz, const void *pairs, const float *g, int batch,
                          float lr, double *loss_dev);

/* Flexible CG (Notay 2000, one stored direction) with preconditioner
 * M(r) = D^-1 r + rms(r) N(r / rms(r), g): Jacobi plus the network's
 * correction (cnn_forward with ||r||^2), so a network with zero output is
 * Jacobi; when net is NULL, M = D^-1 (then FCG reproduces Jacobi-PCG):
 *   q = A p; sigma = p.q; alpha = (p.r)/sigma; x += alpha p; r -= alpha q;
 *   stop on ||r|| <= rtol ||b||; z = M(r); beta = -(z.q)/sigma; p = z + beta p.
 * Fallback: M switches to D^-1 for the rest of the solve (restarting the
 * direction recurrence) when z.r <= 0, a value is not finite, or the best
 * residual has not improved by 10% for 100 iterations. When the recursion has
 * converged, the FP64 true residual judges: above rtol, Jacobi-PCG continues
 * from the current x. The context needs F32 storage and an FP64 x
 * accumulator; the network must use the context's stream; g: DEVICE FP32
 * network channel (may be NULL). info: fallback_used = 0 (none), 1 (switched
 * to Jacobi; outer_iters = the iteration), 2 (Jacobi-PCG continuation).
 * Returns PCG_OK only when the final FP64 true residual is <= rtol, else
 * PCG_E_TRUE_RESIDUAL, PCG_E_NOCONV or PCG_E_BREAKDOWN (x holds the last
 * iterate in every case). */
pcg_status pcg_solve_flexible(pcg_ctx ctx, cnn_net net, const float *g, const void *b, void *x, double rtol,
                              int maxit, pcg_info *info);

/* Jacobi-PCG from x0 = 0 that also records (r_k, x_k) after the iterations
 * listed in snap_iters (host array, increasing, nsnap entries): r_snaps
 * receives nsnap vectors of the storage type, x_snaps nsnap vectors of the
 * accumulator type (= x_dtype, which must equal x_accum). Snapshots past
 * convergence hold the final state. Used to generate (residual, error)
 * training pairs from the FP64 solver. */
pcg_status pcg_solve_snapshots(pcg_ctx ctx, const void *b, void *x, double rtol, int maxit, const int *snap_iters,
                               int nsnap, void *r_snaps, void *x_snaps, pcg_info *info);

/* Training pairs from FP64 snapshots (F64 context): for each j, rho =
 * rms(r_j), pairs[j] = (bf16(r_j / rho), bf16((x_star - x_j) / rho)), laid
 * out as DEVICE BF16 [npairs][2][nx*ny*nz] (the layout cnn_loss_grad reads). */
pcg_status pcg_make_pairs(pcg_ctx ctx, int npairs, const double *r_snaps, const double *x_snaps,
                          const double *x_star, void *pairs);

/* ------------------------------------------------------------------------
 * Batched solves: many independent constant-coefficient problems (the
 * Jacobi-PCG of Sec. VII on grids of different sizes, FP32 vectors, FP64 x,
 * x0 = 0) in ONE persistent kernel launch. Batching is not part of the
 * paper's method; the per-problem iteration is the single-problem solver's.
 *
 * Every work-group of the launch belongs to one problem; a problem's
 * work-groups form a group on one XCD that meets at group barriers twice per
 * iteration. The kernel reads each work-group's XCD from the hardware and,
 * when a group is really on one XCD, synchronises it through that XCD's L2
 * without agent-scope fences. The grid is the device's resident capacity (occupancy query), so
 * all groups run concurrently. Each problem is laid out contiguously, C-order
 * [nz][ny][nx], at its offset in two caller-owned DEVICE arenas: b (FP32) and
 * x (FP64), each of `total` elements (pcg_batch_layout).
 *
 * Internally every problem's r, p and x live in arenas whose rows are padded
 * to a multiple of 4 points (padding held at 0), so 4-wide vector tiles work
 * for any nx; b is read from and x written to the caller's layout.
 *
 * Tile plans: per problem a work-group tile shape (cfg 0: 64x16 points,
 * 1: 128x8, 2: 256x4, all 4-wide FP32 vectors; 5: 64x4 scalar) and a
 * z-chunk. The z-chunk follows from the shape and the
 * group size (fewest planes for the busiest work-group). The shape is given
 * by the caller, read from the JSON tile cache, or measured: the autotuner
 * runs `tune_iters` iterations of every problem still without a shape under
 * each candidate shape (all problems in one launch, twice), keeps for each
 * problem the shape with the shortest wall-clock time, and records it in the
 * cache keyed by device, problem shape and group size.
 * ------------------------------------------------------------------------ */
typedef struct pcg_batch_s *pcg_batch;

/* Create a batch of nprob problems; dims = host int[nprob][3] {nx, ny, nz}
 * (each >= 1, at most 2^31 points). cfgs = host int[nprob] tile shapes (0, 1,
 * 2 or 5), or NULL to use the cache / the
 * autotuner. cache_path: JSON file read and rewritten by the autotuner (NULL:
 * no cache). tune_iters: iterations per tuning launch (<= 0: 20). Allocates
 * the workspace (3 FP32 and 1 FP64 row-padded arenas, per-problem scalars). PCG_E_UNSUPPORTED if
 * more problems than resident work-groups fall on one XCD. */
pcg_status pcg_batch_create(pcg_batch *out, int nprob, const int *dims, const int *cfgs,
                            const char *cache_path, int tune_iters, void *hip_stream);
/* Release the batch (waits for its stream). NULL is a no-op. */
pcg_status pcg_batch_destroy(pcg_batch batch);

/* Host outputs, each optional (NULL): offsets int64[nprob] (element offset of
 * each problem in the arenas, a multiple of 64), total (arena length),
 * plans int[nprob][4] {cfg, zc, work-groups, tiles}, grid int[3]
 * {work-groups of the launch, problems whose shape was measured, problems
 * whose group barriers ran in the XCD-local form in the last solve (all of
 * them when every work-group ran on the XCD the layout assigns it; otherwise
 * those groups use agent-scope fences)}. */
pcg_status pcg_batch_layout(pcg_batch batch, int64_t *offsets, int64_t *total, int *plans, int *grid);

/* Group-barrier form of later solves: 0 (default) = XCD-local where a group's
 * work-groups all run on one XCD, agent-scope fences otherwise; 1 = agent-scope
 * release / acquire fences for every group (the general form, slower; the
 * same arithmetic, so the same results). PCG_E_ARG for another value. */
pcg_status pcg_batch_set_barrier(pcg_batch batch, int form);

/* FP64-residual restarts per problem in later solves: 0 = never (each
 * recursion alone decides, as the oracle's Jacobi-PCG does), -1 = default (3). */
pcg_status pcg_batch_set_restarts(pcg_batch batch, int max_restarts);

/* Solve all problems from x0 = 0 with Jacobi-PCG until ||r_i|| <= rtol ||b_i||
 * (recursive residual) or maxit iterations in total. When a problem's
 * recursion stops, its FP64 true residual b - A x is computed; if that is
 * still above rtol ||b_i||, the problem restarts from x with r = fl32(b - A x)
 * and beta = 0 (at most 3 times, pcg_batch_set_restarts), as pcg_solve does. b: DEVICE FP32 arena
 * (read only); x: DEVICE FP64 arena (written). use_graph = 1 captures
 * [barrier reset, persistent kernel] in a HIP graph on the first call and
 * replays it while (b, x, rtol, maxit) stay the same. Host outputs (NULL to
 * skip): iters int[nprob] (restarts included), relres double[nprob] (FP64
 * ||b - A x|| / ||b||), latency_s double[nprob] (device wall clock from the
 * earliest problem's start to this problem's end), restarts int[nprob],
 * seconds (host wall time of the call). Returns after the launch has ended;
 * The status is the worst over the problems: PCG_E_BREAKDOWN, then
 * PCG_E_NOCONV (maxit), then PCG_E_TRUE_RESIDUAL (a recursion converged but
 * its FP64 true residual is above rtol after the restarts); outputs are
 * written in every case. PCG_E_HIP if a group barrier wait exceeded its bound. */
pcg_status pcg_batch_solve(pcg_batch batch, const float *b, double *x, double rtol, int maxit, int use_graph,
                           int *iters, double *relres, double *latency_s, int *restarts, double *seconds);

/* ------------------------------------------------------------------------
 * General sparse matrices: SpMV in sliced ELLPACK (SELL-C-sigma).
 *
 * Sec. VII-A builds its GPU comparison system's CG from norm, dot, axpy and
 * SpMV, with the seven-point operator stored as a general sparse matrix in a
 * sliced-ELLPACK format. These entry points take any matrix in compressed-row
 * form: row i holds values[k] at column colidx[k] for rowptr[i] <= k <
 * rowptr[i+1] (rowptr[0] = 0, rowptr non-decreasing, 0 <= colidx < ncols).
 *
 * Layout (SELL-C-sigma of Kreutzer, Hager, Wellein, Fehske and Bishop, SIAM
 * J. Sci. Comput. 36(5), 2014): rows are sorted by decreasing length inside
 * windows of sigma consecutive rows (a stable sort: equal lengths keep their
 * order; sigma = 1 keeps the original order), then cut into chunks of C
 * consecutive sorted rows. Chunk c stores width_c slots per row, width_c
 * being the longest row of the chunk, column-major: entry j of the chunk's
 * row l is slot chunk_ptr[c] + j * C + l. A row keeps its entries in storage
 * order; padding slots hold column -1 and value 0. perm[s] is the original
 * row at sorted position s.
 * ------------------------------------------------------------------------ */
typedef struct pcg_sell_s *pcg_sell;

/* Host-only layout of a compressed-row matrix (all pointers HOST). chunk >= 1;
 * sigma = 1 or a multiple of chunk; nrows, ncols in [0, 2^31 - 1]. First call
 * with chunk_ptr, perm, col_out and val_out all NULL: fills *nchunks
 * (ceil(nrows / chunk)) and *nslots (total slots). Second call with
 * chunk_ptr int64[nchunks + 1], perm int32[nrows], col_out int32[nslots] and
 * val_out float[nslots]. PCG_E_ARG for an inconsistent rowptr or a column
 * out of range. No GPU call is made. */
pcg_status pcg_sell_build(int64_t nrows, int64_t ncols, const int64_t *rowptr, const int32_t *colidx,
                          const float *values, int chunk, int sigma, int64_t *nchunks, int64_t *nslots,
                          int64_t *chunk_ptr, int32_t *perm, int32_t *col_out, float *val_out);

/* Build the layout with C = 64 (one wavefront per chunk) from HOST arrays
 * and copy it to device memory that the handle owns (freed by
 * pcg_sell_destroy). hip_stream: the stream the SpMV runs on (NULL: the null
 * stream). PCG_E_NOMEM if the device memory cannot be allocated. */
pcg_status pcg_sell_create(pcg_sell *out, int64_t nrows, int64_t ncols, const int64_t *rowptr,
                           const int32_t *colidx, const float *values, int sigma, void *hip_stream);
/* Release the matrix's device memory. NULL is a no-op. */
pcg_status pcg_sell_destroy(pcg_sell A);
/* Host outputs, each optional: stored entries, slots (padding included),
 * chunks. */
pcg_status pcg_sell_info(pcg_sell A, int64_t *nnz, int64_t *nslots, int64_t *nchunks);

/* y = A x on the handle's stream, asynchronous. x: DEVICE float[ncols]; y:
 * DEVICE float[nrows], 4-byte aligned, not overlapping x (PCG_E_ARG). Each
 * row is summed in FP32 with fused multiply-adds over its entries in storage
 * order, starting from 0. */
pcg_status pcg_sell_spmv(pcg_sell A, const float *x, float *y);

/* Jacobi-PCG on a square stored matrix (symmetric positive definite, with a
 * positive diagonal), the CG of Sec. VII-A's comparison system built on this
 * SpMV: the steps of pcg_solve (Hestenes-Stiefel PCG, Saad Alg. 9.1, M = D,
 * D_i = the sum of row i's entries in column i) from x0 = 0 until the
 * recursive ||r|| <= rtol ||b|| or maxit A p products. r, p, q and D^-1 are
 * FP32, the products and updates FP32, the inner products accumulated in
 * FP64, x accumulated in FP64. When the recursion has converged but the FP64
 * true residual ||b - A x|| is above rtol ||b||, the solve restarts from x
 * with r = fl32(b - A x) (at most 3 times; pcg_sell_set_restarts). b: DEVICE float[n]; x: DEVICE
 * double[n] (written). The first call allocates the workspace (4 FP32 vectors)
 * and checks the diagonal: PCG_E_ARG if a row's diagonal is missing or not
 * positive. Returns after the solve with info filled (iters, status,
 * rel_res_recursive, rel_res_true_fp64, restarts, seconds); PCG_OK only when
 * the FP64 true residual is <= rtol; PCG_E_TRUE_RESIDUAL (the recursion
 * converged, the true residual did not), PCG_E_NOCONV or PCG_E_BREAKDOWN
 * (p.Ap <= 0 or a non-finite value) keep the last iterate in x. Iterations are enqueued 16 at a time; the kernels of iterations past the
 * end return at once. */
pcg_status pcg_sell_solve(pcg_sell A, const float *b, double *x, double rtol, int maxit, pcg_info *info);
/* use_graph = 1 (default): full batches of 16 iterations are captured once
 * as a HIP graph on a private stream and replayed (recaptured when x
 * changes); 0: every kernel is launched eagerly. Same results either way. */
pcg_status pcg_sell_set_graph(pcg_sell A, int use_graph);
/* FP64-residual restarts of pcg_sell_solve after the recursion has converged:
 * 0 = never (the recursion alone decides when to stop, as the oracle's
 * Jacobi-PCG does), -1 = default (3). PCG_E_ARG below -1. */
pcg_status pcg_sell_set_restarts(pcg_sell A, int max_restarts);

/* Message of the last failed call on this thread ("" if none). */
const char *pcg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PCGMI_H */
