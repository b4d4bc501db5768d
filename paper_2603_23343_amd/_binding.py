"""ctypes binding of the C ABI in include/pcgmi.h.

Argument marshalling only: torch tensors supply device pointers and the HIP
stream; every step of the computation runs in the library's HIP kernels. The
library must have been built (paper_2603_23343_amd/build.py); importing this
module without it raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

import torch  # loads the HIP runtime the library binds to

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "libpcgmi.so")

(PCG_OK, PCG_E_ARG, PCG_E_HIP, PCG_E_NOCONV, PCG_E_BREAKDOWN, PCG_E_NOMEM, PCG_E_UNSUPPORTED,
 PCG_E_TRUE_RESIDUAL) = range(8)
# Outcomes of a solve that still fill its outputs (raise_on_error=False returns them).
SOLVE_OUTCOMES = (PCG_E_NOCONV, PCG_E_BREAKDOWN, PCG_E_TRUE_RESIDUAL)
PCG_F32, PCG_BF16, PCG_F16, PCG_F64 = range(4)

STATUS_NAMES = {0: "PCG_OK", 1: "PCG_E_ARG", 2: "PCG_E_HIP", 3: "PCG_E_NOCONV", 4: "PCG_E_BREAKDOWN",
                5: "PCG_E_NOMEM", 6: "PCG_E_UNSUPPORTED", 7: "PCG_E_TRUE_RESIDUAL"}

_TORCH_DT = {torch.float32: PCG_F32, torch.bfloat16: PCG_BF16, torch.float16: PCG_F16, torch.float64: PCG_F64}
DT_TORCH = {v: k for k, v in _TORCH_DT.items()}


class PcgOptions(ctypes.Structure):
    _fields_ = [("chunk_iters", ctypes.c_int), ("x_accum", ctypes.c_int), ("x_dtype", ctypes.c_int),
                ("use_x0", ctypes.c_int), ("use_graph", ctypes.c_int), ("kernel_timing", ctypes.c_int),
                ("tile_x", ctypes.c_int), ("tile_y", ctypes.c_int), ("zchunk", ctypes.c_int),
                ("stag_window", ctypes.c_int), ("max_restarts", ctypes.c_int), ("single_reduction", ctypes.c_int),
                ("zchunk_update", ctypes.c_int), ("x_defer", ctypes.c_int)]


class PcgInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("outer_iters", ctypes.c_int), ("fallback_used", ctypes.c_int),
                ("status", ctypes.c_int), ("rel_res_recursive", ctypes.c_double),
                ("rel_res_true_fp64", ctypes.c_double), ("seconds", ctypes.c_double),
                ("t_1e6", ctypes.c_double), ("t_1e10", ctypes.c_double), ("k1_ms", ctypes.c_double),
                ("k2_ms", ctypes.c_double), ("k1_launches", ctypes.c_int), ("k2_launches", ctypes.c_int),
                ("restarts", ctypes.c_int), ("k2_even_ms", ctypes.c_double), ("k2_even_launches", ctypes.c_int)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class PcgError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def _load():
    if not os.path.exists(LIBPATH):
        raise ImportError(f"{LIBPATH} is not built; run paper_2603_23343_amd/build.py (or __graft_entry__.build())")
    lib = ctypes.CDLL(LIBPATH)
    vp, i, i64, d, f = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_float
    sig = {
        "pcg_options_default": ([ctypes.POINTER(PcgOptions)], i),
        "pcg_create": ([ctypes.POINTER(vp), i, i, i, i, vp, ctypes.POINTER(PcgOptions)], i),
        "pcg_destroy": ([vp], i),
        "stencil_apply": ([vp, vp, vp], i),
        "axpy": ([vp, i64, d, vp, vp, vp], i),
        "dot": ([vp, i64, vp, vp, vp], i),
        "dot_f64": ([vp, i64, vp, vp, vp], i),
        "dot_noalloc": ([i, i64, vp, vp, vp, vp, vp], i),
        "pcg_solve": ([vp, vp, vp, d, i, ctypes.POINTER(PcgInfo)], i),
        "pcg_get_history": ([vp, ctypes.POINTER(d), i, ctypes.POINTER(i)], i),
        "pcg_solve_refined": ([vp, vp, vp, d, d, i, i, ctypes.POINTER(PcgInfo)], i),
        "pcg_refine_history": ([vp, ctypes.POINTER(d), ctypes.POINTER(i), i, ctypes.POINTER(i)], i),
        "pcg_last_error": ([], ctypes.c_char_p),
        "pcg_set_coefficients": ([vp, vp], i),
        "pcg_solve_flexible": ([vp, vp, vp, vp, vp, d, i, ctypes.POINTER(PcgInfo)], i),
        "pcg_set_multigrid": ([vp, i, d, i], i),
        "pcg_mg_levels": ([vp, ctypes.POINTER(i), ctypes.POINTER(i)], i),
        "pcg_mg_apply": ([vp, vp, vp], i),
        "pcg_solve_mg": ([vp, vp, vp, d, i, ctypes.POINTER(PcgInfo)], i),
        "pcg_solve_snapshots": ([vp, vp, vp, d, i, ctypes.POINTER(i), i, vp, vp, ctypes.POINTER(PcgInfo)], i),
        "pcg_make_pairs": ([vp, i, vp, vp, vp, vp], i),
        "cnn_create": ([ctypes.POINTER(vp), vp], i),
        "cnn_destroy": ([vp], i),
        "cnn_num_weights": ([], i),
        "cnn_set_weights": ([vp, vp], i),
        "cnn_get_weights": ([vp, vp], i),
        "cnn_get_adam": ([vp, vp, vp, ctypes.POINTER(i64)], i),
        "cnn_set_adam": ([vp, vp, vp, i64], i),
        "cnn_forward": ([vp, i, i, i, i, vp, vp, vp, vp], i),
        "cnn_loss_grad": ([vp, i, i, i, vp, vp, i, vp, vp], i),
        "cnn_adam_step": ([vp, vp, ctypes.c_float], i),
        "cnn_train_step": ([vp, i, i, i, vp, vp, i, ctypes.c_float, vp], i),
        "cnn_set_operator": ([vp, vp], i),
        "cnn_set_loss_norm": ([vp, i], i),
        "pcg_batch_create": ([ctypes.POINTER(vp), i, ctypes.POINTER(i), ctypes.POINTER(i), ctypes.c_char_p, i, vp], i),
        "pcg_batch_destroy": ([vp], i),
        "pcg_batch_set_barrier": ([vp, i], i),
        "pcg_batch_set_restarts": ([vp, i], i),
        "pcg_batch_layout": ([vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i), ctypes.POINTER(i)], i),
        "pcg_batch_solve": ([vp, vp, vp, d, i, i, ctypes.POINTER(i), ctypes.POINTER(d), ctypes.POINTER(d),
                             ctypes.POINTER(i), ctypes.POINTER(d)], i),
        "pcg_sell_build": ([i64, i64, vp, vp, vp, i, i, ctypes.POINTER(i64), ctypes.POINTER(i64), vp, vp, vp, vp], i),
        "pcg_sell_create": ([ctypes.POINTER(vp), i64, i64, vp, vp, vp, i, vp], i),
        "pcg_sell_destroy": ([vp], i),
        "pcg_sell_info": ([vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)], i),
        "pcg_sell_spmv": ([vp, vp, vp], i),
        "pcg_sell_solve": ([vp, vp, vp, d, i, ctypes.POINTER(PcgInfo)], i),
        "pcg_sell_set_graph": ([vp, i], i),
        "pcg_sell_set_restarts": ([vp, i], i),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


lib = _load()


def pcg_last_error() -> str:
    return lib.pcg_last_error().decode()


def _check(status):
    if status != PCG_OK:
        raise PcgError(status, pcg_last_error())


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return ctypes.c_void_p(t.data_ptr())


def _need(t, n, name, dtype=None):
    """A device tensor with at least n contiguous elements (of dtype)."""
    if t is None or isinstance(t, int):
        return
    if not t.is_cuda or not t.is_contiguous():
        raise PcgError(PCG_E_ARG, f"{name}: expected a contiguous device tensor")
    if t.numel() < n:
        raise PcgError(PCG_E_ARG, f"{name}: {t.numel()} elements, need {n}")
    if dtype is not None and t.dtype != dtype:
        raise PcgError(PCG_E_ARG, f"{name}: dtype {t.dtype}, need {dtype}")


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def dtype_code(dt) -> int:
    if isinstance(dt, int):
        return dt
    return _TORCH_DT[dt]


def pcg_options_default(**overrides) -> PcgOptions:
    o = PcgOptions()
    _check(lib.pcg_options_default(ctypes.byref(o)))
    for k, v in overrides.items():
        if k in ("x_dtype", "x_accum"):
            v = dtype_code(v)
        setattr(o, k, int(v))
    return o


class Context:
    """Owns a pcg_ctx handle; destroyed with the object (or close())."""

    def __init__(self, handle, nx, ny, nz, dtype, stream):
        self.handle = handle
        self.shape = (nz, ny, nx)
        self.dtype = dtype
        self.stream = stream

    @property
    def n(self):
        nz, ny, nx = self.shape
        return nx * ny * nz

    def close(self):
        if self.handle:
            lib.pcg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def _as_parameter_(self):
        return self.handle


def pcg_create(nx, ny, nz, dtype=torch.float32, stream=None, options=None, **opts) -> Context:
    if options is None and opts:
        options = pcg_options_default(**opts)
    h = ctypes.c_void_p()
    s = _stream(stream)
    _check(lib.pcg_create(ctypes.byref(h), int(nx), int(ny), int(nz), dtype_code(dtype), s,
                          None if options is None else ctypes.byref(options)))
    return Context(h, int(nx), int(ny), int(nz), dtype, s)


def pcg_destroy(ctx: Context):
    ctx.close()


def stencil_apply(ctx: Context, x, y):
    _need(x, ctx.n, "x", ctx.dtype)
    _need(y, ctx.n, "y", ctx.dtype)
    _check(lib.stencil_apply(ctx.handle, _ptr(x), _ptr(y)))


def axpy(ctx: Context, n, alpha, x, y, z):
    for t, nm in ((x, "x"), (y, "y"), (z, "z")):
        _need(t, n, nm, ctx.dtype)
    _check(lib.axpy(ctx.handle, int(n), float(alpha), _ptr(x), _ptr(y), _ptr(z)))  # alpha passed as a C double


def dot(ctx: Context, n, x, y, out):
    _need(x, n, "x", ctx.dtype)
    _need(y, n, "y", ctx.dtype)
    _need(out, 1, "out", torch.float32)
    _check(lib.dot(ctx.handle, int(n), _ptr(x), _ptr(y), _ptr(out)))


def dot_f64(ctx: Context, n, x, y, out):
    _need(x, n, "x", ctx.dtype)
    _need(y, n, "y", ctx.dtype)
    _need(out, 1, "out", torch.float64)
    _check(lib.dot_f64(ctx.handle, int(n), _ptr(x), _ptr(y), _ptr(out)))


def dot_noalloc(n, x, y, out, stream=None):
    """Allocation-free dot product of the first n elements of x and y (same
    dtype: FP32, BF16, FP16 or FP64) into the one-element device tensor out
    (FP32 or FP64), on `stream` (default: the current stream)."""
    dt = dtype_code(x.dtype)
    _need(x, n, "x", x.dtype)
    _need(y, n, "y", x.dtype)
    if out.dtype not in (torch.float32, torch.float64):
        raise PcgError(PCG_E_ARG, "out: FP32 or FP64 device tensor expected")
    _need(out, 1, "out", out.dtype)
    f32 = _ptr(out) if out.dtype == torch.float32 else None
    f64 = _ptr(out) if out.dtype == torch.float64 else None
    _check(lib.dot_noalloc(dt, int(n), _ptr(x), _ptr(y), f32, f64, _stream(stream)))


def pcg_solve(ctx: Context, b, x, rtol=1e-6, maxit=500, raise_on_error=True) -> dict:
    _need(b, ctx.n, "b", ctx.dtype)
    _need(x, ctx.n, "x")
    info = PcgInfo()
    st = lib.pcg_solve(ctx.handle, _ptr(b), _ptr(x), float(rtol), int(maxit), ctypes.byref(info))
    out = info.as_dict()
    out["status"] = st
    if st != PCG_OK and (raise_on_error or st not in SOLVE_OUTCOMES):
        raise PcgError(st, pcg_last_error())
    return out


def pcg_get_history(ctx: Context, n=1 << 20):
    import numpy as np

    buf = np.zeros(n, dtype=np.float64)
    cnt = ctypes.c_int(0)
    _check(lib.pcg_get_history(ctx.handle, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n,
                               ctypes.byref(cnt)))
    return buf[: cnt.value].copy()


# Default inner tolerance of refinement per storage type, from a sweep at
# 256^3 (BF16 5e-2 .. 2e-3: the fastest to 1e-6 and to 1e-10; FP16 1e-2 ..
# 1e-4: the fastest to 1e-10).
REFINE_RTOL_INNER = {torch.bfloat16: 5e-3, torch.float16: 3e-3}


def pcg_solve_refined(ctx: Context, b64, x64, rtol_outer=1e-10, rtol_inner=None, max_outer=30, maxit_inner=2000,
                      raise_on_error=True) -> dict:
    """FP64 iterative refinement around the context's reduced-precision PCG."""
    if rtol_inner is None:
        rtol_inner = REFINE_RTOL_INNER.get(ctx.dtype, 1e-3)
    _need(b64, ctx.n, "b64", torch.float64)
    _need(x64, ctx.n, "x64", torch.float64)
    info = PcgInfo()
    st = lib.pcg_solve_refined(ctx.handle, _ptr(b64), _ptr(x64), float(rtol_outer), float(rtol_inner),
                               int(max_outer), int(maxit_inner), ctypes.byref(info))
    out = info.as_dict()
    out["status"] = st
    if st != PCG_OK and (raise_on_error or st not in SOLVE_OUTCOMES):
        raise PcgError(st, pcg_last_error())
    return out


def pcg_refine_history(ctx: Context, n=256):
    import numpy as np

    rel = np.zeros(n, dtype=np.float64)
    inner = np.zeros(n, dtype=np.int32)
    cnt = ctypes.c_int(0)
    _check(lib.pcg_refine_history(ctx.handle, rel.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  inner.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), n, ctypes.byref(cnt)))
    return rel[: cnt.value].copy(), inner[: max(cnt.value - 1, 0)].copy()


def pcg_set_coefficients(ctx: Context, k_cell):
    """Variable-coefficient operator with FP32 cell values k_cell (device,
    kept alive by the context object); None restores constant coefficients."""
    _need(k_cell, ctx.n, "k_cell", torch.float32)
    ctx._kcell = k_cell
    _check(lib.pcg_set_coefficients(ctx.handle, _ptr(k_cell)))


class Cnn:
    """Owns a cnn_net handle (the learned preconditioner's network)."""

    def __init__(self, handle, stream):
        self.handle = handle
        self.stream = stream

    def close(self):
        if self.handle:
            lib.cnn_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cnn_create(stream=None) -> Cnn:
    h = ctypes.c_void_p()
    s = _stream(stream)
    _check(lib.cnn_create(ctypes.byref(h), s))
    return Cnn(h, s)


def cnn_num_weights() -> int:
    return int(lib.cnn_num_weights())


def cnn_set_weights(net: Cnn, w):
    _need(w, cnn_num_weights(), "w", torch.float32)
    _check(lib.cnn_set_weights(net.handle, _ptr(w)))


def cnn_get_weights(net: Cnn, w=None):
    if w is None:
        w = torch.empty(cnn_num_weights(), dtype=torch.float32, device="cuda")
    _need(w, cnn_num_weights(), "w", torch.float32)
    _check(lib.cnn_get_weights(net.handle, _ptr(w)))
    return w


def cnn_get_adam(net: Cnn):
    """Adam's state for a training checkpoint: (m, v, step), m and v FP32
    device tensors of cnn_num_weights() values."""
    m = torch.empty(cnn_num_weights(), dtype=torch.float32, device="cuda")
    v = torch.empty_like(m)
    step = ctypes.c_int64()
    _check(lib.cnn_get_adam(net.handle, _ptr(m), _ptr(v), ctypes.byref(step)))
    return m, v, int(step.value)


def cnn_set_adam(net: Cnn, m, v, step: int):
    """Restore Adam's state (after cnn_set_weights, which resets it)."""
    _need(m, cnn_num_weights(), "m", torch.float32)
    _need(v, cnn_num_weights(), "v", torch.float32)
    _check(lib.cnn_set_adam(net.handle, _ptr(m), _ptr(v), int(step)))


def cnn_forward(net: Cnn, shape, r, g, z, rr=None):
    nz, ny, nx = shape
    n = nx * ny * nz
    _need(r, n, "r")
    _need(g, n, "g", torch.float32)
    _need(z, n, "z", torch.float32)
    _need(rr, 1, "rr", torch.float64)
    _check(lib.cnn_forward(net.handle, nx, ny, nz, dtype_code(r.dtype), _ptr(r), _ptr(g), _ptr(rr), _ptr(z)))


def cnn_loss_grad(net: Cnn, shape, pairs, g, batch, grad=None, loss=None):
    nz, ny, nx = shape
    n = nx * ny * nz
    _need(pairs, 2 * batch * n, "pairs", torch.bfloat16)
    _need(g, n, "g", torch.float32)
    _need(grad, cnn_num_weights(), "grad", torch.float32)
    _need(loss, 1, "loss", torch.float64)
    _check(lib.cnn_loss_grad(net.handle, nx, ny, nz, _ptr(pairs), _ptr(g), int(batch), _ptr(grad), _ptr(loss)))


def cnn_set_operator(net: Cnn, ctx):
    """A-norm loss with ctx's operator (ctx None: relative MSE). The network
    keeps a reference to ctx so that it outlives its use."""
    _check(lib.cnn_set_operator(net.handle, None if ctx is None else ctx.handle))
    net.op_ctx = ctx


def cnn_set_loss_norm(net: Cnn, mode: int):
    """A-norm loss normaliser: 0 = rh.D^-1 rh (default), 1 = rh.eh (the error's energy)."""
    _check(lib.cnn_set_loss_norm(net.handle, int(mode)))


def cnn_adam_step(net: Cnn, grad=None, lr=1e-3):
    _need(grad, cnn_num_weights(), "grad", torch.float32)
    _check(lib.cnn_adam_step(net.handle, _ptr(grad), float(lr)))


def cnn_train_step(net: Cnn, shape, pairs, g, batch, lr=1e-3, loss=None):
    nz, ny, nx = shape
    n = nx * ny * nz
    _need(pairs, 2 * batch * n, "pairs", torch.bfloat16)
    _need(g, n, "g", torch.float32)
    _need(loss, 1, "loss", torch.float64)
    _check(lib.cnn_train_step(net.handle, nx, ny, nz, _ptr(pairs), _ptr(g), int(batch), float(lr), _ptr(loss)))


def pcg_solve_flexible(ctx: Context, net, g, b, x, rtol=1e-6, maxit=2000, raise_on_error=True) -> dict:
    """Flexible CG with the network preconditioner (net=None: Jacobi)."""
    _need(b, ctx.n, "b", torch.float32)
    _need(x, ctx.n, "x")
    _need(g, ctx.n, "g", torch.float32)
    info = PcgInfo()
    st = lib.pcg_solve_flexible(ctx.handle, None if net is None else net.handle, _ptr(g), _ptr(b), _ptr(x),
                                float(rtol), int(maxit), ctypes.byref(info))
    out = info.as_dict()
    out["status"] = st
    if st != PCG_OK and (raise_on_error or st not in SOLVE_OUTCOMES):
        raise PcgError(st, pcg_last_error())
    return out


def pcg_set_multigrid(ctx: Context, nu=1, omega=0.0, coarse_max=0):
    """Build the geometric multigrid hierarchy of the context's operator
    (nu damped-Jacobi sweeps on each side, omega 0 = 6/7, coarse_max 0 = 512)."""
    _check(lib.pcg_set_multigrid(ctx.handle, int(nu), float(omega), int(coarse_max)))


def pcg_mg_levels(ctx: Context):
    """[(nx, ny, nz)] of the hierarchy, finest first."""
    nlev = ctypes.c_int(0)
    dims = (ctypes.c_int * (3 * 16))()
    _check(lib.pcg_mg_levels(ctx.handle, ctypes.byref(nlev), dims))
    return [tuple(dims[3 * l:3 * l + 3]) for l in range(nlev.value)]


def pcg_mg_apply(ctx: Context, g, u):
    """u = V-cycle(g) (FP32 device tensors of the context's grid)."""
    _need(g, ctx.n, "g", torch.float32)
    _need(u, ctx.n, "u", torch.float32)
    _check(lib.pcg_mg_apply(ctx.handle, _ptr(g), _ptr(u)))


def pcg_solve_mg(ctx: Context, b, x, rtol=1e-6, maxit=500, raise_on_error=True) -> dict:
    """PCG with the multigrid V-cycle preconditioner (pcg_set_multigrid first)."""
    _need(b, ctx.n, "b", torch.float32)
    _need(x, ctx.n, "x")
    info = PcgInfo()
    st = lib.pcg_solve_mg(ctx.handle, _ptr(b), _ptr(x), float(rtol), int(maxit), ctypes.byref(info))
    out = info.as_dict()
    out["status"] = st
    if st != PCG_OK and (raise_on_error or st not in SOLVE_OUTCOMES):
        raise PcgError(st, pcg_last_error())
    return out


def pcg_solve_snapshots(ctx: Context, b, x, snap_iters, r_snaps, x_snaps, rtol=1e-12, maxit=10000) -> dict:
    its = (ctypes.c_int * len(snap_iters))(*[int(v) for v in snap_iters])
    _need(b, ctx.n, "b", ctx.dtype)
    _need(x, ctx.n, "x")
    _need(r_snaps, ctx.n * len(snap_iters), "r_snaps", ctx.dtype)
    _need(x_snaps, ctx.n * len(snap_iters), "x_snaps")
    info = PcgInfo()
    _check(lib.pcg_solve_snapshots(ctx.handle, _ptr(b), _ptr(x), float(rtol), int(maxit), its, len(snap_iters),
                                   _ptr(r_snaps), _ptr(x_snaps), ctypes.byref(info)))
    return info.as_dict()


def pcg_make_pairs(ctx: Context, npairs, r_snaps, x_snaps, x_star, pairs):
    _need(r_snaps, ctx.n * npairs, "r_snaps", torch.float64)
    _need(x_snaps, ctx.n * npairs, "x_snaps", torch.float64)
    _need(x_star, ctx.n, "x_star", torch.float64)
    _need(pairs, 2 * ctx.n * npairs, "pairs", torch.bfloat16)
    _check(lib.pcg_make_pairs(ctx.handle, int(npairs), _ptr(r_snaps), _ptr(x_snaps), _ptr(x_star), _ptr(pairs)))


class Batch:
    """Owns a pcg_batch handle: many constant-coefficient problems solved in
    one persistent launch. offsets[i] is problem i's element offset in the
    FP32 b arena and the FP64 x arena (both `total` elements long)."""

    def __init__(self, handle, dims, stream):
        self.handle = handle
        self.dims = [tuple(d) for d in dims]
        self.stream = stream
        n = len(self.dims)
        offs = (ctypes.c_int64 * n)()
        total = ctypes.c_int64()
        plans = (ctypes.c_int * (4 * n))()
        grid = (ctypes.c_int * 3)()
        _check(lib.pcg_batch_layout(handle, offs, ctypes.byref(total), plans, grid))
        self.offsets = list(offs)
        self.total = int(total.value)
        self.plans = [tuple(plans[4 * i:4 * i + 4]) for i in range(n)]  # (cfg, zc, work-groups, tiles)
        self.grid = int(grid[0])
        self.tuned = int(grid[1])

    def __len__(self):
        return len(self.dims)

    def view(self, arena, i):
        nx, ny, nz = self.dims[i]
        return arena[self.offsets[i]:self.offsets[i] + nx * ny * nz]

    def close(self):
        if self.handle:
            lib.pcg_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pcg_batch_create(dims, cfgs=None, cache_path=None, tune_iters=20, stream=None) -> Batch:
    """dims: [(nx, ny, nz)] per problem; cfgs: per-problem tile shapes or None
    (cache / autotuner)."""
    n = len(dims)
    flat = (ctypes.c_int * (3 * n))(*[int(v) for d in dims for v in d])
    cf = None if cfgs is None else (ctypes.c_int * n)(*[int(c) for c in cfgs])
    h = ctypes.c_void_p()
    s = _stream(stream)
    path = None if cache_path is None else os.fsencode(cache_path)
    _check(lib.pcg_batch_create(ctypes.byref(h), n, flat, cf, path, int(tune_iters), s))
    return Batch(h, dims, s)


def pcg_batch_destroy(batch: Batch):
    batch.close()


def pcg_batch_set_restarts(batch: Batch, max_restarts: int):
    """FP64-residual restarts per problem (0 = never, -1 = default 3)."""
    _check(lib.pcg_batch_set_restarts(batch.handle, int(max_restarts)))


def pcg_batch_set_barrier(batch: Batch, form: int):
    """0: XCD-local group barriers where possible (default); 1: agent-scope fences always."""
    _check(lib.pcg_batch_set_barrier(batch.handle, int(form)))


def pcg_batch_solve(batch: Batch, b, x, rtol=1e-6, maxit=500, use_graph=True, raise_on_error=True) -> dict:
    """Solve every problem of the batch; b FP32 and x FP64 device arenas.
    Returns per-problem iters, relres (FP64 true), latency_s, restarts, plus seconds
    (host wall time) and status."""
    _need(b, batch.total, "b", torch.float32)
    _need(x, batch.total, "x", torch.float64)
    n = len(batch)
    its = (ctypes.c_int * n)()
    rel = (ctypes.c_double * n)()
    lat = (ctypes.c_double * n)()
    rst = (ctypes.c_int * n)()
    secs = ctypes.c_double()
    st = lib.pcg_batch_solve(batch.handle, _ptr(b), _ptr(x), float(rtol), int(maxit), 1 if use_graph else 0, its, rel,
                             lat, rst, ctypes.byref(secs))
    if st != PCG_OK and (raise_on_error or st not in SOLVE_OUTCOMES):
        _check(st)
    grid = (ctypes.c_int * 3)()
    _check(lib.pcg_batch_layout(batch.handle, None, None, None, grid))
    return {"status": st, "iters": list(its), "relres": list(rel), "latency_s": list(lat), "restarts": list(rst),
            "seconds": secs.value, "xcd_local": int(grid[2])}


def _csr_host(rowptr, col, val):
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float32)
    if rowptr.ndim != 1 or rowptr.size < 1 or col.size != val.size or int(rowptr[-1]) != col.size:
        raise PcgError(PCG_E_ARG, "compressed rows: rowptr needs nrows + 1 entries ending at len(col) = len(val)")
    return rowptr, col, val


def pcg_sell_build(rowptr, col, val, ncols, chunk=64, sigma=1) -> dict:
    """Host-only sliced-ELLPACK layout of a compressed-row matrix (numpy in
    and out): chunk_ptr, perm, col, val."""
    rowptr, col, val = _csr_host(rowptr, col, val)
    nrows = rowptr.size - 1
    nch, nsl = ctypes.c_int64(), ctypes.c_int64()
    args = (int(nrows), int(ncols), rowptr.ctypes.data, col.ctypes.data, val.ctypes.data, int(chunk), int(sigma))
    _check(lib.pcg_sell_build(*args, ctypes.byref(nch), ctypes.byref(nsl), None, None, None, None))
    cptr = np.empty(nch.value + 1, dtype=np.int64)
    perm = np.empty(nrows, dtype=np.int32)
    scol = np.empty(nsl.value, dtype=np.int32)
    sval = np.empty(nsl.value, dtype=np.float32)
    _check(lib.pcg_sell_build(*args, ctypes.byref(nch), ctypes.byref(nsl), cptr.ctypes.data, perm.ctypes.data,
                              scol.ctypes.data, sval.ctypes.data))
    return {"chunk_ptr": cptr, "perm": perm, "col": scol, "val": sval}


class Sell:
    """Owns a pcg_sell handle: a general sparse matrix in sliced ELLPACK
    (C = 64) in device memory."""

    def __init__(self, handle, nrows, ncols):
        self.handle = handle
        self.nrows, self.ncols = int(nrows), int(ncols)
        nnz, nsl, nch = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib.pcg_sell_info(handle, ctypes.byref(nnz), ctypes.byref(nsl), ctypes.byref(nch)))
        self.nnz, self.nslots, self.nchunks = int(nnz.value), int(nsl.value), int(nch.value)

    def close(self):
        if self.handle:
            lib.pcg_sell_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pcg_sell_create(rowptr, col, val, ncols, sigma=1, stream=None) -> Sell:
    """Upload a compressed-row matrix (host arrays) as sliced ELLPACK."""
    rowptr, col, val = _csr_host(rowptr, col, val)
    nrows = rowptr.size - 1
    h = ctypes.c_void_p()
    _check(lib.pcg_sell_create(ctypes.byref(h), int(nrows), int(ncols), rowptr.ctypes.data, col.ctypes.data,
                               val.ctypes.data, int(sigma), _stream(stream)))
    return Sell(h, nrows, ncols)


def pcg_sell_destroy(A: Sell):
    A.close()


def pcg_sell_spmv(A: Sell, x, y):
    """y = A x (FP32 device tensors), asynchronous on the matrix's stream."""
    _need(x, A.ncols, "x", torch.float32)
    _need(y, A.nrows, "y", torch.float32)
    _check(lib.pcg_sell_spmv(A.handle, _ptr(x), _ptr(y)))


def pcg_sell_solve(A: Sell, b, x, rtol=1e-6, maxit=500, raise_on_error=True) -> dict:
    """Jacobi-PCG on the stored matrix: b FP32, x FP64 device tensors."""
    _need(b, A.nrows, "b", torch.float32)
    _need(x, A.nrows, "x", torch.float64)
    info = PcgInfo()
    st = lib.pcg_sell_solve(A.handle, _ptr(b), _ptr(x), float(rtol), int(maxit), ctypes.byref(info))
    out = info.as_dict()
    out["status"] = st
    if st != PCG_OK and (raise_on_error or st not in SOLVE_OUTCOMES):
        raise PcgError(st, pcg_last_error())
    return out


def pcg_sell_set_graph(A: Sell, use_graph: bool):
    _check(lib.pcg_sell_set_graph(A.handle, 1 if use_graph else 0))


def pcg_sell_set_restarts(A: Sell, max_restarts: int):
    """FP64-residual restarts of pcg_sell_solve (0 = never, -1 = default 3)."""
    _check(lib.pcg_sell_set_restarts(A.handle, int(max_restarts)))
