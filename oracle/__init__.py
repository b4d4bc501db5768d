"""FP64 CPU oracle for the Jacobi-PCG hot path.

TEST INFRASTRUCTURE ONLY. Only tests/, the smoke check and the benchmark's
CPU-baseline leg import this package; the product path never does. It shares
no code with the HIP library: the operator, BLAS-1 and PCG live in plain C
(oracle.c, FP64, fixed-order reductions), and the parts below are plain numpy.

Contents, with the passage each follows:
  stencil / vstencil / vdiag / axpy / dot / pcg / residual
      -> oracle.c (paper Sec. VII: matrix-free seven-point operator with zero
         Dirichlet boundaries, Jacobi preconditioner, PCG; Sec. IV/V:
         element-wise update and global dot).
  csr_spmv
      -> oracle.c: y = A x for a compressed-row matrix (Sec. VII-A: the GPU
         comparison system's SpMV, there on a sliced-ELLPACK matrix).
  csr_pcg
      -> oracle.c: the Jacobi-PCG above on a square compressed-row matrix
         (Sec. VII-A's comparison system runs CG on a stored matrix).
  stencil_loops, assemble_dense
      -> pure-Python twins for tiny grids (brute force).
  round_f32 / round_bf16 / round_f16
      -> round-to-nearest-even to a p-bit significand, written from the
         IEEE 754 definition (quantum 2^(e-p+1), exponent clamped at the
         format's subnormal quantum).
  ir_emulate
      -> iterative refinement (Wilkinson 1963; Moler 1967) around a Jacobi-
         PCG whose vectors are stored in BF16/FP16 with FP32 arithmetic.
         Reference outer-iteration counts. Inner counts: parity unpinned.
  fcg
      -> flexible CG truncated to one direction (Notay 2000), with the
         Jacobi fallback rule.
  conv3d_fwd / conv3d_bwd / cnn_forward / cnn_backward / rel_mse / adam
      -> the learned preconditioner's network (3x3x3 convolutions, zero
         padding, ReLU) and its training step, FP64.
  multigrid (VCycle, mg_pcg, hierarchy, prolong, restrict, smooth)
      -> the geometric multigrid V-cycle (the paper's future work, Sec. VIII)
         and PCG preconditioned by it; see oracle/multigrid.py.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, NOCONV, BREAKDOWN = 0, 3, 4

_dp = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH):
        from . import build as _b

        _b.build()
    lib = ctypes.CDLL(_LIBPATH)
    i, d, i64 = ctypes.c_int, ctypes.c_double, ctypes.c_int64
    lib.oracle_stencil.argtypes = [i, i, i, _dp, _dp]
    lib.oracle_vstencil.argtypes = [i, i, i, _dp, _dp, _dp]
    lib.oracle_vdiag.argtypes = [i, i, i, _dp, _dp]
    lib.oracle_axpy.argtypes = [i64, d, _dp, _dp, _dp]
    lib.oracle_csr_spmv.argtypes = [i64, ctypes.c_void_p, ctypes.c_void_p, _dp, _dp, _dp]
    lib.oracle_csr_spmv.restype = None
    lib.oracle_csr_pcg.argtypes = [i64, ctypes.c_void_p, ctypes.c_void_p, _dp, _dp, _dp, d, i, _dp,
                                   ctypes.POINTER(i), ctypes.POINTER(d)]
    lib.oracle_csr_pcg.restype = i
    lib.oracle_dot.argtypes = [i64, _dp, _dp]
    lib.oracle_dot.restype = d
    lib.oracle_pcg.argtypes = [i, i, i, _dp, _dp, _dp, d, i, _dp,
                               ctypes.POINTER(i), ctypes.POINTER(d)]
    lib.oracle_pcg.restype = i
    lib.oracle_pcg_sr.argtypes = [i, i, i, _dp, _dp, _dp, d, i, _dp,
                                  ctypes.POINTER(i), ctypes.POINTER(d)]
    lib.oracle_pcg_sr.restype = i
    lib.oracle_residual.argtypes = [i, i, i, _dp, _dp, _dp, _dp,
                                    ctypes.POINTER(d), ctypes.POINTER(d)]
    lib.oracle_threads.restype = i
    lib.oracle_set_threads.argtypes = [i]
    lib.oracle_set_threads.restype = None
    _lib = lib
    return lib


def threads() -> int:
    """OpenMP threads used by the C oracle's loops."""
    return int(_load().oracle_threads())


def set_threads(n: int) -> None:
    """Threads of the C oracle's loops from now on (fixed-order reductions:
    the results do not depend on it)."""
    _load().oracle_set_threads(int(n))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _dims(shape):
    nz, ny, nx = shape
    return int(nx), int(ny), int(nz)


# ----------------------------------------------------------------------------
# Operator and BLAS-1 (C, FP64)
# ----------------------------------------------------------------------------

def stencil(x, shape) -> np.ndarray:
    """y = A x, constant coefficients (6 on the diagonal, -1 per face neighbour)."""
    nx, ny, nz = _dims(shape)
    x = _f64(x)
    y = np.empty_like(x)
    _load().oracle_stencil(nx, ny, nz, _ptr(x), _ptr(y))
    return y


def vstencil(kcell, u, shape) -> np.ndarray:
    """y = A_k u: sum over faces of k_f (u_p - u_nb), harmonic-mean k_f."""
    nx, ny, nz = _dims(shape)
    k, u = _f64(kcell), _f64(u)
    y = np.empty_like(u)
    _load().oracle_vstencil(nx, ny, nz, _ptr(k), _ptr(u), _ptr(y))
    return y


def vdiag(kcell, shape) -> np.ndarray:
    """Diagonal of A_k (sum of the six face coefficients)."""
    nx, ny, nz = _dims(shape)
    k = _f64(kcell)
    d = np.empty_like(k)
    _load().oracle_vdiag(nx, ny, nz, _ptr(k), _ptr(d))
    return d


def axpy(alpha, x, y) -> np.ndarray:
    x, y = _f64(x), _f64(y)
    z = np.empty_like(x)
    _load().oracle_axpy(x.size, float(alpha), _ptr(x), _ptr(y), _ptr(z))
    return z


def dot(x, y) -> float:
    x, y = _f64(x), _f64(y)
    return float(_load().oracle_dot(x.size, _ptr(x), _ptr(y)))


def csr_spmv(rowptr, col, val, x) -> np.ndarray:
    """y = A x for A in compressed-row form (rowptr int64, col int32), FP64."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val, x = _f64(val), _f64(x)
    nrows = rowptr.size - 1
    if rowptr[0] != 0 or rowptr[-1] != col.size or col.size != val.size:
        raise ValueError("csr_spmv: inconsistent compressed-row arrays")
    if col.size and (col.min() < 0 or col.max() >= x.size):
        raise ValueError("csr_spmv: column index out of range")
    y = np.empty(nrows, dtype=np.float64)
    if nrows:
        _load().oracle_csr_spmv(nrows, rowptr.ctypes.data, col.ctypes.data, _ptr(val), _ptr(x), _ptr(y))
    return y


def pcg(shape, b, rtol=1e-6, maxit=500, kcell=None, x0=None, history=False):
    """FP64 Jacobi-PCG; returns dict(x, iters, status, relres[, hist])."""
    nx, ny, nz = _dims(shape)
    b = _f64(b)
    x = np.zeros_like(b) if x0 is None else _f64(x0).copy()
    k = None if kcell is None else _f64(kcell)
    hist = np.full(maxit + 1, np.nan) if history else None
    it, rr = ctypes.c_int(0), ctypes.c_double(0.0)
    st = _load().oracle_pcg(nx, ny, nz, None if k is None else _ptr(k), _ptr(b), _ptr(x),
                            float(rtol), int(maxit), None if hist is None else _ptr(hist),
                            ctypes.byref(it), ctypes.byref(rr))
    out = dict(x=x, iters=it.value, status=st, relres=rr.value)
    if history:
        out["hist"] = hist[: it.value + 1]
    return out


def csr_pcg(rowptr, col, val, b, rtol=1e-6, maxit=500, x0=None, history=False):
    """FP64 Jacobi-PCG (the same steps as pcg()) on a square compressed-row
    matrix; D = the sum of each row's diagonal entries. Returns dict(x, iters,
    status, relres[, hist]); status BREAKDOWN if a diagonal is not positive."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val, b = _f64(val), _f64(b)
    n = rowptr.size - 1
    if b.size != n or rowptr[-1] != col.size or col.size != val.size:
        raise ValueError("csr_pcg: inconsistent sizes")
    if col.size and (col.min() < 0 or col.max() >= n):
        raise ValueError("csr_pcg: column index out of range")
    x = np.zeros_like(b) if x0 is None else _f64(x0).copy()
    hist = np.full(maxit + 1, np.nan) if history else None
    it, rr = ctypes.c_int(0), ctypes.c_double(0.0)
    st = _load().oracle_csr_pcg(n, rowptr.ctypes.data, col.ctypes.data, _ptr(val), _ptr(b), _ptr(x), float(rtol),
                                int(maxit), None if hist is None else _ptr(hist), ctypes.byref(it), ctypes.byref(rr))
    out = dict(x=x, iters=it.value, status=st, relres=rr.value)
    if history:
        out["hist"] = hist[: it.value + 1]
    return out


def pcg_sr(shape, b, rtol=1e-6, maxit=500, kcell=None, x0=None, history=False):
    """FP64 Jacobi-PCG with one reduction per iteration (Chronopoulos-Gear,
    J. Comput. Appl. Math. 25, 1989); same results as pcg() in exact
    arithmetic. Returns dict(x, iters, status, relres[, hist])."""
    nx, ny, nz = _dims(shape)
    b = _f64(b)
    x = np.zeros_like(b) if x0 is None else _f64(x0).copy()
    k = None if kcell is None else _f64(kcell)
    hist = np.full(maxit + 1, np.nan) if history else None
    it, rr = ctypes.c_int(0), ctypes.c_double(0.0)
    st = _load().oracle_pcg_sr(nx, ny, nz, None if k is None else _ptr(k), _ptr(b), _ptr(x),
                               float(rtol), int(maxit), None if hist is None else _ptr(hist),
                               ctypes.byref(it), ctypes.byref(rr))
    out = dict(x=x, iters=it.value, status=st, relres=rr.value)
    if history:
        out["hist"] = hist[: it.value + 1]
    return out


def residual(shape, b, x, kcell=None):
    """(r, ||r||_2, max|r|) with r = b - A x in FP64."""
    nx, ny, nz = _dims(shape)
    b, x = _f64(b), _f64(x)
    r = np.empty_like(b)
    n2, am = ctypes.c_double(), ctypes.c_double()
    k = None if kcell is None else _f64(kcell)
    _load().oracle_residual(nx, ny, nz, None if k is None else _ptr(k), _ptr(b), _ptr(x),
                            _ptr(r), ctypes.byref(n2), ctypes.byref(am))
    return r, n2.value, am.value


def true_relres(shape, b, x, kcell=None) -> float:
    _, n2, _ = residual(shape, b, x, kcell)
    nb = math.sqrt(dot(b, b))
    return n2 / nb if nb > 0 else 0.0


# ----------------------------------------------------------------------------
# Pure-Python twins for tiny grids
# ----------------------------------------------------------------------------

def stencil_loops(x, shape) -> np.ndarray:
    """Seven-point operator by explicit loops over points and neighbours."""
    nz, ny, nx = shape
    x = np.asarray(x, dtype=np.float64).reshape(nz, ny, nx)
    y = np.zeros_like(x)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                s = 6.0 * x[k, j, i]
                for (a, b, c) in ((i - 1, j, k), (i + 1, j, k), (i, j - 1, k),
                                  (i, j + 1, k), (i, j, k - 1), (i, j, k + 1)):
                    if 0 <= a < nx and 0 <= b < ny and 0 <= c < nz:
                        s -= x[c, b, a]
                y[k, j, i] = s
    return y.reshape(-1)


def assemble_dense(shape, kcell=None) -> np.ndarray:
    """Dense matrix of the operator, column j = A e_j (tiny grids only)."""
    n = int(np.prod(shape))
    A = np.zeros((n, n))
    e = np.zeros(n)
    for j in range(n):
        e[:] = 0.0
        e[j] = 1.0
        A[:, j] = stencil(e, shape) if kcell is None else vstencil(kcell, e, shape)
    return A


# ----------------------------------------------------------------------------
# Rounding to reduced-precision formats (round to nearest, ties to even)
# ----------------------------------------------------------------------------

def _round_sig(x, p: int, emin: int, emax_val: float) -> np.ndarray:
    """Round FP64 values to a binary format with p significant bits, smallest
    normal exponent emin and largest finite value emax_val.

    The quantum of a value with binary exponent e (x = m 2^e, 1 <= m < 2) is
    2^(e - p + 1), but never below the subnormal quantum 2^(emin - p + 1);
    np.rint rounds halves to even. Magnitudes above the largest finite value
    (after rounding) become infinity.
    """
    x = np.asarray(x, dtype=np.float64)
    ax = np.abs(x)
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        _, e = np.frexp(ax)  # ax = f 2^e, 0.5 <= f < 1  ->  binary exponent e-1
        e = np.maximum(e - 1, emin)
        q = np.ldexp(1.0, e - p + 1)
        r = np.rint(ax / q) * q
        r = np.where(r > emax_val, np.inf, r)
        r = np.where(ax == 0, 0.0, r)
        r = np.where(np.isfinite(ax), r, ax)
    return np.copysign(r, x)


def round_f32(x) -> np.ndarray:
    return _round_sig(x, 24, -126, float(np.finfo(np.float32).max))


def round_bf16(x) -> np.ndarray:
    """FP64 -> FP32 -> BF16, each step to nearest even."""
    return _round_sig(round_f32(x), 8, -126, 3.3895313892515355e38)


def round_f16(x) -> np.ndarray:
    """FP64 -> FP32 -> FP16, each step to nearest even."""
    return _round_sig(round_f32(x), 11, -14, 65504.0)


_ROUND = {"f32": round_f32, "bf16": round_bf16, "f16": round_f16,
          "f64": lambda v: np.asarray(v, dtype=np.float64)}


# ----------------------------------------------------------------------------
# Mixed-precision iterative refinement (emulated storage, FP32 arithmetic)
# ----------------------------------------------------------------------------

def _stencil_f32(v, shape) -> np.ndarray:
    """Constant-coefficient operator evaluated in FP32 arithmetic."""
    nz, ny, nx = shape
    u = np.zeros((nz + 2, ny + 2, nx + 2), dtype=np.float32)
    u[1:-1, 1:-1, 1:-1] = np.asarray(v, dtype=np.float32).reshape(shape)
    c = u[1:-1, 1:-1, 1:-1]
    y = np.float32(6.0) * c
    y = y - u[1:-1, 1:-1, :-2] - u[1:-1, 1:-1, 2:]
    y = y - u[1:-1, :-2, 1:-1] - u[1:-1, 2:, 1:-1]
    y = y - u[:-2, 1:-1, 1:-1] - u[2:, 1:-1, 1:-1]
    return y.reshape(-1)


def inner_pcg_lp(shape, rhat, fmt: str, rtol: float, maxit: int,
                 stag_window: int = 100, stag_drop: float = 0.9, d_fmt: str | None = None):
    """Jacobi-PCG on A d = rhat with every vector (d, r, p) stored in `fmt`
    and FP32 element arithmetic (FP64 for fmt "f64"); scalars and dot sums in
    FP64.

    Stops at ||r|| <= rtol ||rhat|| (recursive), at maxit, on breakdown, or on
    stagnation: the best residual so far has not dropped below stag_drop
    times the previous best mark for stag_window iterations.
    d_fmt: format the correction d accumulates in (default: fmt).
    Returns (d as FP64 values of the stored format, iterations).
    """
    rnd = _ROUND[fmt]
    rnd_d = _ROUND[d_fmt or fmt]
    f32 = np.float64 if fmt == "f64" else np.float32   # element arithmetic type
    dinv = f32(1.0 / 6.0)
    r = rnd(rhat)
    d = np.zeros_like(r)
    p = np.zeros_like(r)
    rr = float(np.dot(r, r))
    nr0 = math.sqrt(rr)
    if nr0 == 0.0:
        return d, 0
    rho = float(dinv) * rr
    beta = 0.0
    best, best_at = nr0, 0
    it = 0
    for it in range(1, maxit + 1):
        p = rnd(dinv * r.astype(f32) + f32(beta) * p.astype(f32))
        q = stencil(p, shape) if fmt == "f64" else _stencil_f32(p, shape)
        sigma = float(np.dot(p, q.astype(np.float64)))
        if not (sigma > 0.0) or not math.isfinite(sigma):
            break
        alpha = f32(rho / sigma)
        d = rnd_d(d.astype(f32) + alpha * p.astype(f32))
        r = rnd(r.astype(f32) - alpha * q)
        rr = float(np.dot(r, r))
        nr = math.sqrt(rr)
        if not math.isfinite(nr) or nr <= rtol * nr0:
            break
        if stag_window > 0:
            if nr < stag_drop * best:
                best, best_at = nr, it
            elif it - best_at >= stag_window:
                break
        rho_new = float(dinv) * rr
        beta = rho_new / rho
        rho = rho_new
    return d, it


def ir_emulate(shape, b, fmt: str = "bf16", rtol_outer: float = 1e-10, rtol_in: float | None = None,
               max_outer: int = 30, maxit_in: int = 2000, d_fmt: str | None = None):
    """FP64 iterative refinement with an emulated low-precision inner PCG.

    x = 0; loop: r = b - A x (FP64); stop when ||r||/||b|| <= rtol_outer;
    s = 1 / max|r|; rhat = fmt(s r); d = inner PCG; x += d / s.
    Returns dict(x, outer, inner (list), history (relres before each step)).
    """
    if rtol_in is None:
        rtol_in = 1e-2 if fmt == "bf16" else 1e-3
    b = _f64(b)
    x = np.zeros_like(b)
    nb = math.sqrt(dot(b, b))
    hist, inner = [], []
    outer = 0
    while True:
        r, n2, amax = residual(shape, b, x)
        t = n2 / nb
        hist.append(t)
        if t <= rtol_outer or outer >= max_outer:
            break
        s = 1.0 / amax
        d, it = inner_pcg_lp(shape, s * r, fmt, rtol_in, maxit_in, d_fmt=d_fmt)
        inner.append(it)
        x = x + d / s
        outer += 1
    return dict(x=x, outer=outer, inner=inner, history=hist)


# ----------------------------------------------------------------------------
# Flexible CG with one stored direction and a Jacobi fallback
# ----------------------------------------------------------------------------

def fcg(shape, b, precond, rtol=1e-6, maxit=2000, kcell=None, stag_window=100, stag_drop=0.9):
    """Flexible CG (Notay 2000, truncation m = 1):

      r = b - A x; z = M(r); p = z
      loop: q = A p; sigma = p.q; alpha = (p.r)/sigma; x += alpha p; r -= alpha q
            stop on ||r|| <= rtol ||b||
            z = M(r); beta = -(z.q)/sigma; p = z + beta p

    M falls back to D^-1 for the rest of the solve when z.r <= 0, a value is
    not finite, or the best ||r|| so far has not improved by 10% for
    stag_window iterations (100: plateaus of plain Jacobi-PCG at 128^3 last
    longer than 20); the direction recurrence restarts from p = z at the switch.
    precond(r) -> z. Returns dict(x, iters, status, relres, fallback_at).
    """
    op = (lambda v: stencil(v, shape)) if kcell is None else (lambda v: vstencil(kcell, v, shape))
    dinv = 1.0 / (np.full(int(np.prod(shape)), 6.0) if kcell is None else vdiag(kcell, shape))
    b = _f64(b)
    x = np.zeros_like(b)
    nb = math.sqrt(dot(b, b))
    if nb == 0.0:
        return dict(x=x, iters=0, status=OK, relres=0.0, fallback_at=None)
    r = b.copy()
    use_m = precond is not None
    fallback_at = None

    def apply_m(v):
        return precond(v) if use_m else dinv * v

    z = apply_m(r)
    if use_m and (not np.all(np.isfinite(z)) or dot(z, r) <= 0.0):
        use_m, fallback_at = False, 0
        z = dinv * r
    p = z.copy()
    norms = [nb]
    best, best_at = 1.0, 0
    status = NOCONV
    k = 0
    for k in range(1, maxit + 1):
        q = op(p)
        sigma = dot(p, q)
        if not (sigma > 0.0) or not math.isfinite(sigma):
            status = BREAKDOWN
            break
        alpha = dot(p, r) / sigma
        x += alpha * p
        r -= alpha * q
        nr = math.sqrt(dot(r, r))
        norms.append(nr)
        if nr <= rtol * nb:
            status = OK
            break
        stag = False
        if nr / nb < stag_drop * best:
            best, best_at = nr / nb, k
        elif use_m and k - best_at >= stag_window:
            stag, best_at = True, k
        z = apply_m(r)
        restart = False
        if use_m:
            bad = (not np.all(np.isfinite(z))) or dot(z, r) <= 0.0
            if bad or stag:
                use_m, fallback_at, restart = False, k, True
                z = dinv * r
        if restart:
            p = z.copy()
        else:
            beta = -dot(z, q) / sigma
            p = z + beta * p
    return dict(x=x, iters=k, status=status, relres=norms[-1] / nb, fallback_at=fallback_at)


# ----------------------------------------------------------------------------
# The learned preconditioner's network (FP64)
# ----------------------------------------------------------------------------
# Activations are NDHWC: [D, H, W, C]. A layer's weight is [27, Cin, Cout]
# with tap t = 9 dz + 3 dy + dx (dz, dy, dx in 0..2 meaning offsets -1..+1).

def _shift(xp, dz, dy, dx, D, H, W):
    return xp[dz:dz + D, dy:dy + H, dx:dx + W, :]


def conv3d_fwd(x, w) -> np.ndarray:
    """y[z,y,x,co] = sum_{taps, ci} x[z+dz-1, y+dy-1, x+dx-1, ci] w[t, ci, co],
    zero outside the grid."""
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    D, H, W, _ = x.shape
    xp = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    y = np.zeros((D, H, W, w.shape[2]))
    for t in range(27):
        dz, dy, dx = t // 9, (t // 3) % 3, t % 3
        y += _shift(xp, dz, dy, dx, D, H, W) @ w[t]
    return y


def conv3d_bwd(x, w, dy):
    """Gradients of conv3d_fwd: (dx, dw).

    dx[p, ci] = sum_t sum_co dy[p - off_t, co] w[t, ci, co]
    dw[t, ci, co] = sum_p x[p + off_t, ci] dy[p, co]
    """
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    dy = np.asarray(dy, dtype=np.float64)
    D, H, W, Cin = x.shape
    xp = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for t in range(27):
        dz, dy_, dx_ = t // 9, (t // 3) % 3, t % 3
        xs = _shift(xp, dz, dy_, dx_, D, H, W)
        dw[t] = xs.reshape(-1, Cin).T @ dy.reshape(-1, dy.shape[-1])
        dxp[dz:dz + D, dy_:dy_ + H, dx_:dx_ + W, :] += dy @ w[t].T
    return dxp[1:-1, 1:-1, 1:-1, :], dw


def cnn_forward(weights, inp, relu=True):
    """Layers conv -> ReLU (all but the last). Returns (output, activations)
    where activations[i] is the input of layer i."""
    acts = [np.asarray(inp, dtype=np.float64)]
    h = acts[0]
    for li, w in enumerate(weights):
        h = conv3d_fwd(h, w)
        if relu and li < len(weights) - 1:
            h = np.maximum(h, 0.0)
        if li < len(weights) - 1:
            acts.append(h)
    return h, acts


def cnn_backward(weights, acts, dout, relu=True):
    """Back-propagation through cnn_forward; returns per-layer weight grads."""
    grads = [None] * len(weights)
    g = np.asarray(dout, dtype=np.float64)
    for li in range(len(weights) - 1, -1, -1):
        dx, dw = conv3d_bwd(acts[li], weights[li], g)
        grads[li] = dw
        if li > 0:
            g = dx * (acts[li] > 0.0) if relu else dx
    return grads


def precond_input(r, g, shape):
    """Network input channels (r / rms(r), g) and the scale rms(r)."""
    r = _f64(r)
    rho = math.sqrt(dot(r, r) / r.size)
    nz, ny, nx = shape
    inp = np.stack([(r / rho).reshape(nz, ny, nx), _f64(g).reshape(nz, ny, nx)], axis=-1)
    return inp, rho


def cnn_apply(weights, r, g, shape) -> np.ndarray:
    """z = rms(r) N(r / rms(r), g), flattened."""
    inp, rho = precond_input(r, g, shape)
    out, _ = cnn_forward(weights, inp)
    return rho * out.reshape(-1)


def rel_mse(pred, target):
    """sum over samples of ||pred - target||^2 / ||target||^2, and its gradient."""
    loss = 0.0
    grads = []
    for p, t in zip(pred, target):
        p = np.asarray(p, dtype=np.float64)
        t = np.asarray(t, dtype=np.float64)
        den = float(np.sum(t * t))
        diff = p - t
        loss += float(np.sum(diff * diff)) / den
        grads.append(2.0 * diff / den)
    return loss, grads


def anorm_loss(pred, rh, eh, shape, kcell=None, energy=False):
    """A-norm error of the preconditioner z = D^-1 rh + pred as an
    approximation of eh (the error belonging to the residual rh), per sample
    normalised by den = rh.D^-1 rh, or with energy=True by den = rh.eh (the
    error's energy eh.A eh when rh = A eh):
        u = pred + D^-1 rh - eh,  L = u.A u / den,  dL/dpred = 2 A u / den
    (A symmetric). Returns (sum over samples of L, list of gradients)."""
    op = (lambda v: stencil(v, shape)) if kcell is None else (lambda v: vstencil(kcell, v, shape))
    n = int(np.prod(shape))
    dinv = 1.0 / (np.full(n, 6.0) if kcell is None else vdiag(kcell, shape))
    loss = 0.0
    grads = []
    for p, r, e in zip(pred, rh, eh):
        p, r, e = (np.asarray(a, dtype=np.float64).reshape(-1) for a in (p, r, e))
        u = p + dinv * r - e
        au = op(u)
        den = float(np.dot(r, e)) if energy else float(np.sum(dinv * r * r))
        loss += float(np.dot(u, au)) / den
        grads.append(2.0 * au / den)
    return loss, grads


def adam(w, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba 2015) with bias correction; returns (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


from . import multigrid  # noqa: E402  (uses the operator above)
from .multigrid import VCycle, hierarchy, mg_pcg, prolong, restrict, smooth  # noqa: E402,F401
