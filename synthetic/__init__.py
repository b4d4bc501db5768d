"""Seeded synthetic inputs for the Jacobi-PCG workloads.

This module is shared by the oracle-side tests and by the GPU path. It holds
no arithmetic of the solver itself: only random draws, their casts to the
storage types, closed-form input fields and the grid-size draws. Everything is
produced on the host as numpy arrays (FP64 draws, cast FP64 -> FP32 with
round-to-nearest-even; FP32 -> BF16/FP16 also round-to-nearest-even).

Grids are stored C-order as [nz][ny][nx] with x contiguous. Points are indexed
0..n-1 in memory; the closed-form fields below use the 1-based position i+1
so that they vanish on the ghost planes at 0 and n+1.
"""
from __future__ import annotations

import math

import numpy as np

# Fixed seeds of the five workloads (plus the held-out/training seed bases).
SEED_C1_B = 1
SEED_C1_X = 2
SEED_C1_Y = 3
SEED_C2_X = 2
SEED_C2_Y = 3
SEED_C3_NOISE = 4
SEED_C4_SIZES = 5
SEED_C4_B_BASE = 1000
SEED_C5_GRF = 6
SEED_C5_TRAIN_BASE = 10000
SEED_C5_HELDOUT_BASE = 20000
# The paper's GPU comparison grid (its Table III): nx x ny x nz, b ~ U[-1, 1].
PAPER_GRID = (512, 112, 64)
SEED_PAPER_GRID_B = 7
# Sparse matrices for the general (compressed-row / sliced-ELLPACK) SpMV.
SEED_SPARSE = 8


def uniform(seed: int, n: int) -> np.ndarray:
    """n FP64 draws from U[-1, 1) with numpy's PCG64 generator."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, int(n))


def uniform_f32(seed: int, n: int) -> np.ndarray:
    """uniform() rounded to FP32 (numpy's cast is round-to-nearest-even)."""
    return uniform(seed, n).astype(np.float32)


def f32_to_bf16_bits(a: np.ndarray) -> np.ndarray:
    """Round FP32 values to BF16 (nearest, ties to even); returns uint16 bits.

    Rounds by adding 0x7FFF plus the lowest kept bit to the FP32 bit pattern
    and truncating; NaNs are kept quiet.
    """
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16).astype(np.uint16)
    nan = np.isnan(np.ascontiguousarray(a, dtype=np.float32))
    r[nan] = ((u[nan] >> 16) | 0x40).astype(np.uint16)
    return r


def bf16_bits_to_f32(bits: np.ndarray) -> np.ndarray:
    """Widen BF16 bit patterns (uint16) to FP32 exactly."""
    return (np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def uniform_bf16_bits(seed: int, n: int) -> np.ndarray:
    """uniform() -> FP32 -> BF16, as uint16 bit patterns."""
    return f32_to_bf16_bits(uniform_f32(seed, n))


def uniform_f16(seed: int, n: int) -> np.ndarray:
    """uniform() -> FP32 -> FP16 (numpy's cast rounds to nearest even)."""
    return uniform_f32(seed, n).astype(np.float16)


def integers(seed: int, n: int, lo: int, hi: int, density: float = 1.0) -> np.ndarray:
    """Integer-valued FP32 vector with entries in [lo, hi]; a fraction
    (1 - density) of the entries is set to zero."""
    rng = np.random.default_rng(seed)
    v = rng.integers(lo, hi + 1, int(n)).astype(np.float32)
    if density < 1.0:
        v[rng.random(int(n)) >= density] = 0.0
    return v


def sine_mode(nx: int, ny: int, nz: int, a: int = 1, b: int = 1, c: int = 1) -> np.ndarray:
    """FP64 grid of sin(pi a (i+1)/(nx+1)) sin(pi b (j+1)/(ny+1)) sin(pi c (k+1)/(nz+1))."""
    sx = np.sin(math.pi * a * np.arange(1, nx + 1) / (nx + 1))
    sy = np.sin(math.pi * b * np.arange(1, ny + 1) / (ny + 1))
    sz = np.sin(math.pi * c * np.arange(1, nz + 1) / (nz + 1))
    return (sz[:, None, None] * sy[None, :, None] * sx[None, None, :]).reshape(-1)


def smooth_plus_noise(n: int, seed: int = SEED_C3_NOISE, amp: float = 1e-3) -> np.ndarray:
    """The refinement workload's exact solution on an n^3 grid (FP64):
    the lowest sine mode plus amp * U[-1, 1) noise."""
    return sine_mode(n, n, n) + amp * uniform(seed, n ** 3)


def batch_sizes(nprob: int = 64, seed: int = SEED_C4_SIZES, lo: int = 16, hi: int = 128) -> list[int]:
    """Cube edges drawn log-uniform in [lo, hi]: rint(exp(U(ln lo, ln hi))), clipped."""
    u = np.random.default_rng(seed).uniform(math.log(lo), math.log(hi), nprob)
    return [int(v) for v in np.clip(np.rint(np.exp(u)), lo, hi)]


def gaussian_random_field(n: int, seed: int = SEED_C5_GRF, corr_len: float = 8.0) -> np.ndarray:
    """Squared-exponential Gaussian random field on an n^3 grid (FP64).

    White noise on a periodic (2n)^3 box is filtered in Fourier space with the
    square root of the spectral density of C(r) = exp(-r^2 / (2 l^2)), the
    central n^3 block is cropped, and the sample is normalised to mean 0 and
    standard deviation 1. Returns the flattened [nz][ny][nx] field.
    """
    m = 2 * n
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((m, m, m))
    k = 2.0 * math.pi * np.fft.fftfreq(m)
    k2 = k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2
    amp = np.exp(-0.25 * corr_len ** 2 * k2)  # sqrt of exp(-l^2 k^2 / 2)
    g = np.fft.ifftn(np.fft.fftn(w) * amp).real
    g = g[:n, :n, :n]
    g = (g - g.mean()) / g.std()
    return np.ascontiguousarray(g).reshape(-1)


def coefficient_field(n: int, seed: int = SEED_C5_GRF) -> np.ndarray:
    """Cell coefficient k = exp(g) of the variable-coefficient workload, FP32."""
    return np.exp(gaussian_random_field(n, seed)).astype(np.float32)


def poisson7_csr(nx: int, ny: int, nz: int):
    """The seven-point operator's matrix in compressed-row form.

    Row p of the [nz][ny][nx] grid holds 6 at column p and -1 at each face
    neighbour inside the grid, columns ascending (-z, -y, -x, p, +x, +y, +z).
    Returns (rowptr int64, col int32, val float32).
    """
    n = nx * ny * nz
    idx = np.arange(n, dtype=np.int64)
    i = idx % nx
    j = (idx // nx) % ny
    k = idx // (nx * ny)
    offs = (-nx * ny, -nx, -1, 0, 1, nx, nx * ny)
    ok = (k > 0, j > 0, i > 0, np.ones(n, dtype=bool), i < nx - 1, j < ny - 1, k < nz - 1)
    cols = np.empty((n, 7), dtype=np.int32)
    mask = np.empty((n, 7), dtype=bool)
    for t in range(7):
        cols[:, t] = idx + offs[t] if offs[t] else idx
        mask[:, t] = ok[t]
    del idx, i, j, k
    counts = mask.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    col = cols[mask]
    val = np.where(col.astype(np.int64) == np.repeat(np.arange(n, dtype=np.int64), counts), 6.0, -1.0)
    return rowptr, col, val.astype(np.float32)


def random_csr(nrows: int, ncols: int, seed: int = SEED_SPARSE, max_len: int = 40,
               empty_frac: float = 0.0, integer: bool = False):
    """A random compressed-row matrix with ragged rows.

    Row lengths are uniform on 1..max_len (a fraction empty_frac of rows is
    empty), columns distinct, uniform over 0..ncols-1 and ascending; values
    U[-1, 1) cast to FP32, or integers in [-3, 3] when integer is set.
    Returns (rowptr int64, col int32, val float32).
    """
    rng = np.random.default_rng(seed)
    lens = rng.integers(1, max_len + 1, nrows)
    lens = np.minimum(lens, ncols)
    if empty_frac > 0:
        lens[rng.random(nrows) < empty_frac] = 0
    rowptr = np.zeros(nrows + 1, dtype=np.int64)
    np.cumsum(lens, out=rowptr[1:])
    col = np.empty(int(rowptr[-1]), dtype=np.int32)
    for r in range(nrows):
        if lens[r]:
            col[rowptr[r]:rowptr[r + 1]] = np.sort(rng.choice(ncols, int(lens[r]), replace=False))
    if integer:
        val = rng.integers(-3, 4, col.size).astype(np.float32)
    else:
        val = rng.uniform(-1.0, 1.0, col.size).astype(np.float32)
    return rowptr, col, val


def random_spd_csr(n: int, seed: int = SEED_SPARSE, max_partners: int = 12):
    """A random symmetric, strictly diagonally dominant matrix (hence SPD).

    Each row i picks 1..max_partners partners j != i uniformly; the pattern is
    made symmetric, each off-diagonal pair gets one value -U(0, 1), and the
    diagonal is 1 + the sum of the row's off-diagonal magnitudes. Values are
    cast to FP32 (dominance keeps a margin of about 1). Columns ascending.
    Returns (rowptr int64, col int32, val float32).
    """
    rng = np.random.default_rng(seed)
    k = rng.integers(1, max_partners + 1, n)
    rows = np.repeat(np.arange(n, dtype=np.int64), k)
    cols = rng.integers(0, n - 1, rows.size)
    cols = np.where(cols >= rows, cols + 1, cols)  # j != i
    lo, hi = np.minimum(rows, cols), np.maximum(rows, cols)
    pairs = np.unique(lo * n + hi)
    vals = -rng.uniform(0.0, 1.0, pairs.size)
    pi, pj = pairs // n, pairs % n
    r = np.concatenate([pi, pj, np.arange(n)])
    c = np.concatenate([pj, pi, np.arange(n)])
    off = np.abs(vals)
    diag = 1.0 + np.bincount(pi, off, n) + np.bincount(pj, off, n)
    v = np.concatenate([vals, vals, diag])
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=n), out=rowptr[1:])
    return rowptr, c.astype(np.int32), v.astype(np.float32)
