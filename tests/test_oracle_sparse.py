"""Pins of the oracle's compressed-row SpMV (no GPU).

The SpMV is the fourth building block of the GPU comparison system's CG in
the paper's Sec. VII-A (norm, dot, axpy, SpMV), there on the seven-point
operator stored in a sliced-ELLPACK format. The oracle computes the plain
definition y_i = sum over row i's entries of a_ij x_j; the pins below fix it
by closed forms (sine eigenvectors of the seven-point matrix, its row sums),
brute force on a dense copy built entry by entry, and symmetry. Jacobi-PCG
on a compressed-row matrix is pinned to the matrix-free oracle's steps on the
stored seven-point matrix, to a dense Cholesky solve, to the monotone A-norm
error of CG, to the one-step solve of a diagonal matrix, and to its status
paths.
"""
import math

import numpy as np
import pytest

import synthetic


@pytest.mark.parametrize("shape,modes", [((5, 7, 9), (1, 2, 3)), ((8, 8, 8), (1, 1, 1)), ((3, 11, 6), (2, 5, 1))])
def test_poisson_csr_sine_eigenvectors(orc, shape, modes):
    """The seven-point matrix times a sine mode (1-based positions) is
    lambda times it, lambda = 6 - 2 sum cos(pi a / (n + 1))."""
    nz, ny, nx = shape
    a, b, c = modes
    rowptr, col, val = synthetic.poisson7_csr(nx, ny, nz)
    v = synthetic.sine_mode(nx, ny, nz, a, b, c)
    lam = 6 - 2 * (math.cos(math.pi * a / (nx + 1)) + math.cos(math.pi * b / (ny + 1))
                   + math.cos(math.pi * c / (nz + 1)))
    y = orc.csr_spmv(rowptr, col, val, v)
    assert np.max(np.abs(y - lam * v)) <= 1e-13


def test_poisson_csr_row_sums(orc):
    """A 1 = number of ghost neighbours: 0 inside, 1 on a face, 2 on an edge,
    3 at a corner."""
    nx, ny, nz = 6, 5, 4
    rowptr, col, val = synthetic.poisson7_csr(nx, ny, nz)
    y = orc.csr_spmv(rowptr, col, val, np.ones(nx * ny * nz))
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ghosts = sum(m.astype(np.int64) for m in (i == 0, i == nx - 1, j == 0, j == ny - 1, k == 0, k == nz - 1))
    ghosts = ghosts.reshape(-1)
    assert np.array_equal(y, ghosts.astype(np.float64))


def test_poisson_csr_matches_matrix_free_operator(orc):
    nx, ny, nz = 9, 4, 7
    x = synthetic.uniform(3, nx * ny * nz)
    y = orc.csr_spmv(*synthetic.poisson7_csr(nx, ny, nz), x)
    assert np.max(np.abs(y - orc.stencil(x, (nz, ny, nx)))) <= 1e-14


@pytest.mark.parametrize("nrows,ncols,empty", [(40, 31, 0.0), (57, 57, 0.3), (1, 9, 0.0)])
def test_csr_spmv_brute_force_integers(orc, nrows, ncols, empty):
    """Integer matrix and vector: the product equals, exactly, the dense copy
    (filled entry by entry) multiplied with plain loops."""
    rowptr, col, val = synthetic.random_csr(nrows, ncols, seed=21, max_len=12, empty_frac=empty, integer=True)
    x = synthetic.integers(22, ncols, -5, 5).astype(np.float64)
    dense = [[0.0] * ncols for _ in range(nrows)]
    for r in range(nrows):
        for k in range(int(rowptr[r]), int(rowptr[r + 1])):
            dense[r][int(col[k])] += float(val[k])
    ref = [sum(dense[r][c] * x[c] for c in range(ncols)) for r in range(nrows)]
    y = orc.csr_spmv(rowptr, col, val, x)
    assert y.tolist() == ref


def test_csr_spmv_symmetry(orc):
    """<A x, y> = <x, A y> for the symmetric seven-point matrix."""
    nx, ny, nz = 7, 6, 5
    csr = synthetic.poisson7_csr(nx, ny, nz)
    x, y = synthetic.uniform(4, nx * ny * nz), synthetic.uniform(5, nx * ny * nz)
    lhs = float(np.dot(orc.csr_spmv(*csr, x), y))
    rhs = float(np.dot(x, orc.csr_spmv(*csr, y)))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)


def test_csr_spmv_empty_rows_and_matrix(orc):
    rowptr = np.array([0, 0, 2, 2], dtype=np.int64)
    col = np.array([1, 0], dtype=np.int32)
    val = np.array([2.0, -1.0], dtype=np.float32)
    y = orc.csr_spmv(rowptr, col, val, np.array([3.0, 5.0]))
    assert y.tolist() == [0.0, 7.0, 0.0]
    assert orc.csr_spmv(np.zeros(1, dtype=np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32),
                        np.zeros(4)).size == 0


# ---------------------------------------------------------------------------
# Jacobi-PCG on a compressed-row matrix
# ---------------------------------------------------------------------------

def test_csr_pcg_matches_matrix_free_pcg(orc):
    """On the stored seven-point matrix the CSR solve takes the matrix-free
    oracle's steps: same iteration count and residual history, same x."""
    nx, ny, nz = 12, 10, 9
    b = synthetic.uniform(7, nx * ny * nz)
    a = orc.csr_pcg(*synthetic.poisson7_csr(nx, ny, nz), b, rtol=1e-8, maxit=500, history=True)
    m = orc.pcg((nz, ny, nx), b, rtol=1e-8, maxit=500, history=True)
    assert a["status"] == m["status"] == orc.OK and a["iters"] == m["iters"]
    assert np.max(np.abs(a["hist"] - m["hist"])) <= 1e-12
    assert np.max(np.abs(a["x"] - m["x"])) <= 1e-12 * np.max(np.abs(m["x"]))


def _dense(rowptr, col, val, n):
    A = np.zeros((n, n))
    for r in range(n):
        for k in range(rowptr[r], rowptr[r + 1]):
            A[r, col[k]] += float(val[k])
    return A


def test_random_spd_generator_is_spd(orc):
    rowptr, col, val = synthetic.random_spd_csr(200, seed=3)
    A = _dense(rowptr, col, val, 200)
    assert np.array_equal(A, A.T)
    np.linalg.cholesky(A)
    assert np.all(np.diff(col[rowptr[0]:rowptr[1]]) > 0)


def test_csr_pcg_against_cholesky(orc):
    """Converged x against a dense Cholesky solve: ||x - x*||_A <= rtol ||b||
    times ||A^-1||^(1/2), and the A-norm error falls monotonically (a CG
    property) along truncated runs."""
    n = 300
    rowptr, col, val = synthetic.random_spd_csr(n, seed=5)
    A = _dense(rowptr, col, val, n)
    b = synthetic.uniform(9, n)
    L = np.linalg.cholesky(A)
    xs = np.linalg.solve(L.T, np.linalg.solve(L, b))
    res = orc.csr_pcg(rowptr, col, val, b, rtol=1e-10, maxit=1000)
    assert res["status"] == orc.OK
    lam_min = np.linalg.eigvalsh(A)[0]
    e = res["x"] - xs
    assert math.sqrt(e @ A @ e) <= 1e-10 * np.linalg.norm(b) / math.sqrt(lam_min) * 1.01
    prev = math.inf
    for k in range(1, 12):
        xk = orc.csr_pcg(rowptr, col, val, b, rtol=0.0, maxit=k)["x"]
        ek = xk - xs
        en = math.sqrt(ek @ A @ ek)
        assert en < prev
        prev = en


def test_csr_pcg_diagonal_matrix_one_step(orc):
    """A diagonal matrix is its own Jacobi preconditioner: one step, exact."""
    n = 50
    d = 1.0 + np.arange(n, dtype=np.float64)
    rowptr = np.arange(n + 1, dtype=np.int64)
    res = orc.csr_pcg(rowptr, np.arange(n, dtype=np.int32), d, np.ones(n), rtol=1e-14, maxit=10)
    assert res["status"] == orc.OK and res["iters"] == 1
    assert np.max(np.abs(res["x"] - 1.0 / d)) <= 1e-15


def test_csr_pcg_status_paths(orc):
    rowptr, col, val = synthetic.random_spd_csr(40, seed=6)
    zero = orc.csr_pcg(rowptr, col, val, np.zeros(40))
    assert zero["status"] == orc.OK and zero["iters"] == 0 and np.all(zero["x"] == 0)
    noconv = orc.csr_pcg(rowptr, col, val, synthetic.uniform(1, 40), rtol=1e-14, maxit=2)
    assert noconv["status"] == orc.NOCONV and noconv["iters"] == 2
    neg = orc.csr_pcg(rowptr, col, -val, synthetic.uniform(1, 40))  # diagonal not positive
    assert neg["status"] == orc.BREAKDOWN and neg["iters"] == 0
