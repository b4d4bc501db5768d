"""Pins of the oracle's operator and BLAS-1 against closed forms, invariants,
brute force and library routines (no GPU).

Operator: the paper's Sec. VI seven-point stencil used as the matrix-free
operator of Sec. VII (zero Dirichlet boundaries, weights 6 / -1).
"""
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

import synthetic

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold_rows(name):
    rows = []
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                rows.append([float(v) for v in line.split()])
    return rows


def _lap1d(n):
    return sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1])


def _kron_sum(nx, ny, nz):
    """Independent assembly: A = Tz (x) I (x) I + I (x) Ty (x) I + I (x) I (x) Tx,
    matching memory order [z][y][x]."""
    Ix, Iy, Iz = sp.identity(nx), sp.identity(ny), sp.identity(nz)
    return (sp.kron(sp.kron(_lap1d(nz), Iy), Ix) + sp.kron(sp.kron(Iz, _lap1d(ny)), Ix)
            + sp.kron(sp.kron(Iz, Iy), _lap1d(nx))).tocsr()


@pytest.mark.parametrize("shape,modes", [((8, 8, 8), (1, 1, 1)), ((7, 9, 11), (2, 3, 5)),
                                         ((16, 12, 10), (4, 1, 9)), ((32, 32, 32), (31, 1, 16))])
def test_sine_eigenvectors(orc, shape, modes):
    """A v = lambda v for v = prod sin(pi a (i+1)/(n+1)) (1-based positions),
    lambda = 6 - 2 (cos(pi a/(nx+1)) + cos(pi b/(ny+1)) + cos(pi c/(nz+1)))."""
    nz, ny, nx = shape
    a, b, c = modes
    v = synthetic.sine_mode(nx, ny, nz, a, b, c)
    lam = 6 - 2 * (math.cos(math.pi * a / (nx + 1)) + math.cos(math.pi * b / (ny + 1))
                   + math.cos(math.pi * c / (nz + 1)))
    y = orc.stencil(v, shape)
    assert np.max(np.abs(y - lam * v)) <= 1e-13 * 8


def _quad(coef, i, j, k):
    (cxx, cyy, czz, cxy, cxz, cyz, cx, cy, cz, c0) = coef
    return (cxx * i * i + cyy * j * j + czz * k * k + cxy * i * j + cxz * i * k + cyz * j * k
            + cx * i + cy * j + cz * k + c0)


@pytest.mark.parametrize("shape", [(5, 6, 7), (3, 3, 3), (9, 4, 6)])
def test_quadratics_exact(orc, shape):
    """(A q)_p = -2 (a_xx + a_yy + a_zz) + sum over p's out-of-grid neighbours g
    of q(g): second differences of a quadratic are exact, mixed and linear
    terms cancel, and each missing neighbour adds back the value it would have
    subtracted. All values are integers, so the comparison is exact."""
    nz, ny, nx = shape
    rng = np.random.default_rng(11)
    coef = [int(v) for v in rng.integers(-3, 4, 10)]
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    q = _quad(coef, i, j, k).astype(np.float64).reshape(-1)
    y = orc.stencil(q, shape).reshape(shape)
    base = -2 * (coef[0] + coef[1] + coef[2])
    for kk in range(nz):
        for jj in range(ny):
            for ii in range(nx):
                exp = base
                for (a, b, c) in ((ii - 1, jj, kk), (ii + 1, jj, kk), (ii, jj - 1, kk),
                                  (ii, jj + 1, kk), (ii, jj, kk - 1), (ii, jj, kk + 1)):
                    if not (0 <= a < nx and 0 <= b < ny and 0 <= c < nz):
                        exp += _quad(coef, a, b, c)
                assert y[kk, jj, ii] == exp


def test_rowsum_golden(orc):
    ones = np.ones(27)
    y = orc.stencil(ones, (3, 3, 3))
    gold = np.array(_gold_rows("rowsum_3x3x3.txt")).reshape(-1)
    assert np.array_equal(y, gold)


def test_rowsum_counts(orc):
    shape = (6, 5, 4)
    y = orc.stencil(np.ones(120), shape).reshape(shape)
    nz, ny, nx = shape
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                g = (i == 0) + (i == nx - 1) + (j == 0) + (j == ny - 1) + (k == 0) + (k == nz - 1)
                assert y[k, j, i] == g


def test_against_kron_assembly(orc):
    """The oracle's operator equals an independent Kronecker-sum assembly."""
    shape = (5, 7, 6)
    A = _kron_sum(6, 7, 5)
    x = synthetic.uniform(3, 210)
    assert np.max(np.abs(orc.stencil(x, shape) - A @ x)) < 1e-14


def test_brute_force_integer(orc):
    """Pure-Python loop twin agrees bit-for-bit on integer data."""
    shape = (4, 5, 6)
    x = synthetic.integers(5, 120, -1000, 1000).astype(np.float64)
    assert np.array_equal(orc.stencil(x, shape), orc.stencil_loops(x, shape))


def test_symmetric_positive_definite(orc):
    A = orc.assemble_dense((3, 4, 5))
    assert np.array_equal(A, A.T)
    np.linalg.cholesky(A)
    x, y = synthetic.uniform(1, 60), synthetic.uniform(2, 60)
    sh = (3, 4, 5)
    assert abs(np.dot(orc.stencil(x, sh), y) - np.dot(x, orc.stencil(y, sh))) < 1e-12


def test_eigs_2x2x2_golden(orc):
    A = orc.assemble_dense((2, 2, 2))
    ev = np.sort(np.linalg.eigvalsh(A))
    gold = np.array(_gold_rows("eigs_2x2x2.txt")[0])
    assert np.max(np.abs(ev - gold)) < 1e-12


def test_axpy_and_dot(orc):
    x, y = synthetic.uniform(2, 100003), synthetic.uniform(3, 100003)
    assert np.array_equal(orc.axpy(0.5, x, y), 0.5 * x + y)
    d = orc.dot(x, y)
    assert abs(d - math.fsum(x * y)) <= 1e-12 * np.sum(np.abs(x * y))


def test_dot_integers_exact(orc):
    x = synthetic.integers(7, 200000, -2, 2).astype(np.float64)
    y = synthetic.integers(8, 200000, -2, 2).astype(np.float64)
    assert orc.dot(x, y) == float(np.sum(x.astype(np.int64) * y.astype(np.int64)))


def test_dot_empty(orc):
    assert orc.dot(np.zeros(0), np.zeros(0)) == 0.0


def test_vstencil_unit_coefficient(orc):
    """k = 1 reproduces the constant operator (exact on integers)."""
    shape = (5, 6, 7)
    x = synthetic.integers(9, 210, -50, 50).astype(np.float64)
    k = np.ones(210)
    assert np.array_equal(orc.vstencil(k, x, shape), orc.stencil(x, shape))
    assert np.array_equal(orc.vdiag(k, shape), np.full(210, 6.0))


def test_vstencil_constant_coefficient(orc):
    shape = (4, 6, 5)
    x = synthetic.integers(9, 120, -50, 50).astype(np.float64)
    assert np.array_equal(orc.vstencil(np.full(120, 4.0), x, shape), 4.0 * orc.stencil(x, shape))


def _fv_assembly(kc, shape):
    """Independent edge-by-edge assembly: each interior face between p and q
    with harmonic-mean coefficient kf adds kf to A_pp and A_qq and -kf to A_pq
    and A_qp; each boundary face of p adds k_p to A_pp."""
    nz, ny, nx = shape
    n = nx * ny * nz
    A = np.zeros((n, n))
    kk = kc.reshape(shape)

    def idx(i, j, k):
        return (k * ny + j) * nx + i

    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                p = idx(i, j, k)
                for (a, b, c) in ((i + 1, j, k), (i, j + 1, k), (i, j, k + 1)):
                    if a < nx and b < ny and c < nz:
                        q = idx(a, b, c)
                        kf = 2 * kk[k, j, i] * kk[c, b, a] / (kk[k, j, i] + kk[c, b, a])
                        A[p, p] += kf
                        A[q, q] += kf
                        A[p, q] -= kf
                        A[q, p] -= kf
                nbnd = (i == 0) + (i == nx - 1) + (j == 0) + (j == ny - 1) + (k == 0) + (k == nz - 1)
                A[p, p] += nbnd * kk[k, j, i]
    return A


def test_vstencil_against_fv_assembly(orc):
    shape = (3, 4, 5)
    kc = np.exp(synthetic.uniform(12, 60))
    A = _fv_assembly(kc, shape)
    Ad = orc.assemble_dense(shape, kcell=kc)
    assert np.max(np.abs(A - Ad)) < 1e-13
    assert np.max(np.abs(Ad - Ad.T)) < 1e-14
    np.linalg.cholesky(Ad)
    assert np.max(np.abs(orc.vdiag(kc, shape) - np.diag(A))) < 1e-13


def test_vstencil_rowsum(orc):
    """A_k 1 = sum of boundary-face coefficients = k_p times p's boundary faces."""
    shape = (4, 5, 6)
    nz, ny, nx = shape
    kc = np.exp(synthetic.uniform(13, 120))
    y = orc.vstencil(kc, np.ones(120), shape).reshape(shape)
    kk = kc.reshape(shape)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                g = (i == 0) + (i == nx - 1) + (j == 0) + (j == ny - 1) + (k == 0) + (k == nz - 1)
                assert abs(y[k, j, i] - g * kk[k, j, i]) <= 1e-13 * max(1.0, kk[k, j, i])


def test_grf_statistics():
    """Squared-exponential field: unit variance and lag-l autocorrelation
    close to exp(-1/2) at l = 8 cells."""
    g = synthetic.gaussian_random_field(64).reshape(64, 64, 64)
    assert abs(g.mean()) < 1e-12 and abs(g.std() - 1) < 1e-12
    lag = 8
    c = np.mean(g[:, :, :-lag] * g[:, :, lag:]) / np.mean(g * g)
    assert abs(c - math.exp(-0.5)) < 0.1
