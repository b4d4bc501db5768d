"""Pins of the oracle's geometric multigrid V-cycle (oracle/multigrid.py):
closed forms of each part and the properties the method fixes.

* prolongation: linear interpolation between cell centres reproduces linear
  functions away from the boundary, and its 1-D weights are 3/4 and 1/4;
* restriction: R = P^T / 8 (adjointness), and a constant field restricts to
  the same constant away from the boundary;
* smoother: one damped-Jacobi sweep on a sine eigenvector of the operator
  multiplies it by 1 - omega lambda / 6 (closed-form eigenvalue);
* coarse operators: k = 1 coarsens to k = 1 and the level operator is
  4^-l times the seven-point operator; k = c scales it by c;
* coarsest level: the exact solve (a one-level V-cycle is A^-1);
* the V-cycle as an operator B: symmetric and positive definite (assembled
  densely on 8^3 with two and three levels, constant and variable
  coefficients), and its error propagation I - B A has eigenvalues below 1;
* PCG with it: the dense Cholesky solution on tiny grids, grid-independent
  iteration counts, termination within the number of distinct eigenvalues.
"""
import math

import numpy as np
import pytest

import synthetic


def test_prolong_1d_weights_by_hand(orc):
    P = orc.multigrid.prolong_1d(6)
    want = np.array([[0.75, 0.0, 0.0],    # fine 0: its coarse 0, other side outside
                     [0.75, 0.25, 0.0],   # fine 1: coarse 0, then coarse 1
                     [0.25, 0.75, 0.0],
                     [0.0, 0.75, 0.25],
                     [0.0, 0.25, 0.75],
                     [0.0, 0.0, 0.75]])
    assert np.array_equal(P, want)


def test_prolong_reproduces_linear_functions(orc):
    """Coarse cell centres sit at fine coordinate 2I + 1/2; a linear function
    sampled there interpolates exactly to the fine cell centres whose two
    coarse neighbours per dimension are inside the grid."""
    fs = (8, 10, 12)
    nz, ny, nx = fs
    Z, Y, X = np.meshgrid(2 * np.arange(nz // 2) + 0.5, 2 * np.arange(ny // 2) + 0.5, 2 * np.arange(nx // 2) + 0.5,
                          indexing="ij")
    ec = 1.5 + 0.25 * X - 2.0 * Y + 0.75 * Z
    u = orc.prolong(ec, fs).reshape(fs)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    lin = 1.5 + 0.25 * x - 2.0 * y + 0.75 * z
    inner = (slice(1, nz - 1), slice(1, ny - 1), slice(1, nx - 1))
    assert np.allclose(u[inner], lin[inner], rtol=0, atol=1e-12)


def test_restrict_is_adjoint_and_averages_constants(orc):
    fs = (6, 8, 10)
    n = int(np.prod(fs))
    r = synthetic.uniform(81, n)
    e = synthetic.uniform(82, n // 8)
    lhs = float(np.dot(orc.restrict(r, fs), e))
    rhs = float(np.dot(r, orc.prolong(e, fs))) / 8.0
    assert abs(lhs - rhs) <= 1e-13 * n
    c = orc.restrict(np.full(n, 3.0), fs).reshape(3, 4, 5)
    assert np.allclose(c[1:-1, 1:-1, 1:-1], 3.0, rtol=0, atol=1e-14)
    # a boundary coarse cell misses the 1/4 weights from outside the grid:
    # (3/4 + 3/4 + 1/4) / 2 = 7/8 per dimension at a face
    assert math.isclose(c[0, 1, 1], 3.0 * 7.0 / 8.0, rel_tol=1e-14)
    assert math.isclose(c[0, 0, 0], 3.0 * (7.0 / 8.0) ** 3, rel_tol=1e-14)


@pytest.mark.parametrize("mode", [(1, 1, 1), (3, 2, 5), (8, 7, 6)])
def test_smoother_on_sine_eigenvector(orc, mode):
    shape = (8, 9, 10)
    nz, ny, nx = shape
    a, b, c = mode
    v = synthetic.sine_mode(nx, ny, nz, a, b, c)
    lam = 6 - 2 * (math.cos(math.pi * a / (nx + 1)) + math.cos(math.pi * b / (ny + 1)) + math.cos(math.pi * c / (nz + 1)))
    lev = orc.hierarchy(shape)[0]
    for omega in (orc.multigrid.OMEGA, 0.5):
        u = orc.smooth(lev, v, np.zeros_like(v), omega)
        assert np.allclose(u, (1.0 - omega * lam / 6.0) * v, rtol=0, atol=1e-13)


def test_coarse_operators(orc):
    shape = (8, 8, 8)
    ones = orc.hierarchy(shape, np.ones(512), coarse_max=8)
    const = orc.hierarchy(shape, None, coarse_max=8)
    assert [lv.shape for lv in ones] == [(8, 8, 8), (4, 4, 4), (2, 2, 2)]
    assert [lv.scale for lv in ones] == [1.0, 0.25, 0.0625]
    for lk, lc in zip(ones, const):
        assert np.all(lk.kcell == 1.0)
        v = synthetic.uniform(83, lk.n)
        assert np.allclose(lk.apply(v), lc.apply(v), rtol=0, atol=1e-13)
        assert np.allclose(lc.apply(v), lc.scale * orc.stencil(v, lc.shape), rtol=0, atol=0)
    k = synthetic.coefficient_field(8).astype(np.float64).reshape(-1)
    for a, b in zip(orc.hierarchy(shape, k, coarse_max=8), orc.hierarchy(shape, 2.5 * k, coarse_max=8)):
        v = synthetic.uniform(84, a.n)
        assert np.allclose(b.apply(v), 2.5 * a.apply(v), rtol=1e-13, atol=1e-13)
    # a coarse cell's k is the mean of its eight children
    lv = orc.hierarchy(shape, k, coarse_max=8)
    assert math.isclose(lv[1].kcell[0], float(np.mean(k.reshape(8, 8, 8)[:2, :2, :2])), rel_tol=1e-14)
    # coarsening stops at an odd dimension and at coarse_max points
    assert [lv.shape for lv in orc.hierarchy((6, 8, 8), coarse_max=8)] == [(6, 8, 8), (3, 4, 4)]
    assert [lv.shape for lv in orc.hierarchy((8, 8, 8))] == [(8, 8, 8)]


def test_one_level_vcycle_is_the_exact_solve(orc):
    shape = (4, 5, 6)
    n = 120
    f = synthetic.uniform(85, n)
    V = orc.VCycle(shape)
    assert len(V.levels) == 1
    A = orc.assemble_dense(shape)
    assert np.allclose(V(f), np.linalg.solve(A, f), rtol=0, atol=1e-12)


def _dense_vcycle(orc, shape, kcell, coarse_max, nu=1):
    V = orc.VCycle(shape, kcell, nu1=nu, nu2=nu, coarse_max=coarse_max)
    n = int(np.prod(shape))
    B = np.zeros((n, n))
    e = np.zeros(n)
    for j in range(n):
        e[:] = 0.0
        e[j] = 1.0
        B[:, j] = V(e)
    return V, B


@pytest.mark.parametrize("coarse_max,nlev", [(64, 2), (8, 3)])
@pytest.mark.parametrize("var", [False, True])
def test_vcycle_symmetric_positive_definite(orc, coarse_max, nlev, var):
    shape = (8, 8, 8)
    k = synthetic.coefficient_field(8).astype(np.float64).reshape(-1) if var else None
    V, B = _dense_vcycle(orc, shape, k, coarse_max)
    assert len(V.levels) == nlev
    assert np.max(np.abs(B - B.T)) <= 1e-12 * np.max(np.abs(B))
    assert np.min(np.linalg.eigvalsh((B + B.T) / 2)) > 0
    A = orc.assemble_dense(shape, k)
    # B A is similar to A^1/2 B A^1/2: real spectrum; I - B A has eigenvalues < 1
    ev = np.sort(np.linalg.eigvals(B @ A).real)
    assert ev[0] > 0
    assert np.max(1.0 - ev) < 1.0
    # with two sweeps each side the error propagation contracts
    if not var:
        _, B2 = _dense_vcycle(orc, shape, k, coarse_max, nu=2)
        ev2 = np.sort(np.linalg.eigvals(B2 @ A).real)
        assert np.max(np.abs(1.0 - ev2)) < np.max(np.abs(1.0 - ev)) + 1e-12


@pytest.mark.parametrize("shape", [(4, 4, 4), (8, 6, 4), (8, 8, 8)])
def test_mg_pcg_matches_cholesky(orc, shape):
    n = int(np.prod(shape))
    b = synthetic.uniform(86, n)
    out = orc.mg_pcg(shape, b, rtol=1e-12, maxit=200, coarse_max=8)
    A = orc.assemble_dense(shape)
    L = np.linalg.cholesky(A)
    x = np.linalg.solve(L.T, np.linalg.solve(L, b))
    assert out["status"] == 0
    assert np.max(np.abs(out["x"] - x)) <= 1e-10 * np.max(np.abs(x))


def test_mg_pcg_terminates_within_distinct_eigenvalues(orc):
    """CG with an SPD preconditioner B terminates (in exact arithmetic) within
    the number of distinct eigenvalues of B A; check the residual is at
    rounding level by then on 4 x 4 x 4 with two levels."""
    shape = (4, 4, 4)
    V, B = _dense_vcycle(orc, shape, None, 8)
    A = orc.assemble_dense(shape)
    ev = np.sort(np.linalg.eigvals(B @ A).real)
    distinct = 1 + int(np.sum(np.diff(ev) > 1e-8 * ev[-1]))
    b = synthetic.uniform(87, 64)
    out = orc.mg_pcg(shape, b, rtol=1e-10, maxit=distinct, coarse_max=8)
    assert out["status"] == 0 and out["iters"] <= distinct


def test_mg_pcg_iterations_grid_independent(orc):
    """The point of the method: the iteration count barely grows with the
    grid, while Jacobi-PCG's doubles with each doubling of n."""
    its = []
    for n in (16, 32, 64):
        b = synthetic.uniform_f32(1, n ** 3).astype(np.float64)
        out = orc.mg_pcg((n, n, n), b, rtol=1e-6, maxit=100)
        assert out["status"] == 0
        assert orc.true_relres((n, n, n), b, out["x"]) <= 1e-6
        its.append(out["iters"])
    assert max(its) <= 15 and its[-1] - its[0] <= 3


def test_mg_pcg_zero_rhs_and_status(orc):
    out = orc.mg_pcg((8, 8, 8), np.zeros(512))
    assert out["status"] == 0 and out["iters"] == 0 and not np.any(out["x"])
    out = orc.mg_pcg((8, 8, 8), synthetic.uniform(88, 512), rtol=1e-14, maxit=2, coarse_max=8)
    assert out["status"] == 3 and out["iters"] == 2
