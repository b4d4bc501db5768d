"""Pins of the oracle's single-reduction Jacobi-PCG (Chronopoulos-Gear,
J. Comput. Appl. Math. 25, 1989): the s = 1 case of s-step CG, which carries
s = A p by a recurrence so an iteration takes its two inner products
together. In exact arithmetic its iterates are those of CG; these tests pin
it to closed forms, a dense Cholesky solve, an independently assembled
matrix with scipy's CG, and the Hestenes-Stiefel oracle. No GPU."""
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synthetic

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _distinct_counts():
    out = {}
    with open(os.path.join(GOLD, "distinct_eigs.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                n, d = line.split()
                out[int(n)] = int(d)
    return out


def _lam(n, a, b, c):
    return 6 - 2 * (math.cos(math.pi * a / (n + 1)) + math.cos(math.pi * b / (n + 1))
                    + math.cos(math.pi * c / (n + 1)))


def test_sr_eigenvector_one_step(orc):
    """b = one eigenvector of the Laplacian: one step, x = v / lambda."""
    n = 16
    v = synthetic.sine_mode(n, n, n, 2, 3, 1)
    out = orc.pcg_sr((n, n, n), v, rtol=1e-12, maxit=50)
    assert out["status"] == orc.OK and out["iters"] == 1
    assert np.max(np.abs(out["x"] - v / _lam(n, 2, 3, 1))) < 1e-13


def test_sr_m_eigenvectors(orc):
    """b = sum of m eigenvectors with distinct eigenvalues: exactly m steps."""
    n = 12
    modes = [(1, 1, 1), (2, 1, 1), (3, 2, 1), (5, 5, 5)]
    lams = [_lam(n, *m) for m in modes]
    b = sum(synthetic.sine_mode(n, n, n, *m) for m in modes)
    out = orc.pcg_sr((n, n, n), b, rtol=1e-11, maxit=50)
    assert out["status"] == orc.OK and out["iters"] == 4
    xe = sum(synthetic.sine_mode(n, n, n, *m) / l for m, l in zip(modes, lams))
    assert np.max(np.abs(out["x"] - xe)) < 1e-11


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_sr_tiny_grids_vs_cholesky(orc, n):
    """Tiny grids: the dense Cholesky solution, in at most as many steps as A
    has distinct eigenvalues (golden counts)."""
    shape = (n, n, n)
    A = orc.assemble_dense(shape)
    b = synthetic.uniform(40 + n, n ** 3)
    xc = sla.cho_solve(sla.cho_factor(A), b)
    out = orc.pcg_sr(shape, b, rtol=1e-13, maxit=200)
    assert out["status"] == orc.OK
    assert out["iters"] <= _distinct_counts()[n]
    assert np.max(np.abs(out["x"] - xc)) <= 1e-12 * np.max(np.abs(xc))


def test_sr_matches_scipy_cg(orc):
    """D = 6 I: the iterates of plain CG on an independently assembled matrix."""
    n = 10
    shape = (n, n, n)
    Ix = sp.identity(n)
    T = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1])
    A = (sp.kron(sp.kron(T, Ix), Ix) + sp.kron(sp.kron(Ix, T), Ix) + sp.kron(sp.kron(Ix, Ix), T)).tocsr()
    b = synthetic.uniform(21, n ** 3)
    its = []
    x_sp, info = spla.cg(A, b, rtol=1e-8, atol=0.0, maxiter=500, callback=lambda xk: its.append(1))
    assert info == 0
    out = orc.pcg_sr(shape, b, rtol=1e-8, maxit=500)
    assert abs(out["iters"] - len(its)) <= 1
    assert np.max(np.abs(out["x"] - x_sp)) <= 1e-7 * np.max(np.abs(x_sp))


def test_sr_iterates_equal_hestenes_stiefel(orc):
    """Variable coefficients (non-constant Jacobi): the residual history and
    the k-step iterates agree with the Hestenes-Stiefel form to rounding for
    the first steps, and both reach the Cholesky solution."""
    shape = (6, 5, 4)
    n = 120
    k = np.exp(synthetic.uniform(9, n))
    b = synthetic.uniform(10, n)
    a = orc.pcg(shape, b, rtol=1e-12, maxit=300, kcell=k, history=True)
    s = orc.pcg_sr(shape, b, rtol=1e-12, maxit=300, kcell=k, history=True)
    m = min(len(a["hist"]), len(s["hist"]), 15)
    assert np.allclose(a["hist"][:m], s["hist"][:m], rtol=1e-8, atol=0.0)
    for steps in (1, 3, 7):
        xa = orc.pcg(shape, b, rtol=0.0, maxit=steps, kcell=k)["x"]
        xs = orc.pcg_sr(shape, b, rtol=0.0, maxit=steps, kcell=k)["x"]
        assert np.max(np.abs(xa - xs)) <= 1e-10 * np.max(np.abs(xa))
    A = orc.assemble_dense(shape, kcell=k)
    xc = sla.cho_solve(sla.cho_factor(A), b)
    assert abs(s["iters"] - a["iters"]) <= 2
    assert np.max(np.abs(s["x"] - xc)) <= 1e-10 * np.max(np.abs(xc))


def test_sr_a_norm_error_monotone(orc):
    """The A-norm of the error decreases at every step (a CG property)."""
    shape = (5, 5, 5)
    A = orc.assemble_dense(shape)
    b = synthetic.uniform(7, 125)
    xs = sla.cho_solve(sla.cho_factor(A), b)
    prev = math.inf
    for k in range(1, 20):
        out = orc.pcg_sr(shape, b, rtol=0.0, maxit=k)
        e = out["x"] - xs
        en = math.sqrt(max(float(e @ A @ e), 0.0))
        assert en <= prev * (1 + 1e-12)
        prev = en
        if en < 1e-13:
            break


def test_sr_status_paths(orc):
    shape = (6, 6, 6)
    out = orc.pcg_sr(shape, np.zeros(216), x0=np.ones(216))
    assert out["status"] == orc.OK and out["iters"] == 0 and not np.any(out["x"])
    out = orc.pcg_sr(shape, synthetic.uniform(1, 216), rtol=1e-12, maxit=2)
    assert out["status"] == orc.NOCONV and out["iters"] == 2
    b = synthetic.uniform(1, 216)
    b[5] = np.nan
    out = orc.pcg_sr(shape, b, rtol=1e-6, maxit=10)
    assert out["status"] == orc.BREAKDOWN
    # a nonzero x0: the history starts from b - A x0
    x0 = synthetic.uniform(3, 216)
    out = orc.pcg_sr(shape, synthetic.uniform(1, 216), rtol=1e-10, maxit=200, x0=x0)
    assert out["status"] == orc.OK
    assert orc.true_relres(shape, synthetic.uniform(1, 216), out["x"]) <= 1e-9
