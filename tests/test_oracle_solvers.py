"""Pins of the oracle's solvers: Jacobi-PCG (paper Sec. VII), the emulated
mixed-precision iterative refinement, flexible CG, and the reduced-precision
rounding helpers. No GPU."""
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla
import torch

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


def test_pcg_eigenvector_one_step(orc):
    """b = one eigenvector: CG ends after one step with x = v / lambda."""
    n = 16
    v = synthetic.sine_mode(n, n, n, 2, 3, 1)
    out = orc.pcg((n, n, n), v, rtol=1e-12, maxit=50)
    assert out["status"] == orc.OK and out["iters"] == 1
    assert np.max(np.abs(out["x"] - v / _lam(n, 2, 3, 1))) < 1e-13


def test_pcg_m_eigenvectors(orc):
    """b = sum of m eigenvectors with distinct eigenvalues: exactly m steps."""
    n = 12
    modes = [(1, 1, 1), (2, 1, 1), (3, 2, 1), (5, 5, 5)]
    lams = [_lam(n, *m) for m in modes]
    assert len(set(round(l, 12) for l in lams)) == 4
    b = sum(synthetic.sine_mode(n, n, n, *m) for m in modes)
    out = orc.pcg((n, n, n), b, rtol=1e-11, maxit=50)
    assert out["status"] == orc.OK and out["iters"] == 4
    xe = sum(synthetic.sine_mode(n, n, n, *m) / l for m, l in zip(modes, lams))
    assert np.max(np.abs(out["x"] - xe)) < 1e-11


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_pcg_tiny_grids_vs_cholesky(orc, n):
    """Tiny grids: PCG matches a dense Cholesky solve and needs at most as many
    steps as A has distinct eigenvalues (golden counts)."""
    shape = (n, n, n)
    A = orc.assemble_dense(shape)
    b = synthetic.uniform(40 + n, n ** 3)
    xc = sla.cho_solve(sla.cho_factor(A), b)
    out = orc.pcg(shape, b, rtol=1e-13, maxit=200)
    assert out["status"] == orc.OK
    assert out["iters"] <= _distinct_counts()[n]
    assert np.max(np.abs(out["x"] - xc)) <= 1e-12 * np.max(np.abs(xc))


def test_pcg_a_norm_error_monotone(orc):
    """The A-norm of the error decreases at every CG step."""
    shape = (5, 5, 5)
    A = orc.assemble_dense(shape)
    b = synthetic.uniform(7, 125)
    xs = sla.cho_solve(sla.cho_factor(A), b)
    prev = math.inf
    for k in range(1, 20):
        out = orc.pcg(shape, b, rtol=0.0, maxit=k)
        e = out["x"] - xs
        en = math.sqrt(max(float(e @ A @ e), 0.0))
        assert en <= prev * (1 + 1e-12)
        prev = en
        if en < 1e-13:
            break


def test_pcg_matches_scipy_cg(orc):
    """Jacobi with D = 6 I gives the iterates of unpreconditioned CG, so the
    oracle matches scipy's CG on an independently assembled matrix."""
    n = 10
    shape = (n, n, n)
    Ix = sp.identity(n)
    T = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1])
    A = (sp.kron(sp.kron(T, Ix), Ix) + sp.kron(sp.kron(Ix, T), Ix) + sp.kron(sp.kron(Ix, Ix), T)).tocsr()
    b = synthetic.uniform(21, n ** 3)
    its = []
    x_sp, info = spla.cg(A, b, rtol=1e-8, atol=0.0, maxiter=500, callback=lambda xk: its.append(1))
    assert info == 0
    out = orc.pcg(shape, b, rtol=1e-8, maxit=500)
    assert abs(out["iters"] - len(its)) <= 1
    assert np.max(np.abs(out["x"] - x_sp)) <= 1e-7 * np.max(np.abs(x_sp))


def test_pcg_status_paths(orc):
    shape = (6, 6, 6)
    # b = 0 -> x = 0, zero iterations
    out = orc.pcg(shape, np.zeros(216), x0=np.ones(216))
    assert out["status"] == orc.OK and out["iters"] == 0 and not np.any(out["x"])
    # maxit exhausted
    out = orc.pcg(shape, synthetic.uniform(1, 216), rtol=1e-12, maxit=2)
    assert out["status"] == orc.NOCONV and out["iters"] == 2
    # NaN in b -> breakdown
    b = synthetic.uniform(1, 216)
    b[5] = np.nan
    out = orc.pcg(shape, b, rtol=1e-6, maxit=10)
    assert out["status"] == orc.BREAKDOWN


def test_pcg_history_and_relres(orc):
    shape = (32, 32, 32)
    b = synthetic.uniform_f32(synthetic.SEED_C1_B, 32 ** 3).astype(np.float64)
    out = orc.pcg(shape, b, rtol=1e-6, maxit=500, history=True)
    assert out["status"] == orc.OK
    h = out["hist"]
    assert h[0] == 1.0 and h[-1] <= 1e-6 and np.all(h[:-1] > 1e-6)
    assert abs(orc.true_relres(shape, b, out["x"]) - out["relres"]) < 1e-9


def test_variable_pcg_vs_cholesky(orc):
    shape = (4, 5, 6)
    kc = np.exp(synthetic.uniform(30, 120))
    A = orc.assemble_dense(shape, kcell=kc)
    b = synthetic.uniform(31, 120)
    xc = sla.cho_solve(sla.cho_factor(A), b)
    out = orc.pcg(shape, b, rtol=1e-13, maxit=500, kcell=kc)
    assert out["status"] == orc.OK
    assert np.max(np.abs(out["x"] - xc)) <= 1e-11 * np.max(np.abs(xc))


# ---------------------------------------------------------------- rounding

def _special_values():
    f = np.float32
    vals = [0.0, -0.0, 1.0, -1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -9, 1.0 + 3 * 2 ** -9, 1.0 + 2 ** -11,
            1.0 + 2 ** -12, 1.0 + 3 * 2 ** -12, 65504.0, 65519.0, 65520.0, 70000.0, 2 ** -14,
            2 ** -24, 2 ** -25, 3 * 2 ** -25, 2 ** -126, 2 ** -130, 3.0e38, np.inf, -np.inf]
    return np.array(vals + list(synthetic.uniform(5, 5000) * 10.0 ** np.arange(-6, 4).repeat(500)),
                    dtype=np.float64)


def test_round_f32_matches_numpy(orc):
    x = np.concatenate([_special_values(), synthetic.uniform(9, 10000) * 1e-3])
    assert np.array_equal(orc.round_f32(x), x.astype(np.float32).astype(np.float64))


def test_round_f16_matches_numpy(orc):
    x = _special_values().astype(np.float32)
    ref = x.astype(np.float16).astype(np.float64)
    got = orc.round_f16(x.astype(np.float64))
    assert np.array_equal(got, ref)


def test_round_bf16_matches_torch(orc):
    x = _special_values().astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    got = orc.round_bf16(x.astype(np.float64))
    assert np.array_equal(got, ref)


# ---------------------------------------------------------------- refinement

@pytest.mark.parametrize("fmt", ["bf16", "f16"])
def test_ir_reaches_1e10(orc, fmt):
    """The FP64 true residual is the criterion: <= 1e-10 after refinement, with
    contraction at every outer step."""
    n = 16
    shape = (n, n, n)
    xs = synthetic.smooth_plus_noise(n)
    b = orc.stencil(xs, shape)
    out = orc.ir_emulate(shape, b, fmt=fmt, rtol_outer=1e-10)
    h = out["history"]
    assert h[-1] <= 1e-10
    assert all(h[i + 1] < h[i] for i in range(len(h) - 1))
    assert out["outer"] <= 12
    assert orc.true_relres(shape, b, out["x"]) <= 1e-10


def test_ir_fp64_inner_one_step(orc):
    """With an FP64 inner solve to 1e-12 one outer step suffices."""
    n = 12
    shape = (n, n, n)
    b = synthetic.uniform(3, n ** 3)
    out = orc.ir_emulate(shape, b, fmt="f64", rtol_outer=1e-10, rtol_in=1e-12)
    assert out["outer"] == 1


# ---------------------------------------------------------------- flexible CG

def test_fcg_jacobi_equals_pcg(orc):
    shape = (12, 12, 12)
    b = synthetic.uniform(4, 12 ** 3)
    ref = orc.pcg(shape, b, rtol=1e-8, maxit=500)
    out = orc.fcg(shape, b, precond=None, rtol=1e-8, maxit=500)
    assert abs(out["iters"] - ref["iters"]) <= 1
    assert np.max(np.abs(out["x"] - ref["x"])) <= 1e-7 * np.max(np.abs(ref["x"]))


def test_fcg_exact_inverse_one_step(orc):
    shape = (4, 4, 4)
    A = orc.assemble_dense(shape)
    cf = sla.cho_factor(A)
    b = synthetic.uniform(5, 64)
    out = orc.fcg(shape, b, precond=lambda r: sla.cho_solve(cf, r), rtol=1e-10)
    assert out["iters"] == 1 and out["fallback_at"] is None


def test_fcg_fallback_on_indefinite(orc):
    """M(r) = -r is indefinite (z.r < 0): the solve falls back to Jacobi at once
    and then runs exactly like Jacobi-PCG."""
    shape = (10, 10, 10)
    b = synthetic.uniform(6, 1000)
    out = orc.fcg(shape, b, precond=lambda r: -r, rtol=1e-8)
    ref = orc.pcg(shape, b, rtol=1e-8, maxit=500)
    assert out["fallback_at"] == 0 and out["status"] == orc.OK
    assert abs(out["iters"] - ref["iters"]) <= 1


def test_fcg_fallback_on_stagnation(orc):
    """A preconditioner that is SPD but useless (a tiny multiple of identity is
    fine; instead use one that returns r scaled by huge noise) stagnates and
    triggers the fallback; the solve still reaches the tolerance."""
    shape = (10, 10, 10)
    b = synthetic.uniform(6, 1000)
    rng = np.random.default_rng(0)
    scale = np.exp(8 * rng.standard_normal(1000))  # wildly ill-conditioned SPD diagonal
    out = orc.fcg(shape, b, precond=lambda r: scale * r, rtol=1e-8, maxit=3000)
    assert out["status"] == orc.OK
    assert orc.true_relres(shape, b, out["x"]) <= 1e-7
