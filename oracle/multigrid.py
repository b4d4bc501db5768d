"""FP64 geometric multigrid V-cycle and PCG with it as the preconditioner.

TEST INFRASTRUCTURE ONLY (part of the oracle package; the product path never
imports it). The paper names multigrid as future work for its solver
(Sec. VIII); the method here is the textbook cell-centred geometric V-cycle
(Trottenberg, Oosterlee and Schueller, "Multigrid", 2001, ch. 2 and 5;
Wesseling, "An Introduction to Multigrid Methods", 1992), in plain numpy on
top of the oracle's FP64 operator. The readings where the method has choices:

* hierarchy: level l+1 halves every dimension of level l (coarse cell
  (I, J, K) is the union of fine cells 2I..2I+1, 2J..2J+1, 2K..2K+1) while all
  three dimensions are even and level l has more than `coarse_max` points;
* coarse operators by rediscretisation: the operator of level l is
  4^-l A[k_l] (A the seven-point operator, 6 / -1 for constant coefficients,
  the harmonic-mean face form for cell coefficients k_l), k_l being the mean
  of the eight children's k_(l-1); the 4^-l keeps the unscaled operator's
  h^2 factor consistent as the spacing doubles;
* prolongation P: per dimension a fine cell takes 3/4 of the coarse cell that
  contains it and 1/4 of the coarse cell on its other side (linear
  interpolation between cell centres), 0 outside the grid; the 3-D weights are
  the products; restriction R = P^T / 8;
* smoother: damped Jacobi u <- u + omega D^-1 (f - A u), omega = 6/7 (the
  best damping of the high frequencies of the 3-D seven-point operator, whose
  D^-1 A spectrum there is [1/3, 2]); nu1 sweeps before and nu2 after the
  coarse correction, from u = 0;
* coarsest level: exact solve (dense Cholesky factorisation in FP64).
With nu1 = nu2 the V-cycle is a symmetric positive definite operator, so it
serves as the preconditioner of ordinary PCG (Saad, Iterative Methods for
Sparse Linear Systems, Alg. 9.1).
"""
from __future__ import annotations

import math

import numpy as np

OMEGA = 6.0 / 7.0
COARSE_MAX = 512


def _ops():
    # the operator lives in the C part of the oracle package
    from . import stencil, vdiag, vstencil

    return stencil, vstencil, vdiag


class Level:
    """One grid of the hierarchy: shape (nz, ny, nx), cell coefficients
    (None: constant), and the scale 4^-l of its operator."""

    def __init__(self, shape, kcell, scale):
        self.shape = tuple(int(v) for v in shape)
        self.kcell = None if kcell is None else np.asarray(kcell, dtype=np.float64).reshape(-1)
        self.scale = float(scale)
        self.n = int(np.prod(self.shape))
        stencil, _, vdiag = _ops()
        if self.kcell is None:
            self.diag = np.full(self.n, 6.0 * self.scale)
        else:
            self.diag = self.scale * vdiag(self.kcell, self.shape)

    def apply(self, u):
        """The level's operator 4^-l A[k_l] applied to u."""
        stencil, vstencil, _ = _ops()
        u = np.asarray(u, dtype=np.float64).reshape(-1)
        if self.kcell is None:
            return self.scale * stencil(u, self.shape)
        return self.scale * vstencil(self.kcell, u, self.shape)


def coarsen_k(kcell, shape):
    """Mean of the eight children of each coarse cell."""
    nz, ny, nx = shape
    k = np.asarray(kcell, dtype=np.float64).reshape(nz // 2, 2, ny // 2, 2, nx // 2, 2)
    return k.mean(axis=(1, 3, 5)).reshape(-1)


def hierarchy(shape, kcell=None, coarse_max=COARSE_MAX):
    """The list of levels, finest first."""
    levels = [Level(shape, kcell, 1.0)]
    while True:
        cur = levels[-1]
        nz, ny, nx = cur.shape
        if cur.n <= coarse_max or nx % 2 or ny % 2 or nz % 2:
            break
        kc = None if cur.kcell is None else coarsen_k(cur.kcell, cur.shape)
        levels.append(Level((nz // 2, ny // 2, nx // 2), kc, cur.scale / 4.0))
    return levels


def prolong_1d(n):
    """Dense (n x n/2) linear interpolation between cell centres, zero
    outside: fine cell i lies in coarse cell i // 2 (weight 3/4); its other
    neighbour is i // 2 - 1 for even i, i // 2 + 1 for odd i (weight 1/4)."""
    nc = n // 2
    P = np.zeros((n, nc))
    for i in range(n):
        c = i // 2
        P[i, c] = 0.75
        o = c - 1 if i % 2 == 0 else c + 1
        if 0 <= o < nc:
            P[i, o] = 0.25
    return P


def _apply_axes(v, mats):
    """v (nz, ny, nx) multiplied along z, y and x by mats = (Mz, My, Mx)."""
    mz, my, mx = mats
    v = np.tensordot(mz, v, axes=([1], [0]))                     # (nz', ny, nx)
    v = np.tensordot(my, v, axes=([1], [1])).transpose(1, 0, 2)  # (nz', ny', nx)
    v = np.tensordot(v, mx, axes=([2], [1]))                     # (nz', ny', nx')
    return v


def prolong(ec, fine_shape):
    """Fine-grid vector P e_c."""
    nz, ny, nx = fine_shape
    e = np.asarray(ec, dtype=np.float64).reshape(nz // 2, ny // 2, nx // 2)
    return _apply_axes(e, (prolong_1d(nz), prolong_1d(ny), prolong_1d(nx))).reshape(-1)


def restrict(r, fine_shape):
    """Coarse-grid vector R r = P^T r / 8."""
    nz, ny, nx = fine_shape
    v = np.asarray(r, dtype=np.float64).reshape(nz, ny, nx)
    return (_apply_axes(v, (prolong_1d(nz).T, prolong_1d(ny).T, prolong_1d(nx).T)) / 8.0).reshape(-1)


def smooth(level, u, f, omega=OMEGA):
    """One damped-Jacobi sweep."""
    return u + omega * (f - level.apply(u)) / level.diag


def coarse_solver(level):
    """Cholesky factor of the coarsest operator (assembled column by column)."""
    n = level.n
    A = np.zeros((n, n))
    e = np.zeros(n)
    for j in range(n):
        e[:] = 0.0
        e[j] = 1.0
        A[:, j] = level.apply(e)
    return np.linalg.cholesky(A)


def _chol_solve(L, f):
    y = np.linalg.solve(L, f)
    return np.linalg.solve(L.T, y)


class VCycle:
    """The V-cycle of a hierarchy as an operator f -> u."""

    def __init__(self, shape, kcell=None, nu1=1, nu2=1, omega=OMEGA, coarse_max=COARSE_MAX):
        self.levels = hierarchy(shape, kcell, coarse_max)
        self.nu1, self.nu2, self.omega = int(nu1), int(nu2), float(omega)
        self.chol = coarse_solver(self.levels[-1])

    def __call__(self, f, l=0):
        lev = self.levels[l]
        f = np.asarray(f, dtype=np.float64).reshape(-1)
        if l == len(self.levels) - 1:
            return _chol_solve(self.chol, f)
        u = np.zeros_like(f)
        for _ in range(self.nu1):
            u = smooth(lev, u, f, self.omega)
        r = f - lev.apply(u)
        ec = self(restrict(r, lev.shape), l + 1)
        u = u + prolong(ec, lev.shape)
        for _ in range(self.nu2):
            u = smooth(lev, u, f, self.omega)
        return u


def mg_pcg(shape, b, rtol=1e-6, maxit=500, kcell=None, nu1=1, nu2=1, omega=OMEGA, coarse_max=COARSE_MAX,
           history=False):
    """PCG (Saad Alg. 9.1) with M^-1 = the V-cycle, x0 = 0, stopping on the
    recursive ||r|| <= rtol ||b||. Returns dict(x, iters, status, relres[, hist])
    with status 0 (converged), 3 (maxit) or 4 (breakdown: p.Ap <= 0)."""
    V = VCycle(shape, kcell, nu1, nu2, omega, coarse_max)
    A = V.levels[0]
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    x = np.zeros_like(b)
    r = b.copy()
    nb = math.sqrt(float(np.dot(b, b)))
    hist = [1.0 if nb > 0 else 0.0]
    if nb == 0.0:
        out = dict(x=x, iters=0, status=0, relres=0.0)
        if history:
            out["hist"] = np.array(hist)
        return out
    z = V(r)
    p = z.copy()
    rho = float(np.dot(r, z))
    status, it = 3, 0
    for it in range(1, maxit + 1):
        q = A.apply(p)
        sigma = float(np.dot(p, q))
        if not (sigma > 0.0) or not math.isfinite(sigma):
            status, it = 4, it - 1
            break
        alpha = rho / sigma
        x += alpha * p
        r -= alpha * q
        nr = math.sqrt(float(np.dot(r, r)))
        hist.append(nr / nb)
        if nr <= rtol * nb:
            status = 0
            break
        z = V(r)
        rho_new = float(np.dot(r, z))
        p = z + (rho_new / rho) * p
        rho = rho_new
    out = dict(x=x, iters=it, status=status, relres=hist[-1], levels=len(V.levels))
    if history:
        out["hist"] = np.array(hist)
    return out
