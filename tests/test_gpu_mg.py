"""GPU parity of the geometric multigrid V-cycle and PCG with it (the
preconditioner the paper names as future work, Sec. VIII) against the FP64
oracle (oracle/multigrid.py), through the C ABI.

Bars:
* hierarchy: the same levels as the oracle's;
* one V-cycle: |u - u_ref| <= 2e-5 max|u_ref| per element. Derivation: the
  GPU runs the oracle's steps in FP32 (unit roundoff 2^-24 = 6e-8); each
  level adds a few roundings per point to sweeps, residual and transfers, and
  the coarsest dense inverse (FP32 copy of an FP64 inverse, m <= 1024 terms
  per row) adds about sqrt(m) 2^-24 relative to the largest terms of A^-1 g;
  across 3-5 levels that stays below 1e-5 of the largest |u| — 2e-5 leaves a
  factor two;
* PCG with the V-cycle: iterations within 2 of the oracle's PCG with the
  FP64 V-cycle (FP32 vs FP64 arithmetic moves the stopping iteration by at
  most one or two at these counts), FP64 true residual <= rtol;
* at the benchmark's 256^3 (oracle too slow for the full solve there): the
  true residual, the grid-independent iteration count, and a V-cycle checked
  against the oracle at 128^3.
"""
import numpy as np
import pytest
import torch

import synthetic
from gpu_helpers import check_status, dev, host64

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2603_23343_amd as P

    return P


def _ctx(P, shape, kcell=None, nu=1, coarse_max=0):
    nz, ny, nx = shape
    ctx = P.pcg_create(nx, ny, nz, torch.float32, x_dtype=torch.float64)
    kd = None
    if kcell is not None:
        kd = dev(kcell.astype(np.float32))
        P.pcg_set_coefficients(ctx, kd)
    P.pcg_set_multigrid(ctx, nu=nu, coarse_max=coarse_max)
    return ctx, kd


CASES = [((32, 32, 32), False, 1), ((16, 24, 40), False, 1), ((32, 32, 32), True, 1), ((32, 32, 32), False, 2),
         ((24, 20, 16), True, 2), ((8, 8, 8), False, 1)]


@pytest.mark.parametrize("shape,var,nu", CASES)
def test_vcycle_matches_oracle(P, orc, shape, var, nu):
    n = int(np.prod(shape))
    print("vcycle", shape, "var" if var else "const", "nu", nu, flush=True)
    k = synthetic.coefficient_field(shape[0]).reshape(-1)[:n] if var and shape[0] == shape[1] == shape[2] else None
    if var and k is None:
        k = np.exp(synthetic.uniform(91, n)).astype(np.float32)
    ctx, kd = _ctx(P, shape, k, nu)
    V = orc.VCycle(shape, None if k is None else k.astype(np.float64), nu1=nu, nu2=nu)
    assert P.pcg_mg_levels(ctx) == [tuple(reversed(lv.shape)) for lv in V.levels]
    g32 = synthetic.uniform_f32(92, n)
    g = dev(g32)
    u = torch.empty_like(g)
    P.pcg_mg_apply(ctx, g, u)
    torch.cuda.synchronize()
    ref = V(g32.astype(np.float64))
    err = np.max(np.abs(host64(u) - ref))
    print("max err", err, "max |u|", np.max(np.abs(ref)), flush=True)
    assert err <= 2e-5 * np.max(np.abs(ref))
    ctx.close()


@pytest.mark.parametrize("shape,var", [((32, 32, 32), False), ((64, 64, 64), False), ((32, 32, 32), True),
                                       ((48, 40, 32), False)])
def test_mg_pcg_iterations(P, orc, shape, var):
    n = int(np.prod(shape))
    print("mg pcg", shape, var, flush=True)
    k = synthetic.coefficient_field(shape[0]).reshape(-1) if var else None
    ctx, kd = _ctx(P, shape, k)
    b32 = synthetic.uniform_f32(synthetic.SEED_C1_B, n)
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    info = P.pcg_solve_mg(ctx, dev(b32), x, 1e-6, 200, raise_on_error=False)
    ref = orc.mg_pcg(shape, b32.astype(np.float64), rtol=1e-6, maxit=200,
                     kcell=None if k is None else k.astype(np.float64))
    print("iters", info["iters"], "oracle", ref["iters"], "fallback", info["fallback_used"], flush=True)
    assert ref["status"] == 0
    check_status(P, info, 1e-6)
    assert info["status"] == P.PCG_OK and info["fallback_used"] == 0
    assert abs(info["iters"] - ref["iters"]) <= 2
    tr = orc.true_relres(shape, b32.astype(np.float64), host64(x), kcell=None if k is None else k.astype(np.float64))
    assert tr <= 1e-6 and abs(tr - info["rel_res_true_fp64"]) <= 1e-6 * tr
    ctx.close()


def test_mg_graph_and_eager_identical(P):
    shape = (32, 32, 32)
    n = 32 ** 3
    b = dev(synthetic.uniform_f32(93, n))
    outs = []
    for use_graph in (1, 0, 1):
        ctx = P.pcg_create(32, 32, 32, torch.float32, x_dtype=torch.float64, use_graph=use_graph)
        P.pcg_set_multigrid(ctx)
        x = torch.zeros(n, dtype=torch.float64, device="cuda")
        info = P.pcg_solve_mg(ctx, b, x, 1e-6, 100)
        outs.append((info["iters"], host64(x).tobytes()))
        ctx.close()
    assert outs[0] == outs[1] == outs[2]


def test_mg_rebuild_follows_coefficients(P, orc):
    """pcg_set_coefficients after pcg_set_multigrid rebuilds the hierarchy:
    the V-cycle equals the oracle's for the new operator, then for constant
    coefficients again."""
    shape = (16, 16, 16)
    n = 4096
    ctx = P.pcg_create(16, 16, 16, torch.float32, x_dtype=torch.float64)
    P.pcg_set_multigrid(ctx, coarse_max=64)
    k = np.exp(synthetic.uniform(94, n)).astype(np.float32)
    kd = dev(k)
    P.pcg_set_coefficients(ctx, kd)
    g32 = synthetic.uniform_f32(95, n)
    g, u = dev(g32), torch.empty(n, device="cuda")
    for kc in (k.astype(np.float64), None):
        P.pcg_mg_apply(ctx, g, u)
        torch.cuda.synchronize()
        ref = orc.VCycle(shape, kc, coarse_max=64)(g32.astype(np.float64))
        assert np.max(np.abs(host64(u) - ref)) <= 2e-5 * np.max(np.abs(ref))
        P.pcg_set_coefficients(ctx, None)
    ctx.close()


def test_mg_errors(P):
    ctx = P.pcg_create(16, 16, 16, torch.float32, x_dtype=torch.float64)
    b = torch.ones(4096, device="cuda")
    x = torch.zeros(4096, dtype=torch.float64, device="cuda")
    with pytest.raises(P.PcgError) as e:
        P.pcg_solve_mg(ctx, b, x)
    assert e.value.status == P.PCG_E_ARG
    with pytest.raises(P.PcgError):
        P.pcg_set_multigrid(ctx, nu=0)
    ctx.close()
    # 33^3 cannot be coarsened: the coarsest grid would hold 35937 points
    ctx = P.pcg_create(33, 33, 33, torch.float32, x_dtype=torch.float64)
    with pytest.raises(P.PcgError) as e:
        P.pcg_set_multigrid(ctx)
    assert e.value.status == P.PCG_E_UNSUPPORTED
    ctx.close()
    ctx = P.pcg_create(16, 16, 16, torch.bfloat16)
    with pytest.raises(P.PcgError) as e:
        P.pcg_set_multigrid(ctx)
    assert e.value.status == P.PCG_E_UNSUPPORTED
    ctx.close()


def test_mg_vcycle_128_against_oracle(P, orc):
    shape = (128, 128, 128)
    n = 128 ** 3
    print("vcycle 128^3", flush=True)
    ctx, _ = _ctx(P, shape)
    g32 = synthetic.uniform_f32(96, n)
    g = dev(g32)
    u = torch.empty_like(g)
    P.pcg_mg_apply(ctx, g, u)
    torch.cuda.synchronize()
    ref = orc.VCycle(shape)(g32.astype(np.float64))
    assert np.max(np.abs(host64(u) - ref)) <= 2e-5 * np.max(np.abs(ref))
    ctx.close()


def test_mg_pcg_256_benchmark_system(P, orc):
    """The benchmark's 256^3 system b = A x* (x* = lowest sine mode + 1e-3
    noise): MG-PCG reaches an FP64 true residual <= 1e-6 in a grid-independent
    number of iterations (the oracle's count at 32^3-64^3 is 10-11)."""
    nn = 256
    shape = (nn, nn, nn)
    print("mg pcg 256^3", flush=True)
    b64 = orc.stencil(synthetic.smooth_plus_noise(nn), shape)
    b32 = b64.astype(np.float32)
    ctx, _ = _ctx(P, shape)
    assert P.pcg_mg_levels(ctx) == [(256 >> l,) * 3 for l in range(6)]
    x = torch.zeros(nn ** 3, dtype=torch.float64, device="cuda")
    info = P.pcg_solve_mg(ctx, dev(b32), x, 1e-6, 100)
    tr = orc.true_relres(shape, b32.astype(np.float64), host64(x))
    print("iters", info["iters"], "true", tr, "s", info["seconds"], flush=True)
    assert info["status"] == P.PCG_OK and tr <= 1e-6
    assert info["iters"] <= 20
    ctx.close()
