// internal.hpp -- host-side interface between the C ABI layer and the
// kernel launchers (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pcgmi.h"

namespace pcgmi {

struct SolveState;

enum DT : int { DT_F32 = PCG_F32, DT_BF16 = PCG_BF16, DT_F16 = PCG_F16, DT_F64 = PCG_F64 };

inline size_t dt_size(int dt) { return dt == DT_F64 ? 8 : dt == DT_F32 ? 4 : 2; }
inline int dt_width(int dt) { return (int)(16 / dt_size(dt)); }  // elements per 16 bytes
// MI355X's last-level cache (AMD Infinity Cache) in front of HBM.
constexpr size_t LLC_BYTES = (size_t)256 << 20;

// Compiled work-group shapes of the z-march kernels: BX x BY threads, each
// thread owning VX consecutive x points (VX = 16 bytes of the storage type,
// or 1 for the scalar shape used when nx is not a multiple of that width).
struct TileCfg {
    int bx, by;
    bool vec;  // one 16-byte vector per thread and plane (else one element)
};
constexpr int NUM_TILE_CFG = 6;
constexpr TileCfg TILE_CFGS[NUM_TILE_CFG] = {
    {16, 16, true}, {32, 8, true}, {64, 4, true}, {16, 4, true}, {16, 8, true}, {64, 4, false}};

struct Plan {
    int cfg;  // index into TILE_CFGS
    int zc;   // planes per work-group
};

// Tile extents of a plan for storage type dt.
inline int plan_tx(const Plan& p, int dt) { return TILE_CFGS[p.cfg].bx * (TILE_CFGS[p.cfg].vec ? dt_width(dt) : 1); }
inline int plan_ty(const Plan& p) { return TILE_CFGS[p.cfg].by; }

struct Geometry {
    int nx, ny, nz;
    int ntx, nty, nzc, zc;
    unsigned nblocks;
    int pitch;  // row stride in elements (nx, or nx padded to the vector width)
};
Geometry make_geometry(int nx, int ny, int nz, const Plan& p, int dt);

// Grid-reduction workspace: `cap` doubles of per-work-group partials and the
// ticket counter. Every reducing launch checks NC * work-groups <= cap on the
// host and fails with hipErrorInvalidValue otherwise.
struct Red {
    double* partials;
    unsigned* ticket;
    size_t cap;
};
constexpr int MAX_RED_COMPONENTS = 6;  // two chained halves of up to 3 components

// The operator of a context: constant coefficients (kc == null) or the
// variable-coefficient operator with cell coefficients kc (FP32) and the
// inverse Jacobi diagonal dinv (storage type).
struct OpDesc {
    const float* kc;
    const void* dinv;
};

// ---- z-march kernels (stencil family) ----
hipError_t launch_stencil(int dt, const Plan& p, const Geometry& g, OpDesc od, const void* x, void* y, hipStream_t s);
// dinv = 1 / diag(A_k) for cell coefficients kc.
hipError_t launch_var_dinv(int dt, const Plan& p, const Geometry& g, const float* kc, void* dinv, hipStream_t s);

// Links of a chain of PCG iteration kernels: each kernel finishes the
// previous kernel's reduction (pin, nin partials per component) on a copy of
// the solve state read from sin, stores the new state in sout (work-group 0)
// and leaves its own partials in pout. pin == null: sin is current.
struct Chain {
    const double* pin;
    unsigned nin;
    const SolveState* sin;
    SolveState* sout;
    double* hist;  // relative residual per iteration (maxit + 1 entries) or null
    double* pout;
};

// Iteration kernel 1: finishes the previous update's r.r (and r.z) into beta,
// the iteration count and the convergence test; then p_new = D^-1 r + beta
// p_old (rounded to storage) and partials of p.Ap.
hipError_t launch_pcg_direction(int dt, const Plan& p, const Geometry& g, OpDesc od, const void* r,
                                const void* pold, void* pnew, const Chain& ch, hipStream_t s);
// Iteration kernel 2: finishes p.Ap into alpha; then q = A p, r -= alpha q
// and partials of r.r (and r.z). x (the accumulator) is of type xdt: FP64,
// FP32 or the storage type. xmode 1: x is left as it is; xmode 2: x +=
// alpha_prev pprev + alpha p (pprev: the previous iteration's direction).
hipError_t launch_pcg_update(int dt, const Plan& p, const Geometry& g, OpDesc od, const void* pdir, void* x,
                             int xdt, void* r, int xmode, const void* pprev, const Chain& ch, hipStream_t s);
// x += alpha p (alpha from *st) over n points; with check_done, nothing when
// the state records a finished solve.
hipError_t launch_x_finish(int dt, int xdt, int64_t n, void* x, const void* p, const SolveState* st,
                           bool check_done, hipStream_t s);
// Finishes the last update's partials of a chain (beta, count, convergence).
hipError_t launch_pcg_close(bool var, const Chain& ch, hipStream_t s);

// Single-reduction form (constant coefficients). Vectors of one iteration.
struct SRBufs {
    const void* r_in;
    const void* w_in;
    const void* s_in;
    void* r_out;
    void* w_out;
    void* s_out;
    void* p;  // in place
};
// Start: w = stored(A D^-1 r), {gamma, delta} -> alpha (grid reduction into st).
hipError_t launch_pcg_sr_start(int dt, const Plan& p, const Geometry& g, const void* r, void* w, SolveState* st,
                               Red red, hipStream_t s);
// One iteration: finishes the previous iteration's {gamma, delta, r.r}, then
// the fused update and stencil; x (type xdt) in place.
hipError_t launch_pcg_sr(int dt, const Plan& p, const Geometry& g, const SRBufs& b, void* x, int xdt, const Chain& ch,
                         hipStream_t s);
hipError_t launch_pcg_sr_close(const Chain& ch, hipStream_t s);
// r = stored(b - A x0) computed in FP64 (x0 of type xdt), totals {r.r, b.b}
// -> solve start. Uses the FP64 residual shape (pres, gres).
hipError_t launch_pcg_start_x0(int dt, int xdt, const Plan& pres, const Geometry& gres, OpDesc od, const void* b,
                               const void* x0, void* r, SolveState* st, double* hist, Red red, hipStream_t s);
// FP64 residual of b (type bdt) and x (type xdt): out = {||r||^2, max|r|}.
hipError_t launch_residual64(int bdt, int xdt, const Plan& p, const Geometry& g, OpDesc od, const void* b,
                             const void* x, double* out, Red red, hipStream_t s);

// Refinement: rhat (storage type dt) = stored(scale (b - A x)), FP64 b and x.
hipError_t launch_cast_scaled(int dt, const Plan& pres, const Geometry& gres, OpDesc od, const double* b,
                              const double* x, double scale, void* rhat, hipStream_t s);
// Refinement: x += d / scale, d of type ddt.
hipError_t launch_correct(int ddt, int64_t n, const void* d, double scale, double* x, hipStream_t s);

// ---- streaming kernels ----
hipError_t launch_axpy(int dt, int64_t n, double alpha, const void* x, const void* y, void* z, hipStream_t s);
// out_f32 and/or out_f64 (device) receive the dot; either may be null.
hipError_t launch_dot(int dt, int64_t n, const void* x, const void* y, float* out_f32, double* out_f64, Red red,
                      hipStream_t s);
// r = b, x = 0, p0 = 0; totals {b.b, b.b, sum dinv b^2} -> solve start (dinv
// from the array when given, else the solve state's constant).
hipError_t launch_pcg_start_zero(int dt, int64_t n, const void* b, void* r, void* x, int xdt, void* p0,
                                 const void* dinv, SolveState* st, double* hist, Red red, hipStream_t s);
// Fill n elements of type dt (or FP64 when dt == DT_F64) with zero.
hipError_t launch_zero(int dt, int64_t n, void* p, hipStream_t s);
// Convert n elements: dst (type ddt) = src (type sdt), rounding to nearest even.
hipError_t launch_convert(int sdt, int ddt, int64_t n, const void* src, void* dst, hipStream_t s);

// flexible CG (FP32 storage)
hipError_t launch_flex_direction(const Plan& p, const Geometry& g, OpDesc od, const float* z, const float* pold,
                                 float* pnew, float* q, const float* r, SolveState* st, Red red, hipStream_t s);
hipError_t launch_flex_update(int64_t n, const float* p, const float* pold, const float* q, float* r, double* x,
                              SolveState* st, double* hist, Red red, hipStream_t s);
hipError_t launch_flex_select(int64_t n, float* z, const float* r, const float* q, const float* dinv, SolveState* st,
                              bool redo_pass, Red red, hipStream_t s);
// geometric multigrid V-cycle (FP32): levels finest first; level l solves the
// unscaled seven-point system A[k_l] u = g_l, and g_(l+1) = P^T r_l / 2.
constexpr int MG_MAX_LEVELS = 16;
struct MgLevel {
    int nx, ny, nz;
    int64_t n;
    Plan plan;
    Geometry geo;
    const float* k;     // cell coefficients (null: constant coefficients)
    const float* dinv;  // 1 / diag(A[k]) (null: the constant 1/6)
    float* g;           // right-hand side (levels >= 1; level 0 gets the caller's)
    float* u[2];        // iterates (sweeps ping-pong)
    float* r;           // residual (all levels but the coarsest)
    float* out;         // result of the level's V-cycle (levels >= 1)
};
struct MgHierarchy {
    int nlev = 0;
    int nu = 1;              // damped-Jacobi sweeps before and after the correction
    float omega = 6.f / 7.f;
    MgLevel lv[MG_MAX_LEVELS] = {};
    float* ainv = nullptr;   // inverse of the coarsest operator (m x m, symmetric)
};
// The flexible iteration's select step fused into the V-cycle's last sweep:
// q = A p, the solve state and the reduction workspace.
struct MgSelect {
    const float* q;
    SolveState* st;
    Red red;
};
// out = V-cycle(g) on level 0 (out must not alias g or the level's buffers);
// every kernel returns at once while *done != 0. With sel (two or more
// levels) the last sweep also forms z.q and z.r and applies the flexible
// iteration's beta step (FinFlexBeta).
hipError_t launch_mg_vcycle(const MgHierarchy& H, const float* g, float* out, const int* done, hipStream_t s,
                           const MgSelect* sel = nullptr);
// kc = mean of the 2 x 2 x 2 children of kf (nx, ny, nz even).
hipError_t launch_mg_coarsen_k(const float* kf, int nx, int ny, int nz, float* kc, hipStream_t s);
// training pairs from solver snapshots
hipError_t launch_make_pair(int64_t n, const double* r, const double* x, const double* xs, const double* rr,
                            void* out, hipStream_t s);
hipStream_t cnn_stream_of(cnn_net n);
hipStream_t cnn_swap_stream(cnn_net n, hipStream_t s);
pcg_status cnn_prepare(cnn_net n, int nx, int ny, int nz, uint64_t* epoch);

constexpr int DOT_MAX_BLOCKS = 2048;
constexpr int STREAM_THREADS = 256;

}  // namespace pcgmi
