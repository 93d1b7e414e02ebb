// context.hpp -- the solver context and the host-side steps shared by the
// single-solve C ABI (api.hip) and the batching server (server.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "kernels.hpp"
#include "pot3d.h"

using pot3d::BatchFin;
using pot3d::BatchSlot;
using pot3d::DevScalars;
using pot3d::GridArgs;
using pot3d::RowCoef;
using pot3d::StencilVecs;
using pot3d::kTileMarch16;
using pot3d::kTileMarch8;
using pot3d::kTileWave2;
using pot3d::kTileWave4;

struct pot3d_ctx {
    int device = 0;
    int nr = 0, nt = 0, np = 0, pitch = 0;
    long long n = 0, npad = 0;
    int precision = POT3D_FP64;
    int tile_p = kTileMarch16, tile_r = kTileWave4, tile_o = kTileWave2;   // set by choose_launch
    int max_blocks = 0;
    int num_cu = 256;
    int graph_m = 16;
    GridArgs grid_p{}, grid_r{}, grid_o{};   // update-p, update-r, other passes

    int upper_bc = POT3D_UPPER_SOURCE_SURFACE;
    std::vector<double> rf, tf, pf;
    std::vector<RowCoef> rows_h;
    std::vector<double> dphi_h, ih_h, bfac_h;
    std::vector<double> vr_h, vt_h;   // cell volume factors r_i^2 dr_i and sin(theta_j) dtheta_j
    double inv_volume = 0.0;          // 1 / shell volume as the sum of the cell volumes

    // device memory
    RowCoef *rows = nullptr;
    double *dphi = nullptr, *ih = nullptr, *bfac = nullptr;
    double *x = nullptr, *r = nullptr, *p[2] = {nullptr, nullptr};
    double *bplane = nullptr, *br = nullptr, *partial = nullptr, *poles = nullptr;
    double *vr = nullptr, *vt = nullptr;   // closed wall: cell volume factors
    double *ftab = nullptr;   // field output: fr (nr+1), ft (nt+1), 1/r_i (nr), 1/sin(theta_j) (nt)
    std::vector<double> ftab_h;
    double *bcs = nullptr;   // closed wall: [0] monopole of Br, [1] keep flag, [2] gauge mean
    DevScalars *sc = nullptr;
    DevScalars *h_sc = nullptr;     // pinned: two status slots for polling
    hipStream_t stream = nullptr;
    hipEvent_t ev_poll[2] = {nullptr, nullptr};
    hipEvent_t ev_t0 = nullptr, ev_t1 = nullptr, ev_loop0 = nullptr, ev_loop1 = nullptr;
    hipGraphExec_t graph = nullptr;

    // FP32-refined mode
    float *r32 = nullptr, *p32[2] = {nullptr, nullptr}, *e32 = nullptr;
    DevScalars *sc32 = nullptr;
    hipGraphExec_t graph32 = nullptr;
    double inner_tol = 0.0;   // 0: the mode's default
    int max_outer = 50;
    int refine_mode = POT3D_REFINE_RELIABLE;

    // Single solves (FP64 iterations, or the FP32 inner iterations of the
    // refined mode): one sweep (default) or two passes per iteration
    int iteration = POT3D_ITER_ONE_SWEEP;
    int sweep_rows = 4;           // one-sweep kernel: box rows per wavefront
    GridArgs grid_s{};
    double *r2 = nullptr;         // one-sweep iteration: the second residual buffer (FP64)
    float *r32b = nullptr;        // ... (FP32 inner iterations)
    hipGraphExec_t graph_s = nullptr;     // FP64 sweeps
    hipGraphExec_t graph32s = nullptr;    // FP32 inner sweeps

    // Preconditioner of single solves (the FP64 iterations, or the FP32 inner
    // ones of the refined mode): point Jacobi (PC1) or the phi-line blocks,
    // which iterate in two passes plus a line pass that writes z.
    int precond = POT3D_PC_JACOBI;
    double *z = nullptr;          // phi-line: z = M^-1 r
    float *z32 = nullptr;         // ... of the FP32 inner iterations (refined mode)
    int line_blocks = 0;          // workgroups of a line pass
    hipGraphExec_t graph_l = nullptr, graph32l = nullptr;

    bool serving = false;         // a batching-server slot: iterates in the server's graph, captures none
    bool have_solution = false;
    bool field_ready = false;     // x and the b plane belong to the last solve
    pot3d_stats stats{};
    std::string err;
};

namespace pot3d {
namespace host {

// Record msg as the context's (or, for ctx = NULL, the thread's) last error.
int fail(pot3d_ctx *ctx, int code, const std::string &msg);
// Integer environment variable, or dflt if unset or not a number.
int env_int(const char *name, int dflt);

#define HIP_TRY(ctx, call)                                                                   \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail((ctx), e_ == hipErrorOutOfMemory ? POT3D_ENOMEM : POT3D_EDEVICE,     \
                        std::string(#call) + ": " + hipGetErrorString(e_));                 \
    } while (0)

// Restores the caller's current device on scope exit.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// Tile shapes of the two iteration passes for a precision (the defaults, or
// the POT3D_TILE[_P|_R] overrides); every context of the process uses them.
void default_tiles(int precision, int *tile_p, int *tile_r);
int validate_grid(const double *rf, int nr, const double *tf, int nt, const double *pf, int np, int upper_bc,
                  int precision, pot3d_ctx **out);
// The operator's separable tables from the faces (see api.hip): rows
// (nr * nt), dphi, ih (np), bfac (nt), vr (nr), vt (nt), 1 / shell volume;
// work holds 2 nr + 2 nt + np doubles.  Allocates nothing.
void fill_tables(int nr, int nt, int np, const double *rf, const double *tf, const double *pf, int upper_bc,
                 RowCoef *rows, double *dphi, double *ih, double *bfac, double *vr, double *vt, double *inv_volume,
                 double *work);
// Launch shapes from the grid fields of c (nr, nt, np, pitch, npad,
// precision, num_cu): a stencil pass of `tile` with about `target`
// workgroups, and the one-sweep kernel with `rows` box rows per wavefront.
GridArgs make_grid(const pot3d_ctx *c, int tile, int target, int ci_fixed);
GridArgs make_sweep_grid(const pot3d_ctx *c, int rows, int target);
// x update mode of sweep `it` of a captured sequence (SweepVecs::xmode), and
// the HBM bytes per unknown per iteration of the one-sweep form that go with it.
int sweep_xmode(int it);
double sweep_bytes(bool fp32);
// The r/x update mode of iteration `it` of a captured sequence of m two-pass
// (or phi-line) iterations, and the bytes per unknown of a two-pass iteration
// that go with it (the phi-line iteration adds 16 N, 8 N in FP32).
int update_r_mode(int it, int m);
double two_pass_bytes(bool fp32, int m);
// Allocate a context on `device` (tables, vectors, graphs).  serving = true:
// no graph capture (the server's batched graph iterates it).
int create_context(const double *rf, int nr, const double *tf, int nt, const double *pf, int np, int upper_bc,
                   int precision, int device, bool serving, pot3d_ctx **out);
void free_ctx(pot3d_ctx *c);
// Device bytes held by a context.
size_t context_bytes(const pot3d_ctx *c);
StencilVecs<double> base_vecs(pot3d_ctx *c);
// b from Br (device) and the starting x (phi0 or zero).
int prepare_solve(pot3d_ctx *c, const double *br_dev, const double *phi0, hipMemcpyKind kind_in, hipStream_t s);
// FP64: r = b - A x, p_old = 0, scalars initialised, first residual test.
int start_fp64(pot3d_ctx *c, hipStream_t s, double tol, int maxit);
// Refined: r = b - A x in FP64 and the outer test; waits, then *out holds the scalars.
int refined_outer_check(pot3d_ctx *c, hipStream_t s, DevScalars *out);
// Refined: normalised FP32 residual, e = 0, and the inner PCG start (a
// restart, or in reliable-update mode the continuation of the previous
// segment `prev`, which ran in normalisation scale_prev).  outer: the scalars
// of the outer check just made.
int refined_start_inner(pot3d_ctx *c, hipStream_t s, double tol, int maxit_left, const DevScalars &outer,
                        const DevScalars *prev, double scale_prev);
// Refined: x += ||r|| e.
int refined_correct(pot3d_ctx *c, hipStream_t s);
// True residual, pole values, Phi out, statistics; returns the solve status.
int finish_solve(pot3d_ctx *c, double *phi_out, hipMemcpyKind kind_out, hipStream_t s, DevScalars fin, int launches,
                 int total_iters, int outer, double bytes_per_unknown, int *iters, double *relres_true);

}  // namespace host
}  // namespace pot3d
