// noalloc.hip -- an FP64 solve that allocates nothing: pot3d_solve_noalloc.
//
// For callers that cannot allocate device memory (code under stream capture,
// tight serving loops, harnesses that forbid it).  It runs the same kernels
// as a context's one-sweep FP64 point-Jacobi solve (pot3d_solve_device), but
// every buffer beyond the caller's inputs and outputs -- the metric tables,
// the right-hand-side layer, the PCG vectors x, r (two), p (two), the
// per-workgroup partial sums and the scalar block -- lives in one file-scope
// device array, `scratch`, of kScratchBytes.  The tables are built on the host
// into static staging arrays and copied in.  Nothing here calls hipMalloc,
// hipFree, hipHostMalloc or graph instantiation: the iterations are launched
// one by one and polled every kPollSweeps sweeps with a copy of the scalar
// block into static host memory.
//
// Each GPU holds its own copy of `scratch`, at its own address, until the
// process ends.  In host code the array's name only stands in for it, so the
// device address is taken once per device with hipGetSymbolAddress (on the
// first call on that device) and only that address is handed to kernels and
// copies.  A process-wide lock serializes the calls, so concurrent callers of
// this entry point do not race on the array; it keeps the last call's
// contents, and everything that must start at zero is cleared by each call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>

#include "context.hpp"

namespace pot3d {
namespace host {

constexpr size_t kScratchBytes = 96ull << 20;   // 96 MiB per GPU

// The scratch buffer of every pot3d_solve_noalloc call on a GPU.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxRows = 65536;                 // nr * nt
constexpr int kMaxAxis = 4096;                  // nr, nt, np each
constexpr int kMaxDevices = 64;
constexpr int kPollSweeps = 32;

struct DeviceState {
    bool ready = false;
    char *base = nullptr;   // device address of this GPU's `scratch`
    int num_cu = 0;
    int sweep_per_cu = 0;
};

std::mutex g_lock;
DeviceState g_dev[kMaxDevices];

// host staging (under g_lock)
RowCoef h_rows[kMaxRows];
double h_dphi[kMaxAxis], h_ih[kMaxAxis], h_bfac[kMaxAxis], h_vr[kMaxAxis], h_vt[kMaxAxis];
double h_work[5 * kMaxAxis];
DevScalars h_sc;

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Set-up on the current device, once: the device address of `scratch`.
int setup_device(int dev)
{
    DeviceState &d = g_dev[dev];
    if (d.ready) return POT3D_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(nullptr, POT3D_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    hipDeviceProp_t prop{};
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return fail(nullptr, POT3D_EDEVICE, "hipGetDeviceProperties failed");
    d.base = static_cast<char *>(ptr);
    d.num_cu = std::max(1, prop.multiProcessorCount);
    d.sweep_per_cu = std::max(1, sweep_blocks_per_cu<double>(4));
    d.ready = true;
    return POT3D_OK;
}

#define NA_TRY(call)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return fail(nullptr, POT3D_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

}  // namespace
}  // namespace host
}  // namespace pot3d

using namespace pot3d;
using namespace pot3d::host;

extern "C" int pot3d_solve_noalloc(const double *r_faces, int nr, const double *t_faces, int nt,
                                   const double *p_faces, int np, int upper_bc, const double *d_br,
                                   const double *d_phi0, double *d_phi, void *stream, double tol, int maxit,
                                   int *iters, double *relres_true)
{
    pot3d_ctx *dummy = nullptr;
    int v = validate_grid(r_faces, nr, t_faces, nt, p_faces, np, upper_bc, POT3D_FP64, &dummy);
    if (v != POT3D_OK) return v;
    if (!d_br || !d_phi) return fail(nullptr, POT3D_EINVAL, "br and phi are required");
    if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(nullptr, POT3D_EINVAL, "tol must be finite and >= 0");
    if (maxit < 0) return fail(nullptr, POT3D_EINVAL, "maxit must be >= 0");
    if (nr > kMaxAxis || nt > kMaxAxis || np > kMaxAxis || (long long)nr * nt > kMaxRows)
        return fail(nullptr, POT3D_EINVAL, "grid exceeds the no-allocation limits (nr, nt, np <= 4096, nr*nt <= 65536)");

    // layout of the scratch array for this grid (every piece 256-byte aligned)
    pot3d_ctx shape;   // launch-shape fields only; owns nothing
    shape.nr = nr;
    shape.nt = nt;
    shape.np = np;
    shape.pitch = ((np + 7) / 8) * 8;
    shape.n = (long long)nr * nt * np;
    shape.npad = (long long)nr * nt * shape.pitch;
    shape.precision = POT3D_FP64;
    shape.upper_bc = upper_bc;

    std::lock_guard<std::mutex> guard_lock(g_lock);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return fail(nullptr, POT3D_EDEVICE, "no current HIP device");
    int rc = setup_device(dev);
    if (rc != POT3D_OK) return rc;
    DeviceState &ds = g_dev[dev];
    shape.num_cu = ds.num_cu;

    GridArgs go = make_grid(&shape, kTileWave2, 2048, 0);
    GridArgs gs = make_sweep_grid(&shape, 4, ds.sweep_per_cu * ds.num_cu);
    const int maxblk = std::max(1, std::max(go.nblocks, gs.nblocks));
    const size_t vec = (size_t)shape.npad * sizeof(double);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align256(bytes);
        return o;
    };
    const size_t o_sc = take(sizeof(DevScalars));
    const size_t o_part = take((size_t)kMaxPartials * maxblk * sizeof(double));
    const size_t o_bcs = take(4 * sizeof(double));
    const size_t o_rows = take((size_t)nr * nt * sizeof(RowCoef));
    const size_t o_dphi = take((size_t)np * sizeof(double));
    const size_t o_ih = take((size_t)np * sizeof(double));
    const size_t o_bfac = take((size_t)nt * sizeof(double));
    const size_t o_vr = take((size_t)nr * sizeof(double));
    const size_t o_vt = take((size_t)nt * sizeof(double));
    const size_t o_bpl = take((size_t)nt * shape.pitch * sizeof(double));
    size_t o_vec[5];
    for (size_t &o : o_vec) o = take(vec);
    if (off > kScratchBytes)
        return fail(nullptr, POT3D_EINVAL,
                    "grid exceeds the no-allocation limit: " + std::to_string(off) + " bytes of scratch needed, " +
                        std::to_string(kScratchBytes) + " available");

    char *base = ds.base;
    DevScalars *sc = reinterpret_cast<DevScalars *>(base + o_sc);
    double *partial = reinterpret_cast<double *>(base + o_part);
    double *bcs = reinterpret_cast<double *>(base + o_bcs);
    RowCoef *rows = reinterpret_cast<RowCoef *>(base + o_rows);
    double *dphi = reinterpret_cast<double *>(base + o_dphi);
    double *ih = reinterpret_cast<double *>(base + o_ih);
    double *bfac = reinterpret_cast<double *>(base + o_bfac);
    double *vr = reinterpret_cast<double *>(base + o_vr);
    double *vt = reinterpret_cast<double *>(base + o_vt);
    double *bplane = reinterpret_cast<double *>(base + o_bpl);
    double *x = reinterpret_cast<double *>(base + o_vec[0]);
    double *rb[2] = {reinterpret_cast<double *>(base + o_vec[1]), reinterpret_cast<double *>(base + o_vec[2])};
    double *pb[2] = {reinterpret_cast<double *>(base + o_vec[3]), reinterpret_cast<double *>(base + o_vec[4])};
    for (GridArgs *g : {&go, &gs}) {
        g->rows = rows;
        g->dphi = dphi;
        g->ih = ih;
    }

    // tables on the host (static staging), then into the scratch array
    double inv_volume = 0.0;
    fill_tables(nr, nt, np, r_faces, t_faces, p_faces, upper_bc, h_rows, h_dphi, h_ih, h_bfac, h_vr, h_vt,
                &inv_volume, h_work);
    hipStream_t s = stream ? reinterpret_cast<hipStream_t>(stream) : nullptr;
    NA_TRY(hipMemcpyAsync(rows, h_rows, (size_t)nr * nt * sizeof(RowCoef), hipMemcpyHostToDevice, s));
    NA_TRY(hipMemcpyAsync(dphi, h_dphi, (size_t)np * sizeof(double), hipMemcpyHostToDevice, s));
    NA_TRY(hipMemcpyAsync(ih, h_ih, (size_t)np * sizeof(double), hipMemcpyHostToDevice, s));
    NA_TRY(hipMemcpyAsync(bfac, h_bfac, (size_t)nt * sizeof(double), hipMemcpyHostToDevice, s));
    NA_TRY(hipMemcpyAsync(vr, h_vr, (size_t)nr * sizeof(double), hipMemcpyHostToDevice, s));
    NA_TRY(hipMemcpyAsync(vt, h_vt, (size_t)nt * sizeof(double), hipMemcpyHostToDevice, s));
    h_sc = DevScalars{};
    h_sc.tol = tol;
    h_sc.maxit = maxit;
    NA_TRY(hipMemcpyAsync(sc, &h_sc, sizeof(DevScalars), hipMemcpyHostToDevice, s));

    // everything that must start at zero (padding included), then b and x
    for (double *buf : {x, rb[0], rb[1], pb[0], pb[1]}) NA_TRY(launch_fill<double>(buf, shape.npad, 0.0, s));
    NA_TRY(launch_fill<double>(bplane, (long long)nt * shape.pitch, 0.0, s));
    NA_TRY(launch_fill<double>(bcs, 4, 0.0, s));
    const bool closed = upper_bc == POT3D_UPPER_CLOSED_WALL;
    if (closed) NA_TRY(launch_monopole(d_br, bfac, dphi, nt, np, bcs, s));
    NA_TRY(launch_rhs(d_br, bfac, dphi, nt, np, shape.pitch, closed ? bcs : nullptr, bplane, s));
    const size_t rowb = (size_t)np * sizeof(double), pitchb = (size_t)shape.pitch * sizeof(double);
    if (d_phi0) NA_TRY(hipMemcpy2DAsync(x, pitchb, d_phi0, rowb, rowb, (size_t)nr * nt, hipMemcpyDeviceToDevice, s));

    // r = b - A x, the first test; then sweeps (the one-sweep PCG iteration)
    StencilVecs<double> rv{};
    rv.sc = sc;
    rv.partial = partial;
    rv.in = x;
    rv.r = rb[0];
    rv.bplane = bplane;
    rv.store_r = 1;
    rv.ignore_done = 1;
    NA_TRY(launch_stencil<double>(kResidual, kTileWave2, go, rv, s));
    NA_TRY(launch_finish(kFinInit, sc, partial, go.nblocks, s));
    const long long max_sweeps = (long long)maxit + 2 * kPollSweeps;
    long long j = 0;
    for (;;) {
        for (int q = 0; q < kPollSweeps; ++q, ++j) {
            SweepVecs<double> sv{};
            sv.r_in = rb[j & 1];
            sv.r_out = rb[(j + 1) & 1];
            sv.p_old = pb[j & 1];
            sv.p_new = pb[(j + 1) & 1];
            sv.x = x;
            sv.sc = sc;
            sv.partial = partial;
            sv.xmode = sweep_xmode((int)(j & 1));   // x once per pair of sweeps; j starts even
            NA_TRY(launch_sweep<double>(4, gs, sv, s));
            NA_TRY(launch_finish(kFinSweep, sc, partial, gs.nblocks, s));
        }
        NA_TRY(hipMemcpyAsync(&h_sc, sc, sizeof(DevScalars), hipMemcpyDeviceToHost, s));
        NA_TRY(hipStreamSynchronize(s));
        if (h_sc.done || j > max_sweeps) break;
    }
    if (!h_sc.done) return fail(nullptr, POT3D_EDEVICE, "iteration loop ended without the device done flag");
    const DevScalars fin = h_sc;
    // the x increment the last sweep may have left to a next one
    NA_TRY(launch_x_catchup<double>(x, sc, nr, nt, np, shape.pitch, s));

    // the answer: gauge (closed wall), true residual, Phi into the caller's array
    if (fin.zero_solution) NA_TRY(launch_fill<double>(x, shape.npad, 0.0, s));
    else if (closed)
        NA_TRY(launch_gauge(x, vr, vt, dphi, nr, nt, np, shape.pitch, inv_volume, partial, maxblk, bcs + 2, s));
    StencilVecs<double> tv = rv;
    tv.store_r = 0;
    NA_TRY(launch_stencil<double>(kResidual, kTileWave2, go, tv, s));
    NA_TRY(launch_finish(kFinTrue, sc, partial, go.nblocks, s));
    NA_TRY(hipMemcpy2DAsync(d_phi, rowb, x, pitchb, rowb, (size_t)nr * nt, hipMemcpyDeviceToDevice, s));
    NA_TRY(hipMemcpyAsync(&h_sc, sc, sizeof(DevScalars), hipMemcpyDeviceToHost, s));
    NA_TRY(hipStreamSynchronize(s));
    if (iters) *iters = fin.k;
    if (relres_true) *relres_true = fin.zero_solution ? 0.0 : h_sc.relres_true;
    if (fin.status == POT3D_EBREAKDOWN) return fail(nullptr, POT3D_EBREAKDOWN, "breakdown: non-finite data or p.Ap <= 0");
    if (fin.status == POT3D_ENOCONV) return fail(nullptr, POT3D_ENOCONV, "iteration cap reached before tol");
    return fin.status;
}
