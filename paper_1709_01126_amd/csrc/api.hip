// api.hip -- host driver and C ABI of the potential-field PCG solver.
//
// A context owns, on one device:
//   * the separable metric tables of the Sec. 2.2 operator (per (i, j) row
//     and per k);
//   * the PCG vectors x, r, p (two buffers, alternating) in a padded
//     phi-fastest layout;
//   * the right-hand-side layer, the per-workgroup partial sums and the
//     scalar state;
//   * a HIP graph of m PCG iterations.
// A solve copies Br in, builds b and the initial residual, replays the graph
// until the device sets its done flag, then recomputes the true residual and
// the pole values (eq. (3)) and copies Phi out.  There is one host<->device
// copy of each array per solve; the paper keeps its data resident the same
// way (Sec. 3.1).  Inside the loop the host only polls a 64-byte status block
// once per graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "pot3d.h"

using namespace pot3d;

namespace {

thread_local std::string g_thread_error;

constexpr double kTwoPi = 6.283185307179586476925286766559;

int env_int(const char *name, int dflt)
{
    const char *s = std::getenv(name);
    if (!s || !*s) return dflt;
    return std::atoi(s);
}

}  // namespace

struct pot3d_ctx {
    int device = 0;
    int nr = 0, nt = 0, np = 0, pitch = 0;
    long long n = 0, npad = 0;
    int precision = POT3D_FP64;
    int tj = 16, ci = 1;
    int graph_m = 16;
    GridArgs grid{};

    std::vector<double> rf, tf, pf;
    std::vector<RowCoef> rows_h;
    std::vector<double> dphi_h, ih_h, bfac_h;

    // device memory
    RowCoef *rows = nullptr;
    double *dphi = nullptr, *ih = nullptr, *bfac = nullptr;
    double *x = nullptr, *r = nullptr, *p[2] = {nullptr, nullptr};
    double *bplane = nullptr, *br = nullptr, *partial = nullptr, *poles = nullptr;
    DevScalars *sc = nullptr;
    DevScalars *h_sc = nullptr;     // pinned: two status slots for polling
    hipStream_t stream = nullptr;
    hipEvent_t ev_poll[2] = {nullptr, nullptr};
    hipEvent_t ev_t0 = nullptr, ev_t1 = nullptr, ev_loop0 = nullptr, ev_loop1 = nullptr;
    hipGraphExec_t graph = nullptr;

    bool have_solution = false;
    pot3d_stats stats{};
    std::string err;
};

namespace {

int fail(pot3d_ctx *ctx, int code, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    else g_thread_error = msg;
    return code;
}

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

bool finite_increasing(const double *a, int n1)
{
    for (int q = 0; q < n1; ++q)
        if (!std::isfinite(a[q])) return false;
    for (int q = 0; q + 1 < n1; ++q)
        if (!(a[q + 1] > a[q])) return false;
    return true;
}

int validate_grid(const double *rf, int nr, const double *tf, int nt, const double *pf, int np, int upper_bc,
                  int precision, pot3d_ctx **out)
{
    if (!out) return fail(nullptr, POT3D_EINVAL, "out is NULL");
    if (!rf || !tf || !pf) return fail(nullptr, POT3D_EINVAL, "face array is NULL");
    if (nr < 2 || nt < 2 || np < 3) return fail(nullptr, POT3D_EINVAL, "need nr >= 2, nt >= 2, np >= 3");
    if ((long long)nr * nt > (1LL << 30) || (long long)nr * nt * np > (1LL << 40))
        return fail(nullptr, POT3D_EINVAL, "grid too large");
    if (!finite_increasing(rf, nr + 1) || !(rf[0] > 0.0))
        return fail(nullptr, POT3D_EINVAL, "r faces must be finite, positive and strictly increasing");
    if (!finite_increasing(tf, nt + 1))
        return fail(nullptr, POT3D_EINVAL, "theta faces must be finite and strictly increasing");
    if (std::fabs(tf[0]) > 1e-12 || std::fabs(tf[nt] - M_PI) > 1e-12)
        return fail(nullptr, POT3D_EINVAL, "theta faces must span exactly [0, pi]");
    if (!finite_increasing(pf, np + 1))
        return fail(nullptr, POT3D_EINVAL, "phi faces must be finite and strictly increasing");
    if (std::fabs(pf[np] - pf[0] - kTwoPi) > 1e-12)
        return fail(nullptr, POT3D_EINVAL, "phi faces must span exactly 2 pi");
    if (upper_bc == POT3D_UPPER_CLOSED_WALL)
        return fail(nullptr, POT3D_EINVAL, "closed-wall upper boundary (singular system) is not supported");
    if (upper_bc != POT3D_UPPER_SOURCE_SURFACE) return fail(nullptr, POT3D_EINVAL, "unknown upper_bc");
    if (precision != POT3D_FP64) return fail(nullptr, POT3D_EINVAL, "unsupported precision");
    return POT3D_OK;
}

// Separable metric tables of the volume-scaled operator (Sec. 2.2 scheme with
// the spherical metric restored).  Cell centres are face midpoints; the top
// face Phi = 0 couples through a half-cell difference onto the diagonal.
void build_tables(pot3d_ctx *c)
{
    const int nr = c->nr, nt = c->nt, np = c->np;
    const double *rf = c->rf.data(), *tf = c->tf.data(), *pf = c->pf.data();
    std::vector<double> rc(nr), dr(nr), tc(nt), dt(nt), pc(np);
    for (int i = 0; i < nr; ++i) { rc[i] = 0.5 * (rf[i] + rf[i + 1]); dr[i] = rf[i + 1] - rf[i]; }
    for (int j = 0; j < nt; ++j) { tc[j] = 0.5 * (tf[j] + tf[j + 1]); dt[j] = tf[j + 1] - tf[j]; }
    for (int k = 0; k < np; ++k) pc[k] = 0.5 * (pf[k] + pf[k + 1]);

    c->rows_h.assign((size_t)nr * nt, RowCoef{});
    for (int i = 0; i < nr; ++i) {
        for (int j = 0; j < nt; ++j) {
            const double sj = std::sin(tc[j]);
            const double face = sj * dt[j];   // r-face area / (r^2 dphi)
            RowCoef &e = c->rows_h[(size_t)i * nt + j];
            e.rm = (i > 0) ? face * rf[i] * rf[i] / (rc[i] - rc[i - 1]) : 0.0;
            e.rp = (i < nr - 1) ? face * rf[i + 1] * rf[i + 1] / (rc[i + 1] - rc[i]) : 0.0;
            const double dtop = (i == nr - 1) ? face * rf[nr] * rf[nr] / (rf[nr] - rc[nr - 1]) : 0.0;
            // pole faces (j = 0 below, j = nt-1 above) have sin(theta) = 0: no coupling
            e.tm = (j > 0) ? dr[i] * std::sin(tf[j]) / (tc[j] - tc[j - 1]) : 0.0;
            e.tp = (j < nt - 1) ? dr[i] * std::sin(tf[j + 1]) / (tc[j + 1] - tc[j]) : 0.0;
            e.s = e.rm + e.rp + e.tm + e.tp + dtop;
            e.pq = dr[i] * dt[j] / sj;
        }
    }
    c->dphi_h.resize(np);
    c->ih_h.resize(np);
    for (int k = 0; k < np; ++k) {
        c->dphi_h[k] = pf[k + 1] - pf[k];
        const double gap = (k < np - 1) ? pc[k + 1] - pc[k] : pc[0] + kTwoPi - pc[np - 1];
        c->ih_h[k] = 1.0 / gap;
    }
    c->bfac_h.resize(nt);
    for (int j = 0; j < nt; ++j) c->bfac_h[j] = std::sin(tc[j]) * dt[j] * rf[0] * rf[0];
}

// Workgroup shape: TJ polar rows x 64 azimuthal cells, radial chunks sized so
// that one launch has about `target` workgroups.
void choose_launch(pot3d_ctx *c)
{
    int tj = env_int("POT3D_TJ", 16);
    if (tj != 8 && tj != 16 && tj != 32) tj = 16;
    const int target = std::max(1, env_int("POT3D_TARGET_BLOCKS", 2048));
    const int ntj = (c->nt + tj - 1) / tj;
    const int ntk = (c->np + kWave - 1) / kWave;
    const long long tiles = (long long)ntj * ntk;
    int ci = env_int("POT3D_CI", 0);
    if (ci <= 0) {
        long long want = (target + tiles - 1) / tiles;
        want = std::max<long long>(1, std::min<long long>(want, c->nr));
        ci = (int)((c->nr + want - 1) / want);
    }
    ci = std::max(1, std::min(ci, c->nr));
    const int nchunk = (c->nr + ci - 1) / ci;
    c->tj = tj;
    c->ci = ci;
    GridArgs &g = c->grid;
    g.nr = c->nr;
    g.nt = c->nt;
    g.np = c->np;
    g.pitch = c->pitch;
    g.plane = (long long)c->nt * c->pitch;
    g.ci = ci;
    g.nchunk = nchunk;
    g.ntj = ntj;
    g.ntk = ntk;
    g.nblocks = (int)(tiles * nchunk);
}

StencilVecs<double> base_vecs(pot3d_ctx *c)
{
    StencilVecs<double> v{};
    v.sc = c->sc;
    v.partial = c->partial;
    return v;
}

int capture_graph(pot3d_ctx *c)
{
    if (c->graph) return POT3D_OK;
    hipStream_t s = c->stream;
    HIP_TRY(c, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int it = 0; it < c->graph_m && e == hipSuccess; ++it) {
        StencilVecs<double> a = base_vecs(c);
        a.in = c->r;
        a.pold = c->p[it & 1];
        a.pnew = c->p[(it + 1) & 1];
        e = launch_stencil<double>(kUpdateP, c->tj, c->grid, a, s);
        if (e == hipSuccess) e = launch_finish(kFinSigma, c->sc, c->partial, c->grid.nblocks, s);
        if (e == hipSuccess) {
            StencilVecs<double> bv = base_vecs(c);
            bv.in = c->p[(it + 1) & 1];
            bv.r = c->r;
            bv.x = c->x;
            e = launch_stencil<double>(kUpdateR, c->tj, c->grid, bv, s);
        }
        if (e == hipSuccess) e = launch_finish(kFinRho, c->sc, c->partial, c->grid.nblocks, s);
    }
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(s, &graph);
    if (e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(c, POT3D_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    }
    if (e2 != hipSuccess) return fail(c, POT3D_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e2));
    hipError_t e3 = hipGraphInstantiate(&c->graph, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e3 != hipSuccess) return fail(c, POT3D_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e3));
    return POT3D_OK;
}

void free_ctx(pot3d_ctx *c)
{
    if (!c) return;
    DeviceGuard guard(c->device);
    if (c->graph) (void)hipGraphExecDestroy(c->graph);
    for (hipEvent_t *e : {&c->ev_poll[0], &c->ev_poll[1], &c->ev_t0, &c->ev_t1, &c->ev_loop0, &c->ev_loop1})
        if (*e) (void)hipEventDestroy(*e);
    if (c->stream) (void)hipStreamDestroy(c->stream);
    void *bufs[] = {c->rows, c->dphi, c->ih, c->bfac, c->x, c->r, c->p[0], c->p[1],
                    c->bplane, c->br, c->partial, c->poles, c->sc};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    if (c->h_sc) (void)hipHostFree(c->h_sc);
    delete c;
}

template <typename T>
hipError_t dalloc(T **p, size_t count)
{
    return hipMalloc(reinterpret_cast<void **>(p), std::max<size_t>(1, count) * sizeof(T));
}

// Copy between an unpadded phi-fastest array (row length np) and the padded
// internal layout (row length pitch); rows = nr * nt.
hipError_t copy_rows(void *dst, size_t dpitch, const void *src, size_t spitch, size_t width, size_t rows,
                     hipMemcpyKind kind, hipStream_t s)
{
    return hipMemcpy2DAsync(dst, dpitch, src, spitch, width, rows, kind, s);
}

int check_solve_args(pot3d_ctx *c, const void *br, const void *phi, double tol, int maxit)
{
    if (!c) return fail(nullptr, POT3D_EINVAL, "ctx is NULL");
    if (!br) return fail(c, POT3D_EINVAL, "br is NULL");
    if (!phi) return fail(c, POT3D_EINVAL, "phi is NULL");
    if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(c, POT3D_EINVAL, "tol must be finite and >= 0");
    if (maxit < 0) return fail(c, POT3D_EINVAL, "maxit must be >= 0");
    return POT3D_OK;
}

// The solve proper.  br_dev: device Br (nt*np); phi0: initial guess or NULL
// (host or device per `kind_in`); phi_out: destination (host or device).
int run_solve(pot3d_ctx *c, const double *br_dev, const double *phi0, hipMemcpyKind kind_in, double *phi_out,
              hipMemcpyKind kind_out, hipStream_t s, double tol, int maxit, int *iters, double *relres_true)
{
    const size_t rowb = (size_t)c->np * sizeof(double), pitchb = (size_t)c->pitch * sizeof(double);
    const size_t nrows = (size_t)c->nr * c->nt;
    c->have_solution = false;
    HIP_TRY(c, hipEventRecord(c->ev_t0, s));

    HIP_TRY(c, launch_rhs(br_dev, c->bfac, c->dphi, c->nt, c->np, c->pitch, c->bplane, s));
    if (phi0) HIP_TRY(c, copy_rows(c->x, pitchb, phi0, rowb, rowb, nrows, kind_in, s));
    else HIP_TRY(c, launch_fill<double>(c->x, c->npad, 0.0, s));
    HIP_TRY(c, launch_fill<double>(c->p[0], c->npad, 0.0, s));

    DevScalars init{};
    init.tol = tol;
    init.maxit = maxit;
    c->h_sc[0] = init;
    HIP_TRY(c, hipMemcpyAsync(c->sc, &c->h_sc[0], sizeof(DevScalars), hipMemcpyHostToDevice, s));

    // r = b - A x0 and the first residual test
    StencilVecs<double> rv = base_vecs(c);
    rv.in = c->x;
    rv.r = c->r;
    rv.bplane = c->bplane;
    rv.store_r = 1;
    rv.ignore_done = 1;
    HIP_TRY(c, launch_stencil<double>(kResidual, c->tj, c->grid, rv, s));
    HIP_TRY(c, launch_finish(kFinInit, c->sc, c->partial, c->grid.nblocks, s));

    // Replay the m-iteration graph, keeping one graph queued ahead of the poll.
    HIP_TRY(c, hipEventRecord(c->ev_loop0, s));
    int launches = 0;
    int slot = 0;
    HIP_TRY(c, hipGraphLaunch(c->graph, s));
    ++launches;
    HIP_TRY(c, hipMemcpyAsync(&c->h_sc[slot], c->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipEventRecord(c->ev_poll[slot], s));
    const long long max_launches = (long long)maxit / c->graph_m + 3;
    for (;;) {
        const int nxt = slot ^ 1;
        HIP_TRY(c, hipGraphLaunch(c->graph, s));
        ++launches;
        HIP_TRY(c, hipMemcpyAsync(&c->h_sc[nxt], c->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, s));
        HIP_TRY(c, hipEventRecord(c->ev_poll[nxt], s));
        HIP_TRY(c, hipEventSynchronize(c->ev_poll[slot]));
        if (c->h_sc[slot].done || launches > max_launches) break;
        slot = nxt;
    }
    HIP_TRY(c, hipEventRecord(c->ev_loop1, s));

    // True residual ||b - A x|| (no store), pole values, Phi out.
    StencilVecs<double> tv = base_vecs(c);
    tv.in = c->x;
    tv.bplane = c->bplane;
    tv.store_r = 0;
    tv.ignore_done = 1;
    HIP_TRY(c, hipStreamSynchronize(s));
    DevScalars fin = c->h_sc[slot];
    HIP_TRY(c, hipMemcpy(&fin, c->sc, sizeof(DevScalars), hipMemcpyDeviceToHost));
    if (!fin.done) return fail(c, POT3D_EDEVICE, "iteration loop ended without the device done flag");
    if (fin.zero_solution) HIP_TRY(c, launch_fill<double>(c->x, c->npad, 0.0, s));
    HIP_TRY(c, launch_stencil<double>(kResidual, c->tj, c->grid, tv, s));
    HIP_TRY(c, launch_finish(kFinTrue, c->sc, c->partial, c->grid.nblocks, s));
    HIP_TRY(c, launch_poles(c->x, c->dphi, c->nr, c->nt, c->np, c->pitch, kTwoPi, c->poles, s));
    HIP_TRY(c, copy_rows(phi_out, rowb, c->x, pitchb, rowb, nrows, kind_out, s));
    HIP_TRY(c, hipMemcpyAsync(&c->h_sc[0], c->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipEventRecord(c->ev_t1, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    fin = c->h_sc[0];

    float ms_total = 0.f, ms_loop = 0.f;
    (void)hipEventElapsedTime(&ms_total, c->ev_t0, c->ev_t1);
    (void)hipEventElapsedTime(&ms_loop, c->ev_loop0, c->ev_loop1);
    pot3d_stats &st = c->stats;
    st.iters = fin.k;
    st.outer = 1;
    st.status = fin.status;
    st.graph_launches = launches;
    st.relres = fin.relres;
    st.relres_true = fin.zero_solution ? 0.0 : fin.relres_true;
    st.solve_ms = ms_total;
    st.loop_ms = ms_loop;
    st.bytes_per_iter = 64.0 * (double)c->n;
    st.n = c->n;
    st.pitch = c->pitch;
    st.tile_j = c->tj;
    st.chunk_i = c->ci;
    st.blocks = c->grid.nblocks;
    c->have_solution = true;
    if (iters) *iters = fin.k;
    if (relres_true) *relres_true = st.relres_true;
    if (fin.status == POT3D_EBREAKDOWN) return fail(c, POT3D_EBREAKDOWN, "breakdown: non-finite data or p.Ap <= 0");
    if (fin.status == POT3D_ENOCONV) return fail(c, POT3D_ENOCONV, "iteration cap reached before tol");
    return fin.status;
}

}  // namespace

extern "C" {

const char *pot3d_version(void) { return "pot3d-mi355x 0.1 (gfx950, FP64 Jacobi-PCG)"; }

const char *pot3d_last_error(const pot3d_ctx *ctx)
{
    if (ctx) return ctx->err.c_str();
    return g_thread_error.c_str();
}

int pot3d_create(const double *r_faces, int nr, const double *t_faces, int nt, const double *p_faces, int np,
                 int upper_bc, int precision, int device, pot3d_ctx **out)
{
    int v = validate_grid(r_faces, nr, t_faces, nt, p_faces, np, upper_bc, precision, out);
    if (v != POT3D_OK) return v;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return fail(nullptr, POT3D_EDEVICE, "no HIP device");
    if (device < 0 || device >= ndev) return fail(nullptr, POT3D_EINVAL, "device index out of range");
    DeviceGuard guard(device);
    if (!guard.ok) return fail(nullptr, POT3D_EDEVICE, "hipSetDevice failed");

    pot3d_ctx *c = new pot3d_ctx();
    c->device = device;
    c->nr = nr;
    c->nt = nt;
    c->np = np;
    c->precision = precision;
    const int align = std::max(1, env_int("POT3D_PITCH_ALIGN", 8));
    c->pitch = ((np + align - 1) / align) * align;
    c->n = (long long)nr * nt * np;
    c->npad = (long long)nr * nt * c->pitch;
    c->graph_m = std::max(2, env_int("POT3D_GRAPH_ITERS", 16));
    c->graph_m += c->graph_m & 1;   // even, so the p buffers alternate consistently across replays
    c->rf.assign(r_faces, r_faces + nr + 1);
    c->tf.assign(t_faces, t_faces + nt + 1);
    c->pf.assign(p_faces, p_faces + np + 1);
    build_tables(c);
    choose_launch(c);

    auto bail = [&](hipError_t e, const char *what) {
        std::string m = std::string(what) + ": " + hipGetErrorString(e);
        free_ctx(c);
        return fail(nullptr, e == hipErrorOutOfMemory ? POT3D_ENOMEM : POT3D_EDEVICE, m);
    };
    hipError_t e;
#define CREATE_TRY(call)                      \
    do {                                      \
        e = (call);                           \
        if (e != hipSuccess) return bail(e, #call); \
    } while (0)
    CREATE_TRY(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    CREATE_TRY(hipEventCreate(&c->ev_poll[0]));
    CREATE_TRY(hipEventCreate(&c->ev_poll[1]));
    CREATE_TRY(hipEventCreate(&c->ev_t0));
    CREATE_TRY(hipEventCreate(&c->ev_t1));
    CREATE_TRY(hipEventCreate(&c->ev_loop0));
    CREATE_TRY(hipEventCreate(&c->ev_loop1));
    CREATE_TRY(dalloc(&c->rows, c->rows_h.size()));
    CREATE_TRY(dalloc(&c->dphi, (size_t)np));
    CREATE_TRY(dalloc(&c->ih, (size_t)np));
    CREATE_TRY(dalloc(&c->bfac, (size_t)nt));
    CREATE_TRY(dalloc(&c->x, (size_t)c->npad));
    CREATE_TRY(dalloc(&c->r, (size_t)c->npad));
    CREATE_TRY(dalloc(&c->p[0], (size_t)c->npad));
    CREATE_TRY(dalloc(&c->p[1], (size_t)c->npad));
    CREATE_TRY(dalloc(&c->bplane, (size_t)nt * c->pitch));
    CREATE_TRY(dalloc(&c->br, (size_t)nt * np));
    CREATE_TRY(dalloc(&c->partial, (size_t)3 * c->grid.nblocks));
    CREATE_TRY(dalloc(&c->poles, (size_t)2 * nr));
    CREATE_TRY(dalloc(&c->sc, 1));
    CREATE_TRY(hipHostMalloc(reinterpret_cast<void **>(&c->h_sc), 2 * sizeof(DevScalars), hipHostMallocDefault));
    CREATE_TRY(hipMemcpyAsync(c->rows, c->rows_h.data(), c->rows_h.size() * sizeof(RowCoef), hipMemcpyHostToDevice, c->stream));
    CREATE_TRY(hipMemcpyAsync(c->dphi, c->dphi_h.data(), np * sizeof(double), hipMemcpyHostToDevice, c->stream));
    CREATE_TRY(hipMemcpyAsync(c->ih, c->ih_h.data(), np * sizeof(double), hipMemcpyHostToDevice, c->stream));
    CREATE_TRY(hipMemcpyAsync(c->bfac, c->bfac_h.data(), nt * sizeof(double), hipMemcpyHostToDevice, c->stream));
    for (double *b : {c->x, c->r, c->p[0], c->p[1]}) CREATE_TRY(launch_fill<double>(b, c->npad, 0.0, c->stream));
    CREATE_TRY(launch_fill<double>(c->bplane, (long long)nt * c->pitch, 0.0, c->stream));
    CREATE_TRY(launch_fill<double>(c->poles, 2LL * nr, 0.0, c->stream));
    CREATE_TRY(hipMemsetAsync(c->sc, 0, sizeof(DevScalars), c->stream));
    CREATE_TRY(hipStreamSynchronize(c->stream));
#undef CREATE_TRY
    c->grid.rows = c->rows;
    c->grid.dphi = c->dphi;
    c->grid.ih = c->ih;
    // The iteration graph is captured once, on the idle context stream.
    if (capture_graph(c) != POT3D_OK) {
        std::string m = c->err;
        free_ctx(c);
        return fail(nullptr, POT3D_EDEVICE, m);
    }
    *out = c;
    return POT3D_OK;
}

int pot3d_solve(pot3d_ctx *ctx, const double *br, double tol, int maxit, const double *phi0, double *phi, int *iters,
                double *relres_true)
{
    int v = check_solve_args(ctx, br, phi, tol, maxit);
    if (v != POT3D_OK) return v;
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return fail(ctx, POT3D_EDEVICE, "hipSetDevice failed");
    HIP_TRY(ctx, hipMemcpyAsync(ctx->br, br, (size_t)ctx->nt * ctx->np * sizeof(double), hipMemcpyHostToDevice,
                                ctx->stream));
    return run_solve(ctx, ctx->br, phi0, hipMemcpyHostToDevice, phi, hipMemcpyDeviceToHost, ctx->stream, tol, maxit,
                     iters, relres_true);
}

int pot3d_solve_device(pot3d_ctx *ctx, const double *d_br, const double *d_phi0, double *d_phi, void *stream,
                       double tol, int maxit, int *iters, double *relres_true)
{
    int v = check_solve_args(ctx, d_br, d_phi, tol, maxit);
    if (v != POT3D_OK) return v;
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return fail(ctx, POT3D_EDEVICE, "hipSetDevice failed");
    hipStream_t s = stream ? reinterpret_cast<hipStream_t>(stream) : ctx->stream;
    return run_solve(ctx, d_br, d_phi0, hipMemcpyDeviceToDevice, d_phi, hipMemcpyDeviceToDevice, s, tol, maxit, iters,
                     relres_true);
}

int pot3d_apply_device(pot3d_ctx *ctx, const double *d_x, double *d_y, void *stream)
{
    if (!ctx) return fail(nullptr, POT3D_EINVAL, "ctx is NULL");
    if (!d_x || !d_y) return fail(ctx, POT3D_EINVAL, "x or y is NULL");
    if (d_x == d_y) return fail(ctx, POT3D_EINVAL, "x and y must be distinct");
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return fail(ctx, POT3D_EDEVICE, "hipSetDevice failed");
    hipStream_t s = stream ? reinterpret_cast<hipStream_t>(stream) : ctx->stream;
    const size_t rowb = (size_t)ctx->np * sizeof(double), pitchb = (size_t)ctx->pitch * sizeof(double);
    const size_t nrows = (size_t)ctx->nr * ctx->nt;
    HIP_TRY(ctx, copy_rows(ctx->p[1], pitchb, d_x, rowb, rowb, nrows, hipMemcpyDeviceToDevice, s));
    StencilVecs<double> a = base_vecs(ctx);
    a.in = ctx->p[1];
    a.y = ctx->r;
    a.ignore_done = 1;
    HIP_TRY(ctx, launch_stencil<double>(kApply, ctx->tj, ctx->grid, a, s));
    HIP_TRY(ctx, copy_rows(d_y, rowb, ctx->r, pitchb, rowb, nrows, hipMemcpyDeviceToDevice, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    return POT3D_OK;
}

int pot3d_rhs_device(pot3d_ctx *ctx, const double *d_br, double *d_b, void *stream)
{
    if (!ctx) return fail(nullptr, POT3D_EINVAL, "ctx is NULL");
    if (!d_br || !d_b) return fail(ctx, POT3D_EINVAL, "br or b is NULL");
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return fail(ctx, POT3D_EDEVICE, "hipSetDevice failed");
    hipStream_t s = stream ? reinterpret_cast<hipStream_t>(stream) : ctx->stream;
    const size_t rowb = (size_t)ctx->np * sizeof(double), pitchb = (size_t)ctx->pitch * sizeof(double);
    HIP_TRY(ctx, launch_rhs(d_br, ctx->bfac, ctx->dphi, ctx->nt, ctx->np, ctx->pitch, ctx->bplane, s));
    HIP_TRY(ctx, launch_fill<double>(d_b, ctx->n, 0.0, s));
    HIP_TRY(ctx, copy_rows(d_b, rowb, ctx->bplane, pitchb, rowb, (size_t)ctx->nt, hipMemcpyDeviceToDevice, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    return POT3D_OK;
}

int pot3d_pole_values(const pot3d_ctx *ctx, double *north, double *south)
{
    if (!ctx) return fail(nullptr, POT3D_EINVAL, "ctx is NULL");
    pot3d_ctx *c = const_cast<pot3d_ctx *>(ctx);
    if (!north || !south) return fail(c, POT3D_EINVAL, "north or south is NULL");
    if (!ctx->have_solution) return fail(c, POT3D_EINVAL, "no solution yet");
    DeviceGuard guard(ctx->device);
    std::vector<double> h((size_t)2 * ctx->nr);
    HIP_TRY(c, hipMemcpy(h.data(), ctx->poles, h.size() * sizeof(double), hipMemcpyDeviceToHost));
    std::memcpy(north, h.data(), ctx->nr * sizeof(double));
    std::memcpy(south, h.data() + ctx->nr, ctx->nr * sizeof(double));
    return POT3D_OK;
}

int pot3d_get_stats(const pot3d_ctx *ctx, pot3d_stats *out)
{
    if (!ctx) return fail(nullptr, POT3D_EINVAL, "ctx is NULL");
    if (!out) return fail(const_cast<pot3d_ctx *>(ctx), POT3D_EINVAL, "out is NULL");
    *out = ctx->stats;
    out->n = ctx->n;
    out->pitch = ctx->pitch;
    out->tile_j = ctx->tj;
    out->chunk_i = ctx->ci;
    out->blocks = ctx->grid.nblocks;
    out->bytes_per_iter = 64.0 * (double)ctx->n;
    return POT3D_OK;
}

int pot3d_time_kernels(pot3d_ctx *ctx, int reps, double *ms_update_p, double *ms_update_r)
{
    if (!ctx) return fail(nullptr, POT3D_EINVAL, "ctx is NULL");
    if (reps <= 0 || !ms_update_p || !ms_update_r) return fail(ctx, POT3D_EINVAL, "reps > 0 and outputs required");
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return fail(ctx, POT3D_EDEVICE, "hipSetDevice failed");
    hipStream_t s = ctx->stream;
    DevScalars st{};
    st.alpha = 1e-3;
    st.beta = 0.5;
    st.rho = 1.0;
    st.bnorm = 1.0;
    st.tol = 0.0;
    st.maxit = 1 << 30;
    ctx->h_sc[0] = st;
    HIP_TRY(ctx, hipMemcpyAsync(ctx->sc, &ctx->h_sc[0], sizeof(DevScalars), hipMemcpyHostToDevice, s));
    StencilVecs<double> a = base_vecs(ctx);
    a.in = ctx->r;
    a.pold = ctx->p[0];
    a.pnew = ctx->p[1];
    StencilVecs<double> bv = base_vecs(ctx);
    bv.in = ctx->p[1];
    bv.r = ctx->r;
    bv.x = ctx->x;
    HIP_TRY(ctx, launch_stencil<double>(kUpdateP, ctx->tj, ctx->grid, a, s));   // warm-up
    HIP_TRY(ctx, launch_stencil<double>(kUpdateR, ctx->tj, ctx->grid, bv, s));
    HIP_TRY(ctx, hipEventRecord(ctx->ev_t0, s));
    for (int q = 0; q < reps; ++q) HIP_TRY(ctx, launch_stencil<double>(kUpdateP, ctx->tj, ctx->grid, a, s));
    HIP_TRY(ctx, hipEventRecord(ctx->ev_t1, s));
    HIP_TRY(ctx, hipEventRecord(ctx->ev_loop0, s));
    for (int q = 0; q < reps; ++q) HIP_TRY(ctx, launch_stencil<double>(kUpdateR, ctx->tj, ctx->grid, bv, s));
    HIP_TRY(ctx, hipEventRecord(ctx->ev_loop1, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    float ma = 0.f, mb = 0.f;
    HIP_TRY(ctx, hipEventElapsedTime(&ma, ctx->ev_t0, ctx->ev_t1));
    HIP_TRY(ctx, hipEventElapsedTime(&mb, ctx->ev_loop0, ctx->ev_loop1));
    *ms_update_p = ma / reps;
    *ms_update_r = mb / reps;
    ctx->have_solution = false;
    return POT3D_OK;
}

void pot3d_destroy(pot3d_ctx *ctx) { free_ctx(ctx); }

}  // extern "C"
