// server.hip -- continuous batching of potential-field solves on one GPU.
//
// Requests (a grid, a surface map Br, tol, maxit) queue on the host.  Each
// step of the server:
//   1. retires finished slots: true residual, pole values, Phi copied out.
//      In FP32-refined mode a finished inner solve instead gets its
//      correction, an FP64 outer test, and either a new inner solve or
//      retirement;
//   2. admits queued requests, in arrival order, while a slot is free, their
//      device footprint fits the HBM budget, and the bytes that all active
//      solves stream per iteration stay within the cache budget (by default
//      the 256 MB memory-side cache) -- or the server is idle.  Solves that
//      run from the cache alone are thus not batched into ones that would
//      stream from HBM, and bandwidth-bound solves, which batching cannot
//      speed up, run alone.  A request that does not fit beside the running
//      solves is passed over by later ones that do (small solves batch while
//      a large one waits for the server to drain), at most kMaxOvertake
//      times.  Per-grid contexts (tables and vectors) are cached and reused;
//      idle ones are evicted oldest first when the budget needs it;
//   3. queues one replay of a captured graph of m batched PCG iterations (in
//      the one-sweep form, the default: 2m sweeps of one batched sweep and one
//      finisher each; in the two-pass form m iterations of two batched passes
//      and two finishers; the form is fixed when the server is created).
//      Each kernel of it covers every active slot (a slot table in device
//      memory maps workgroups to slots), and slots that have converged are
//      masked by their own done flags.
// A step queues its replay before it reads the statuses of the previous one,
// so in steps where no solve ends or starts the device has the next replay
// queued while the host decides.  A step that retires or admits a request
// waits for the stream (Phi out, the refined mode's outer check, the slot
// tables), so the pipeline drains there.  A slot that finished in replay k
// runs through replay k+1 as a no-op, and retirement and admission are
// ordered after it on the same stream.
// The graphs read the slot tables at run time, so requests join and leave
// between replays without recapture; one graph is captured per launch width
// (pair of widths in the two-pass form) the first time a batch needs it.
// Every slot runs exactly the launch shape, tile order and reduction order of
// a single solve on the same grid in the same form, so each result is
// bitwise the one the request gets from pot3d_solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "context.hpp"

using namespace pot3d;
using namespace pot3d::host;

namespace {

struct Request {
    long long id = 0;
    int nr = 0, nt = 0, np = 0;
    std::vector<double> rf, tf, pf, br;
    double tol = 0.0;
    int maxit = 0;
    double *phi_out = nullptr;                 // caller's buffer (from submit), or NULL
    std::unique_ptr<double[]> phi_buf;         // otherwise Phi is kept here until taken
    int status = POT3D_OK, iters = 0, outer = 0;
    double relres_true = 0.0;
    double t_submit = 0.0, t_admit = -1.0, t_done = -1.0;
    bool done = false;
    int overtaken = 0;   // later requests admitted while this one waited for streaming budget
};

struct Slot {
    pot3d_ctx *ctx = nullptr;
    Request *req = nullptr;
    bool active = false;
    int total_inner = 0, outer = 0, launches = 0;
    unsigned phase = 0;   // bumped whenever the slot's solve (re)starts on the device
    DevScalars last_inner{};   // refined: scalars of the inner segment that just ended
    double scale_prev = 0.0;   // refined: the normalisation that segment ran in
};

// A captured batched graph: launch widths of the two passes, last use.
struct BatchGraph {
    int wp = 0, wr = 0;
    unsigned long long last_use = 0;
    hipGraphExec_t exec = nullptr;
};

// What a queued replay covered: per slot, the request and phase at launch.
struct Replay {
    bool pending = false;
    std::vector<Request *> req;
    std::vector<unsigned> phase;
    hipEvent_t done = nullptr;
};

constexpr int kBlockAlign = 8;   // slot offsets keep the XCD of a workgroup unchanged
constexpr int kMaxOvertake = 8;  // later requests that may pass one waiting for streaming budget

int round_up(int v, int a) { return (v + a - 1) / a * a; }

}  // namespace

struct pot3d_server {
    int device = 0, precision = POT3D_FP64, max_slots = 0, graph_m = 16;
    int tile_p = kTileMarch8, tile_r = kTileMarch8;   // launch shapes of every slot
    bool sweep = true;       // one-sweep batches (else two passes)
    int sweep_rows = 4;      // box rows per wavefront of every slot's sweep kernel
    size_t budget = 0, used = 0;
    size_t cache_budget = size_t(256) << 20;   // bytes streamed per iteration by the active set
    hipStream_t stream = nullptr, capture_stream = nullptr;
    std::deque<Request *> queue;
    std::map<long long, std::unique_ptr<Request>> requests;
    long long next_id = 1, finished = 0, replays = 0;
    unsigned next_phase = 0;
    std::vector<Slot> slots;
    std::vector<pot3d_ctx *> idle;   // cached contexts, oldest first
    // slot tables [parity][slot]: update-p and update-r, FP64 or FP32
    BatchSlot<double> *d_p64[2] = {nullptr, nullptr}, *d_r64[2] = {nullptr, nullptr};
    BatchSlot<float> *d_p32[2] = {nullptr, nullptr}, *d_r32[2] = {nullptr, nullptr};
    BatchFin *d_finp = nullptr, *d_finr = nullptr;
    std::vector<BatchSlot<double>> h_p64[2], h_r64[2];
    std::vector<BatchSlot<float>> h_p32[2], h_r32[2];
    std::vector<BatchFin> h_finp, h_finr;
    // one-sweep slot tables [parity][slot] (the finishers use d_finp)
    BatchSweep<double> *d_s64[2] = {nullptr, nullptr};
    BatchSweep<float> *d_s32[2] = {nullptr, nullptr};
    std::vector<BatchSweep<double>> h_s64[2];
    std::vector<BatchSweep<float>> h_s32[2];
    DevScalars *h_status = nullptr;   // pinned, [2][slot]: statuses after the two latest replays
    Replay replay[2];
    int last = -1;                    // replay buffer of the most recent launch
    std::vector<BatchGraph> graphs;   // captured batched graphs by launch widths
    unsigned long long graph_clock = 0;
    int need_p = 0, need_r = 0;   // workgroups the active slots own in each pass (need_p: the sweep)
    std::chrono::steady_clock::time_point t0;
    std::string err;

    double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
};

namespace {

thread_local std::string g_server_error;

int sfail(pot3d_server *sv, int code, const std::string &msg)
{
    if (sv) sv->err = msg;
    else g_server_error = msg;
    return code;
}

#define SV_TRY(sv, call)                                                                             \
    do {                                                                                             \
        hipError_t e_ = (call);                                                                      \
        if (e_ != hipSuccess)                                                                        \
            return sfail((sv), e_ == hipErrorOutOfMemory ? POT3D_ENOMEM : POT3D_EDEVICE,             \
                         std::string(#call) + ": " + hipGetErrorString(e_));                        \
    } while (0)

#define SV_CALL(sv, ctx, call)                                                                       \
    do {                                                                                             \
        int rc_ = (call);                                                                            \
        if (rc_ != POT3D_OK) return sfail((sv), rc_, pot3d_last_error(ctx));                          \
    } while (0)

template <typename T>
hipError_t dalloc(T **p, size_t count)
{
    return hipMalloc(reinterpret_cast<void **>(p), std::max<size_t>(1, count) * sizeof(T));
}

template <typename V>
int capture_batched(pot3d_server *sv, BatchSlot<V> *const *dp, BatchSlot<V> *const *dr, BatchSweep<V> *const *ds,
                    int wp, int wr, hipGraphExec_t *out)
{
    hipStream_t s = sv->capture_stream;
    SV_TRY(sv, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    if (sv->sweep) {
        // 2m sweeps: the parity of the r and p buffers continues across replays
        for (int it = 0; it < 2 * sv->graph_m && e == hipSuccess; ++it) {
            e = launch_sweep_batch<V>(sv->sweep_rows, ds[it & 1], sv->max_slots, wp, sweep_xmode(it), s);
            if (e == hipSuccess) e = launch_finish_batch(kFinSweep, sv->d_finp, sv->max_slots, s);
        }
    }
    for (int it = 0; !sv->sweep && it < sv->graph_m && e == hipSuccess; ++it) {
        e = launch_stencil_batch<V>(kUpdateP, sv->tile_p, dp[it & 1], sv->max_slots, wp, s);
        if (e == hipSuccess) e = launch_finish_batch(kFinSigma, sv->d_finp, sv->max_slots, s);
        if (e == hipSuccess)
            e = launch_stencil_batch<V>(update_r_mode(it, sv->graph_m), sv->tile_r, dr[it & 1], sv->max_slots, wr, s);
        if (e == hipSuccess) e = launch_finish_batch(kFinRho, sv->d_finr, sv->max_slots, s);
    }
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(s, &graph);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return sfail(sv, POT3D_EDEVICE, std::string("batched graph capture: ") +
                                            hipGetErrorString(e != hipSuccess ? e : e2));
    }
    hipError_t e3 = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e3 != hipSuccess) return sfail(sv, POT3D_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e3));
    return POT3D_OK;
}

// The graph whose passes launch exactly the workgroups the active slots own
// (wp for the p update, wr for the r/x update), captured on first need, so
// that no launch carries idle workgroups.  At most kMaxGraphs are kept; the
// least recently used one goes first.
constexpr size_t kMaxGraphs = 64;

int graph_for(pot3d_server *sv, int wp, int wr, hipGraphExec_t *out)
{
    for (size_t q = 0; q < sv->graphs.size(); ++q) {
        if (sv->graphs[q].wp == wp && sv->graphs[q].wr == wr) {
            sv->graphs[q].last_use = ++sv->graph_clock;
            *out = sv->graphs[q].exec;
            return POT3D_OK;
        }
    }
    if (sv->graphs.size() >= kMaxGraphs) {
        size_t oldest = 0;
        for (size_t q = 1; q < sv->graphs.size(); ++q)
            if (sv->graphs[q].last_use < sv->graphs[oldest].last_use) oldest = q;
        // the stream may still replay it: wait before destroying
        SV_TRY(sv, hipStreamSynchronize(sv->stream));
        (void)hipGraphExecDestroy(sv->graphs[oldest].exec);
        sv->graphs.erase(sv->graphs.begin() + oldest);
    }
    hipGraphExec_t g = nullptr;
    const int rc = sv->precision == POT3D_FP64 ? capture_batched<double>(sv, sv->d_p64, sv->d_r64, sv->d_s64, wp, wr, &g)
                                               : capture_batched<float>(sv, sv->d_p32, sv->d_r32, sv->d_s32, wp, wr, &g);
    if (rc != POT3D_OK) return rc;
    sv->graphs.push_back(BatchGraph{wp, wr, ++sv->graph_clock, g});
    *out = g;
    return POT3D_OK;
}

// Slot tables from the current slots (inactive slots own no workgroups).
template <typename V>
void fill_tables(pot3d_server *sv, std::vector<BatchSlot<V>> *hp, std::vector<BatchSlot<V>> *hr,
                 std::vector<BatchSweep<V>> *hs)
{
    int offp = 0, offr = 0;
    for (int q = 0; q < sv->max_slots; ++q) {
        const Slot &sl = sv->slots[q];
        for (int par = 0; par < 2; ++par) {
            hp[par][q] = BatchSlot<V>{};
            hr[par][q] = BatchSlot<V>{};
            hs[par][q] = BatchSweep<V>{};
        }
        sv->h_finp[q] = BatchFin{};
        sv->h_finr[q] = BatchFin{};
        if (!sl.active) continue;
        pot3d_ctx *c = sl.ctx;
        V *r, *r2, *x, *p[2];
        DevScalars *sc;
        if constexpr (std::is_same<V, double>::value) {
            r = c->r;
            r2 = c->r2;
            x = c->x;
            p[0] = c->p[0];
            p[1] = c->p[1];
            sc = c->sc;
        } else {
            r = c->r32;
            r2 = c->r32b;
            x = c->e32;
            p[0] = c->p32[0];
            p[1] = c->p32[1];
            sc = c->sc32;
        }
        if (sv->sweep) {
            V *rb[2] = {r, r2};
            for (int par = 0; par < 2; ++par) {
                BatchSweep<V> &a = hs[par][q];
                a.g = c->grid_s;
                a.v.r_in = rb[par];
                a.v.r_out = rb[par ^ 1];
                a.v.p_old = p[par];
                a.v.p_new = p[par ^ 1];
                a.v.x = x;
                a.v.sc = sc;
                a.v.partial = c->partial;
                a.offset = offp;
                a.active = 1;
            }
            sv->h_finp[q] = BatchFin{sc, c->partial, c->grid_s.nblocks, 1};
            offp += round_up(c->grid_s.nblocks, kBlockAlign);
            continue;
        }
        for (int par = 0; par < 2; ++par) {
            BatchSlot<V> &a = hp[par][q];
            a.g = c->grid_p;
            a.v.in = r;
            a.v.pold = p[par];
            a.v.pnew = p[par ^ 1];
            a.v.sc = sc;
            a.v.partial = c->partial;
            a.out = p[par ^ 1];
            a.offset = offp;
            a.active = 1;
            BatchSlot<V> &b = hr[par][q];
            b.g = c->grid_r;
            b.v.in = p[par ^ 1];
            b.v.pold = p[par];   // p_{k-1}, for the r/x update that pairs two iterations
            b.v.r = r;
            b.v.x = x;
            b.v.sc = sc;
            b.v.partial = c->partial;
            b.out = r;
            b.offset = offr;
            b.active = 1;
        }
        sv->h_finp[q] = BatchFin{sc, c->partial, c->grid_p.nblocks, 1};
        sv->h_finr[q] = BatchFin{sc, c->partial, c->grid_r.nblocks, 1};
        offp += round_up(c->grid_p.nblocks, kBlockAlign);
        offr += round_up(c->grid_r.nblocks, kBlockAlign);
    }
    sv->need_p = offp;
    sv->need_r = offr;
}

int upload_tables(pot3d_server *sv)
{
    hipStream_t s = sv->stream;
    const size_t n = sv->max_slots;
    if (sv->precision == POT3D_FP64) {
        fill_tables<double>(sv, sv->h_p64, sv->h_r64, sv->h_s64);
        for (int par = 0; par < 2; ++par) {
            SV_TRY(sv, hipMemcpyAsync(sv->d_p64[par], sv->h_p64[par].data(), n * sizeof(BatchSlot<double>),
                                      hipMemcpyHostToDevice, s));
            SV_TRY(sv, hipMemcpyAsync(sv->d_r64[par], sv->h_r64[par].data(), n * sizeof(BatchSlot<double>),
                                      hipMemcpyHostToDevice, s));
            SV_TRY(sv, hipMemcpyAsync(sv->d_s64[par], sv->h_s64[par].data(), n * sizeof(BatchSweep<double>),
                                      hipMemcpyHostToDevice, s));
        }
    } else {
        fill_tables<float>(sv, sv->h_p32, sv->h_r32, sv->h_s32);
        for (int par = 0; par < 2; ++par) {
            SV_TRY(sv, hipMemcpyAsync(sv->d_p32[par], sv->h_p32[par].data(), n * sizeof(BatchSlot<float>),
                                      hipMemcpyHostToDevice, s));
            SV_TRY(sv, hipMemcpyAsync(sv->d_r32[par], sv->h_r32[par].data(), n * sizeof(BatchSlot<float>),
                                      hipMemcpyHostToDevice, s));
            SV_TRY(sv, hipMemcpyAsync(sv->d_s32[par], sv->h_s32[par].data(), n * sizeof(BatchSweep<float>),
                                      hipMemcpyHostToDevice, s));
        }
    }
    SV_TRY(sv, hipMemcpyAsync(sv->d_finp, sv->h_finp.data(), n * sizeof(BatchFin), hipMemcpyHostToDevice, s));
    SV_TRY(sv, hipMemcpyAsync(sv->d_finr, sv->h_finr.data(), n * sizeof(BatchFin), hipMemcpyHostToDevice, s));
    // the tables are pageable host vectors: finish the copies before they change
    SV_TRY(sv, hipStreamSynchronize(s));
    return POT3D_OK;
}

// Bytes one iteration of a request streams: FP64 x, r and two directions (and
// the second r of the one-sweep form), or in refined mode the FP32 vectors of
// the inner solve.
size_t stream_bytes(const pot3d_server *sv, const Request *r)
{
    const size_t pitch = (size_t)(r->np + 7) / 8 * 8;
    const size_t vectors = sv->sweep ? 5 : 4;
    return (size_t)r->nr * r->nt * pitch * vectors * (sv->precision == POT3D_FP32_REFINED ? 4 : 8);
}

bool same_grid(const pot3d_ctx *c, const Request *r)
{
    return c->nr == r->nr && c->nt == r->nt && c->np == r->np && c->rf == r->rf && c->tf == r->tf && c->pf == r->pf;
}

void release_context(pot3d_server *sv, pot3d_ctx *c)
{
    sv->idle.push_back(c);
}

void evict_one(pot3d_server *sv)
{
    pot3d_ctx *c = sv->idle.front();
    sv->idle.erase(sv->idle.begin());
    sv->used -= context_bytes(c);
    free_ctx(c);
}

// A context for r: a cached one with the same grid, or a new one if the budget
// allows (evicting idle contexts oldest first).  *ctx = NULL: not now.
int acquire_context(pot3d_server *sv, Request *r, pot3d_ctx **ctx)
{
    *ctx = nullptr;
    for (size_t q = 0; q < sv->idle.size(); ++q) {
        if (same_grid(sv->idle[q], r)) {
            *ctx = sv->idle[q];
            sv->idle.erase(sv->idle.begin() + q);
            return POT3D_OK;
        }
    }
    // estimate before allocating: 4 FP64 vectors (+4 or 5 FP32 in refined mode,
    // +1 FP64 in the FP64 one-sweep form) of the padded size, plus tables
    const long long pitch = (r->np + 7) / 8 * 8;
    const size_t per_cell = sv->precision == POT3D_FP32_REFINED ? (sv->sweep ? 52 : 48) : (sv->sweep ? 40 : 32);
    const size_t need = (size_t)r->nr * r->nt * pitch * per_cell +
                        (size_t)r->nr * r->nt * 64 + (size_t)r->nt * pitch * 16 + (1u << 20);
    while (sv->used + need > sv->budget && !sv->idle.empty()) evict_one(sv);
    if (sv->used + need > sv->budget) return POT3D_OK;   // wait for a slot to retire
    pot3d_ctx *c = nullptr;
    int rc = create_context(r->rf.data(), r->nr, r->tf.data(), r->nt, r->pf.data(), r->np, POT3D_UPPER_SOURCE_SURFACE,
                            sv->precision, sv->device, true, &c);
    if (rc != POT3D_OK) return sfail(sv, rc, pot3d_last_error(nullptr));
    if (c->tile_p != sv->tile_p || c->tile_r != sv->tile_r || c->sweep_rows != sv->sweep_rows ||
        (sv->sweep && (c->precision == POT3D_FP64 ? !c->r2 : !c->r32b))) {
        free_ctx(c);
        return sfail(sv, POT3D_EINVAL, "context launch shape differs from the server's batched kernels");
    }
    sv->used += context_bytes(c);
    *ctx = c;
    return POT3D_OK;
}

void complete(pot3d_server *sv, Slot &sl, int status, int iters, int outer, double relres_true)
{
    Request *r = sl.req;
    r->status = status;
    r->iters = iters;
    r->outer = outer;
    r->relres_true = relres_true;
    r->t_done = sv->now();
    r->done = true;
    ++sv->finished;
    release_context(sv, sl.ctx);
    sl = Slot{};
}

// Retire a slot whose solve has ended: true residual, pole values, Phi out.
int retire(pot3d_server *sv, Slot &sl, DevScalars fin, int total_iters, int outer)
{
    pot3d_ctx *c = sl.ctx;
    Request *r = sl.req;
    double *dst = r->phi_out;
    if (!dst) {
        r->phi_buf.reset(new double[(size_t)r->nr * r->nt * r->np]);
        dst = r->phi_buf.get();
    }
    int iters = 0;
    double rel = 0.0;
    SV_TRY(sv, hipEventRecord(c->ev_loop1, sv->stream));
    const bool fp32 = sv->precision == POT3D_FP32_REFINED;
    const double per_unknown = sv->sweep ? sweep_bytes(fp32) : two_pass_bytes(fp32, sv->graph_m);
    // the x increment the slot's last sweep may have left (FP64; refined
    // slots caught up their correction before the outer test)
    if (!fp32) SV_TRY(sv, launch_x_catchup<double>(c->x, c->sc, c->nr, c->nt, c->np, c->pitch, sv->stream));
    const int rc = finish_solve(c, dst, hipMemcpyDeviceToHost, sv->stream, fin, sl.launches, total_iters, outer,
                                per_unknown, &iters, &rel);
    if (rc != POT3D_OK && rc != POT3D_ENOCONV && rc != POT3D_EBREAKDOWN) return sfail(sv, rc, pot3d_last_error(c));
    complete(sv, sl, rc, iters, outer, rel);
    return POT3D_OK;
}

// Refined slot: the outer test, then retire or start the next inner solve.
int refined_advance(pot3d_server *sv, Slot &sl)
{
    pot3d_ctx *c = sl.ctx;
    Request *r = sl.req;
    DevScalars out{};
    SV_CALL(sv, c, refined_outer_check(c, sv->stream, &out));
    if (out.done) return retire(sv, sl, out, sl.total_inner, sl.outer);
    if (sl.outer >= c->max_outer || sl.total_inner >= r->maxit) {
        out.status = POT3D_ENOCONV;
        return retire(sv, sl, out, sl.total_inner, sl.outer);
    }
    SV_CALL(sv, c, refined_start_inner(c, sv->stream, r->tol, r->maxit - sl.total_inner, out,
                                       sl.outer > 0 ? &sl.last_inner : nullptr, sl.scale_prev));
    sl.scale_prev = out.scale;
    sl.phase = ++sv->next_phase;
    return POT3D_OK;
}

int admit(pot3d_server *sv, Slot &sl, Request *r, pot3d_ctx *c)
{
    hipStream_t s = sv->stream;
    sl = Slot{};
    sl.ctx = c;
    sl.req = r;
    sl.active = true;
    sl.phase = ++sv->next_phase;
    r->t_admit = sv->now();
    SV_TRY(sv, hipEventRecord(c->ev_t0, s));
    SV_TRY(sv, hipMemcpyAsync(c->br, r->br.data(), r->br.size() * sizeof(double), hipMemcpyHostToDevice, s));
    SV_CALL(sv, c, prepare_solve(c, c->br, nullptr, hipMemcpyHostToDevice, s));
    SV_TRY(sv, hipEventRecord(c->ev_loop0, s));
    if (sv->precision == POT3D_FP64) {
        SV_CALL(sv, c, start_fp64(c, s, r->tol, r->maxit));
        return POT3D_OK;
    }
    DevScalars init{};
    init.tol = r->tol;
    init.maxit = r->maxit;
    c->h_sc[0] = init;
    SV_TRY(sv, hipMemcpyAsync(c->sc, &c->h_sc[0], sizeof(DevScalars), hipMemcpyHostToDevice, s));
    return refined_advance(sv, sl);
}

}  // namespace

extern "C" {

const char *pot3d_server_last_error(const pot3d_server *sv) { return sv ? sv->err.c_str() : g_server_error.c_str(); }

int pot3d_server_create(int device, int precision, int max_slots, double hbm_budget_bytes, pot3d_server **out)
{
    if (!out) return sfail(nullptr, POT3D_EINVAL, "out is NULL");
    *out = nullptr;
    if (precision != POT3D_FP64 && precision != POT3D_FP32_REFINED) return sfail(nullptr, POT3D_EINVAL, "bad precision");
    if (max_slots < 1 || max_slots > 64) return sfail(nullptr, POT3D_EINVAL, "max_slots must be in [1, 64]");
    if (!(hbm_budget_bytes >= 0.0) || !std::isfinite(hbm_budget_bytes))
        return sfail(nullptr, POT3D_EINVAL, "hbm_budget_bytes must be finite and >= 0 (0: 80% of free memory)");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return sfail(nullptr, POT3D_EDEVICE, "no HIP device");
    if (device < 0 || device >= ndev) return sfail(nullptr, POT3D_EINVAL, "device index out of range");
    DeviceGuard guard(device);
    if (!guard.ok) return sfail(nullptr, POT3D_EDEVICE, "hipSetDevice failed");

    auto sv = std::make_unique<pot3d_server>();
    sv->device = device;
    sv->precision = precision;
    sv->max_slots = max_slots;
    sv->t0 = std::chrono::steady_clock::now();
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return sfail(nullptr, POT3D_EDEVICE, "hipMemGetInfo failed");
    sv->budget = hbm_budget_bytes > 0.0 ? (size_t)hbm_budget_bytes : (size_t)(0.8 * (double)free_b);
    default_tiles(precision, &sv->tile_p, &sv->tile_r);
    sv->sweep = env_int("POT3D_ITERATION", POT3D_ITER_ONE_SWEEP) != POT3D_ITER_TWO_PASS;
    const int rows = env_int("POT3D_SWEEP_ROWS", 4);
    sv->sweep_rows = valid_sweep_rows(rows) ? rows : 4;
    sv->slots.assign(max_slots, Slot{});
    for (int par = 0; par < 2; ++par) {
        sv->h_p64[par].assign(max_slots, BatchSlot<double>{});
        sv->h_r64[par].assign(max_slots, BatchSlot<double>{});
        sv->h_p32[par].assign(max_slots, BatchSlot<float>{});
        sv->h_r32[par].assign(max_slots, BatchSlot<float>{});
        sv->h_s64[par].assign(max_slots, BatchSweep<double>{});
        sv->h_s32[par].assign(max_slots, BatchSweep<float>{});
    }
    sv->h_finp.assign(max_slots, BatchFin{});
    sv->h_finr.assign(max_slots, BatchFin{});
    pot3d_server *p = sv.get();
    auto bail = [&](int code) {
        pot3d_server_destroy(sv.release());
        return code;
    };
    hipError_t e = hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking);
    for (int b = 0; b < 2 && e == hipSuccess; ++b) {
        p->replay[b].req.assign(max_slots, nullptr);
        p->replay[b].phase.assign(max_slots, 0);
        e = hipEventCreateWithFlags(&p->replay[b].done, hipEventDisableTiming);
    }
    for (int par = 0; par < 2 && e == hipSuccess; ++par) {
        if (precision == POT3D_FP64) {
            e = dalloc(&p->d_p64[par], max_slots);
            if (e == hipSuccess) e = dalloc(&p->d_r64[par], max_slots);
            if (e == hipSuccess) e = dalloc(&p->d_s64[par], max_slots);
        } else {
            e = dalloc(&p->d_p32[par], max_slots);
            if (e == hipSuccess) e = dalloc(&p->d_r32[par], max_slots);
            if (e == hipSuccess) e = dalloc(&p->d_s32[par], max_slots);
        }
    }
    if (e == hipSuccess) e = dalloc(&p->d_finp, max_slots);
    if (e == hipSuccess) e = dalloc(&p->d_finr, max_slots);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&p->h_status), 2 * max_slots * sizeof(DevScalars),
                                           hipHostMallocDefault);
    if (e != hipSuccess) {
        sfail(nullptr, POT3D_EDEVICE, std::string("server allocation: ") + hipGetErrorString(e));
        return bail(POT3D_EDEVICE);
    }
    if (upload_tables(p) != POT3D_OK) {
        g_server_error = p->err;
        return bail(POT3D_EDEVICE);
    }
    // one graph now, so that capture problems show here
    hipGraphExec_t g0 = nullptr;
    const int rc = graph_for(p, kBlockAlign, p->sweep ? 0 : kBlockAlign, &g0);
    if (rc != POT3D_OK) {
        g_server_error = p->err;
        return bail(rc);
    }
    *out = sv.release();
    return POT3D_OK;
}

int pot3d_server_submit(pot3d_server *sv, const double *r_faces, int nr, const double *t_faces, int nt,
                        const double *p_faces, int np, const double *br, double tol, int maxit, double *phi_out,
                        long long *id)
{
    if (!sv) return sfail(nullptr, POT3D_EINVAL, "server is NULL");
    if (!id || !br) return sfail(sv, POT3D_EINVAL, "br and id are required");
    pot3d_ctx *dummy = nullptr;
    if (validate_grid(r_faces, nr, t_faces, nt, p_faces, np, POT3D_UPPER_SOURCE_SURFACE, sv->precision, &dummy) !=
        POT3D_OK)
        return sfail(sv, POT3D_EINVAL, pot3d_last_error(nullptr));
    if (!(tol >= 0.0) || !std::isfinite(tol) || maxit < 0) return sfail(sv, POT3D_EINVAL, "bad tol or maxit");
    auto r = std::make_unique<Request>();
    r->id = sv->next_id++;
    r->nr = nr;
    r->nt = nt;
    r->np = np;
    r->rf.assign(r_faces, r_faces + nr + 1);
    r->tf.assign(t_faces, t_faces + nt + 1);
    r->pf.assign(p_faces, p_faces + np + 1);
    r->br.assign(br, br + (size_t)nt * np);
    r->tol = tol;
    r->maxit = maxit;
    r->phi_out = phi_out;
    r->t_submit = sv->now();
    *id = r->id;
    sv->queue.push_back(r.get());
    sv->requests[r->id] = std::move(r);
    return POT3D_OK;
}

int pot3d_server_step(pot3d_server *sv, int *n_active, int *n_queued, long long *n_finished)
{
    if (!sv) return sfail(nullptr, POT3D_EINVAL, "server is NULL");
    DeviceGuard guard(sv->device);
    if (!guard.ok) return sfail(sv, POT3D_EDEVICE, "hipSetDevice failed");
    hipStream_t s = sv->stream;
    const int prev = sv->last;
    // 1. queue the next replay of the active slots (the tables are current),
    //    with a copy of each slot's scalars after it
    int launched = -1;
    int active = 0;
    for (const Slot &sl : sv->slots) active += sl.active ? 1 : 0;
    if (active > 0) {
        const int b = prev == 0 ? 1 : 0;
        hipGraphExec_t g = nullptr;
        const int rc = graph_for(sv, sv->need_p, sv->need_r, &g);
        if (rc != POT3D_OK) return rc;
        SV_TRY(sv, hipGraphLaunch(g, s));
        ++sv->replays;
        Replay &rp = sv->replay[b];
        for (int q = 0; q < sv->max_slots; ++q) {
            Slot &sl = sv->slots[q];
            rp.req[q] = sl.active ? sl.req : nullptr;
            rp.phase[q] = sl.phase;
            if (!sl.active) continue;
            sl.launches += 1;
            DevScalars *src = sv->precision == POT3D_FP64 ? sl.ctx->sc : sl.ctx->sc32;
            SV_TRY(sv, hipMemcpyAsync(&sv->h_status[b * sv->max_slots + q], src, sizeof(DevScalars),
                                      hipMemcpyDeviceToHost, s));
        }
        SV_TRY(sv, hipEventRecord(rp.done, s));
        rp.pending = true;
        launched = b;
    }
    // 2. slots whose current solve ended in the previous replay (the one just
    //    queued is a no-op for them; what follows is ordered after it)
    bool changed = false;
    if (prev >= 0 && sv->replay[prev].pending) {
        Replay &rp = sv->replay[prev];
        SV_TRY(sv, hipEventSynchronize(rp.done));
        rp.pending = false;
        for (int q = 0; q < sv->max_slots; ++q) {
            Slot &sl = sv->slots[q];
            if (!sl.active || rp.req[q] != sl.req || rp.phase[q] != sl.phase) continue;
            const DevScalars st = sv->h_status[prev * sv->max_slots + q];
            if (!st.done) continue;
            changed = true;
            if (sv->precision == POT3D_FP64) {
                const int rc = retire(sv, sl, st, st.k, 1);
                if (rc != POT3D_OK) return rc;
                continue;
            }
            sl.total_inner += st.k;
            sl.outer += 1;
            sl.last_inner = st;
            if (st.status == POT3D_EBREAKDOWN) {
                DevScalars out = st;
                out.status = POT3D_EBREAKDOWN;
                const int rc = retire(sv, sl, out, sl.total_inner, sl.outer);
                if (rc != POT3D_OK) return rc;
                continue;
            }
            SV_TRY(sv, launch_x_catchup<float>(sl.ctx->e32, sl.ctx->sc32, sl.ctx->nr, sl.ctx->nt, sl.ctx->np,
                                               sl.ctx->pitch, s));
            SV_CALL(sv, sl.ctx, refined_correct(sl.ctx, s));
            const int rc = refined_advance(sv, sl);
            if (rc != POT3D_OK) return rc;
        }
    }
    sv->last = launched;
    // 3. admissions
    size_t streaming = 0;
    int running = 0;
    for (const Slot &sl : sv->slots)
        if (sl.active) {
            streaming += stream_bytes(sv, sl.req);
            ++running;
        }
    for (Slot &sl : sv->slots) {
        if (sl.active || sv->queue.empty()) continue;
        // the first queued request, in arrival order, that fits the streaming
        // budget beside the running solves; the ones it passes are counted, and
        // one that has been passed kMaxOvertake times blocks the queue until it
        // fits (at the latest when the server is idle)
        size_t pick = sv->queue.size();
        bool blocked = false;
        for (size_t qi = 0; qi < sv->queue.size(); ++qi) {
            const size_t sb_q = stream_bytes(sv, sv->queue[qi]);
            if (running == 0 || sv->cache_budget == 0 || streaming + sb_q <= sv->cache_budget) {
                pick = qi;
                break;
            }
            if (sv->queue[qi]->overtaken >= kMaxOvertake) {
                blocked = true;
                break;
            }
        }
        if (blocked || pick == sv->queue.size()) break;
        Request *r = sv->queue[pick];
        const size_t sb = stream_bytes(sv, r);
        pot3d_ctx *c = nullptr;
        int rc = acquire_context(sv, r, &c);
        if (rc != POT3D_OK) {   // the request cannot run on this server
            sv->queue.erase(sv->queue.begin() + (long)pick);
            r->status = rc;
            r->t_done = sv->now();
            r->done = true;
            ++sv->finished;
            continue;
        }
        if (!c) break;   // wait for memory
        for (size_t qi = 0; qi < pick; ++qi) sv->queue[qi]->overtaken += 1;
        sv->queue.erase(sv->queue.begin() + (long)pick);
        changed = true;
        rc = admit(sv, sl, r, c);
        if (rc != POT3D_OK) return rc;
        if (sl.active) {
            streaming += sb;
            ++running;
        }
    }
    if (changed) {
        const int rc = upload_tables(sv);
        if (rc != POT3D_OK) return rc;
    }
    active = 0;
    for (const Slot &sl : sv->slots) active += sl.active ? 1 : 0;
    if (n_active) *n_active = active;
    if (n_queued) *n_queued = (int)sv->queue.size();
    if (n_finished) *n_finished = sv->finished;
    return POT3D_OK;
}

int pot3d_server_result(pot3d_server *sv, long long id, double *phi, pot3d_request_info *info)
{
    if (!sv) return sfail(nullptr, POT3D_EINVAL, "server is NULL");
    auto it = sv->requests.find(id);
    if (it == sv->requests.end()) return sfail(sv, POT3D_EINVAL, "unknown request id");
    Request *r = it->second.get();
    if (info) {
        info->id = r->id;
        info->done = r->done ? 1 : 0;
        info->status = r->status;
        info->iters = r->iters;
        info->outer = r->outer;
        info->nr = r->nr;
        info->nt = r->nt;
        info->np = r->np;
        info->relres_true = r->relres_true;
        info->t_submit = r->t_submit;
        info->t_admit = r->t_admit;
        info->t_done = r->t_done;
    }
    if (r->done && phi) {
        const size_t n = (size_t)r->nr * r->nt * r->np;
        const double *src = r->phi_out ? r->phi_out : r->phi_buf.get();
        if (src && src != phi) std::memcpy(phi, src, n * sizeof(double));
        sv->requests.erase(it);
    }
    return POT3D_OK;
}

int pot3d_server_set_cache_budget(pot3d_server *sv, double bytes)
{
    if (!sv) return sfail(nullptr, POT3D_EINVAL, "server is NULL");
    if (!(bytes >= 0.0) || !std::isfinite(bytes)) return sfail(sv, POT3D_EINVAL, "bytes must be finite and >= 0");
    sv->cache_budget = (size_t)bytes;
    return POT3D_OK;
}

int pot3d_server_get_stats(const pot3d_server *sv, pot3d_server_stats *out)
{
    if (!sv || !out) return sfail(const_cast<pot3d_server *>(sv), POT3D_EINVAL, "server and out are required");
    out->replays = sv->replays;
    out->finished = sv->finished;
    int active = 0;
    for (const Slot &sl : sv->slots) active += sl.active ? 1 : 0;
    out->active = active;
    out->queued = (int)sv->queue.size();
    out->cached_contexts = (int)sv->idle.size();
    out->max_slots = sv->max_slots;
    out->graph_iters = sv->sweep ? 2 * sv->graph_m : sv->graph_m;   // sweeps replay 2m iterations
    out->used_bytes = (double)sv->used;
    out->budget_bytes = (double)sv->budget;
    return POT3D_OK;
}

void pot3d_server_destroy(pot3d_server *sv)
{
    if (!sv) return;
    DeviceGuard guard(sv->device);
    if (sv->stream) (void)hipStreamSynchronize(sv->stream);
    for (Slot &sl : sv->slots)
        if (sl.ctx) free_ctx(sl.ctx);
    for (pot3d_ctx *c : sv->idle) free_ctx(c);
    for (auto &g : sv->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    void *bufs[] = {sv->d_p64[0], sv->d_p64[1], sv->d_r64[0], sv->d_r64[1], sv->d_p32[0], sv->d_p32[1],
                    sv->d_r32[0], sv->d_r32[1], sv->d_s64[0], sv->d_s64[1], sv->d_s32[0], sv->d_s32[1],
                    sv->d_finp, sv->d_finr};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    if (sv->h_status) (void)hipHostFree(sv->h_status);
    for (Replay &r : sv->replay)
        if (r.done) (void)hipEventDestroy(r.done);
    if (sv->capture_stream) (void)hipStreamDestroy(sv->capture_stream);
    if (sv->stream) (void)hipStreamDestroy(sv->stream);
    delete sv;
}

}  // extern "C"
