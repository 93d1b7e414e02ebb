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
// way (Sec. 3.1).  Inside the loop the host only polls a 128-byte status block
// once per graph.
//
// FP32-refined contexts add FP32 copies of r, p (two buffers) and a correction
// e, a second scalar block and a second graph whose kernels run in FP32 (dot
// products still accumulate in FP64).  An outer loop in FP64 recomputes
// r = b - A x, solves A e = r / ||r|| in FP32 to a looser inner tolerance, and
// adds ||r|| e to x, until the FP64 residual meets tol.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "context.hpp"

namespace pot3d {
namespace host {

thread_local std::string g_thread_error;

int fail(pot3d_ctx *ctx, int code, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    else g_thread_error = msg;
    return code;
}

constexpr double kTwoPi = 6.283185307179586476925286766559;

int env_int(const char *name, int dflt)
{
    const char *s = std::getenv(name);
    if (!s || !*s) return dflt;
    return std::atoi(s);
}


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
    if (upper_bc != POT3D_UPPER_SOURCE_SURFACE && upper_bc != POT3D_UPPER_CLOSED_WALL)
        return fail(nullptr, POT3D_EINVAL, "unknown upper_bc");
    if (precision != POT3D_FP64 && precision != POT3D_FP32_REFINED)
        return fail(nullptr, POT3D_EINVAL, "unsupported precision");
    return POT3D_OK;
}

// Separable metric tables of the volume-scaled operator (Sec. 2.2 scheme with
// the spherical metric restored).  Cell centres are face midpoints; the top
// face Phi = 0 couples through a half-cell difference onto the diagonal.
// Writes rows (nr * nt), dphi, ih (np), bfac (nt), vr (nr), vt (nt) and
// 1 / (shell volume); work holds 2 nr + 2 nt + np doubles.  Allocates nothing.
void fill_tables(int nr, int nt, int np, const double *rf, const double *tf, const double *pf, int upper_bc,
                 RowCoef *rows, double *dphi, double *ih, double *bfac, double *vr, double *vt, double *inv_volume,
                 double *work)
{
    double *rc = work, *dr = rc + nr, *tc = dr + nr, *dt = tc + nt, *pc = dt + nt;
    for (int i = 0; i < nr; ++i) { rc[i] = 0.5 * (rf[i] + rf[i + 1]); dr[i] = rf[i + 1] - rf[i]; }
    for (int j = 0; j < nt; ++j) { tc[j] = 0.5 * (tf[j] + tf[j + 1]); dt[j] = tf[j + 1] - tf[j]; }
    for (int k = 0; k < np; ++k) pc[k] = 0.5 * (pf[k] + pf[k + 1]);

    for (int i = 0; i < nr; ++i) {
        for (int j = 0; j < nt; ++j) {
            const double sj = std::sin(tc[j]);
            const double face = sj * dt[j];   // r-face area / (r^2 dphi)
            RowCoef e{};
            e.rm = (i > 0) ? face * rf[i] * rf[i] / (rc[i] - rc[i - 1]) : 0.0;
            e.rp = (i < nr - 1) ? face * rf[i + 1] * rf[i + 1] / (rc[i + 1] - rc[i]) : 0.0;
            // the top face: Phi = 0 there (source surface), or no flux (closed wall)
            const double dtop = (i == nr - 1 && upper_bc == POT3D_UPPER_SOURCE_SURFACE)
                                    ? face * rf[nr] * rf[nr] / (rf[nr] - rc[nr - 1]) : 0.0;
            // pole faces (j = 0 below, j = nt-1 above) have sin(theta) = 0: no coupling
            e.tm = (j > 0) ? dr[i] * std::sin(tf[j]) / (tc[j] - tc[j - 1]) : 0.0;
            e.tp = (j < nt - 1) ? dr[i] * std::sin(tf[j + 1]) / (tc[j + 1] - tc[j]) : 0.0;
            e.s = e.rm + e.rp + e.tm + e.tp + dtop;
            e.pq = dr[i] * dt[j] / sj;
            rows[(size_t)i * nt + j] = e;
        }
    }
    for (int k = 0; k < np; ++k) {
        dphi[k] = pf[k + 1] - pf[k];
        const double gap = (k < np - 1) ? pc[k + 1] - pc[k] : pc[0] + kTwoPi - pc[np - 1];
        ih[k] = 1.0 / gap;
    }
    for (int j = 0; j < nt; ++j) bfac[j] = std::sin(tc[j]) * dt[j] * rf[0] * rf[0];
    double sr = 0.0, st = 0.0, sp = 0.0;
    for (int i = 0; i < nr; ++i) sr += (vr[i] = rc[i] * rc[i] * dr[i]);
    for (int j = 0; j < nt; ++j) st += (vt[j] = std::sin(tc[j]) * dt[j]);
    for (int k = 0; k < np; ++k) sp += dphi[k];
    *inv_volume = 1.0 / (sr * st * sp);
}

void build_tables(pot3d_ctx *c)
{
    const int nr = c->nr, nt = c->nt, np = c->np;
    const double *rf = c->rf.data(), *tf = c->tf.data();
    std::vector<double> work((size_t)2 * nr + 2 * nt + np);
    c->rows_h.assign((size_t)nr * nt, RowCoef{});
    c->dphi_h.resize(np);
    c->ih_h.resize(np);
    c->bfac_h.resize(nt);
    c->vr_h.resize(nr);
    c->vt_h.resize(nt);
    fill_tables(nr, nt, np, rf, tf, c->pf.data(), c->upper_bc, c->rows_h.data(), c->dphi_h.data(), c->ih_h.data(),
                c->bfac_h.data(), c->vr_h.data(), c->vt_h.data(), &c->inv_volume, work.data());
    const double *rc = work.data(), *tc = rc + 2 * nr;
    // field output: inverse centre spacings of the r- and theta-faces (0 where
    // the face carries the boundary value or no field), 1 / r_i, 1 / sin(theta_j)
    c->ftab_h.assign((size_t)(nr + 1) + (nt + 1) + nr + nt, 0.0);
    double *fr = c->ftab_h.data(), *ft = fr + nr + 1, *rinv = ft + nt + 1, *sinv = rinv + nr;
    for (int i = 1; i < nr; ++i) fr[i] = 1.0 / (rc[i] - rc[i - 1]);
    fr[nr] = c->upper_bc == POT3D_UPPER_SOURCE_SURFACE ? 1.0 / (rf[nr] - rc[nr - 1]) : 0.0;
    for (int j = 1; j < nt; ++j) ft[j] = 1.0 / (tc[j] - tc[j - 1]);
    for (int i = 0; i < nr; ++i) rinv[i] = 1.0 / rc[i];
    for (int j = 0; j < nt; ++j) sinv[j] = 1.0 / std::sin(tc[j]);
}

// Launch shape of one stencil pass.  `tile` picks the kernel:
//   8/16/32 = workgroup tiles of that many polar rows x 64 cells (LDS plane);
//   102/104/108 = wavefront tiles of 2/4/8 rows x 128 cells.
// Radial chunks are sized so that one launch has about `target` workgroups.
GridArgs make_grid(const pot3d_ctx *c, int tile, int target, int ci_fixed)
{
    const int rows = tile_rows(tile), cols = tile_cols(tile);
    const int ntj = (c->nt + rows - 1) / rows;
    const int ntk = (c->np + cols - 1) / cols;
    const long long tiles = (long long)ntj * ntk;
    // a wave tile is one wavefront; a workgroup holds four
    const long long per_block = tile_is_wave(tile) ? kWaves : 1;
    int ci = ci_fixed > 0 ? ci_fixed : env_int("POT3D_CI", 0);
    if (ci <= 0) {
        // as many radial chunks as keep the launch within `target` workgroups
        long long want = ((long long)target * per_block) / tiles;
        want = std::max<long long>(1, std::min<long long>(want, c->nr));
        ci = (int)((c->nr + want - 1) / want);
    }
    ci = std::max(1, std::min(ci, c->nr));
    GridArgs g{};
    g.nr = c->nr;
    g.nt = c->nt;
    g.np = c->np;
    g.pitch = c->pitch;
    g.plane = (long long)c->nt * c->pitch;
    g.ci = ci;
    g.nchunk = (c->nr + ci - 1) / ci;
    g.ntj = ntj;
    g.ntk = ntk;
    g.nblocks = (int)((tiles * g.nchunk + per_block - 1) / per_block);
    g.npad = c->npad;
    return g;
}

// Launch shape of the one-sweep kernel (`rows` box rows per wavefront):
// tiles of tj x tk interior cells (tj <= 4 rows - 4; tk = 48 cells by
// default, a multiple of 16 so that a tile's stores cover whole 128-byte
// lines) over radial chunks of ci layers.  Every workgroup walks its chunk
// from start to end, so the launch runs fastest as a single wave of
// workgroups that fills as many of the `target` resident slots as possible:
// the rule takes the tile height (FP64: down to 4 rows below the maximum;
// FP32: the maximum) and the chunk count (chunks of at least 16 layers) with
// the most workgroups up to `target`, preferring taller tiles.  Measured at
// 151 x 301 x 601: FP64 (768 slots), 11-row tiles in 2 chunks, 728
// workgroups, 299 us per sweep against 314 us for 12-row tiles (676
// workgroups) and 348 us for 11-row tiles in 3 chunks (1092); FP32 (1280
// slots, which hide latency better, so the ring of shorter tiles costs more
// than empty slots), 12-row tiles in 3 chunks, 1014 workgroups, 182 us
// against 194 us for 10-row tiles (1209).  A grid with more tiles than slots
// takes the tallest tiles and whole-radius chunks.  POT3D_SWEEP_TJ,
// POT3D_SWEEP_TK and POT3D_SWEEP_CI override.
GridArgs make_sweep_grid(const pot3d_ctx *c, int rows, int target)
{
    const int tjmax = 4 * rows - 4;
    const int tk = std::max(1, std::min(60, env_int("POT3D_SWEEP_TK", 48)));
    const int ntk = (c->np + tk - 1) / tk;
    const int tj_env = std::min(tjmax, env_int("POT3D_SWEEP_TJ", 0));
    const int ci_env = env_int("POT3D_SWEEP_CI", 0);
    int tj = tj_env > 0 ? tj_env : tjmax;
    int ci = ci_env > 0 ? ci_env : c->nr;
    if (tj_env <= 0 || ci_env <= 0) {
        long long best = 0;
        const int min_ci = std::min(c->nr, 16);
        const int lowest = c->precision == POT3D_FP32_REFINED ? tjmax : std::max(1, tjmax - 4);
        for (int t = tjmax; t >= lowest; --t) {
            if (tj_env > 0 && t != tj_env) continue;
            const long long tiles = (long long)((c->nt + t - 1) / t) * ntk;
            for (int nch = 1; nch <= c->nr; ++nch) {
                const int cc = ci_env > 0 ? ci_env : (c->nr + nch - 1) / nch;
                if (cc < min_ci && ci_env <= 0) break;
                const long long blocks = tiles * ((c->nr + cc - 1) / cc);
                if (blocks > target) break;
                if (blocks > best) {
                    best = blocks;
                    tj = t;
                    ci = cc;
                }
                if (ci_env > 0) break;
            }
        }
    }
    tj = std::max(1, std::min(tj, c->nt));
    ci = std::max(1, std::min(ci, c->nr));
    const int ntj = (c->nt + tj - 1) / tj;   // every tile starts inside the grid
    GridArgs g{};
    g.nr = c->nr;
    g.nt = c->nt;
    g.np = c->np;
    g.pitch = c->pitch;
    g.plane = (long long)c->nt * c->pitch;
    g.ci = ci;
    g.nchunk = (c->nr + ci - 1) / ci;
    g.ntj = ntj;
    g.ntk = ntk;
    g.tj = tj;
    g.tk = tk;
    g.nblocks = (int)((long long)ntj * ntk * g.nchunk);
    g.npad = c->npad;
    return g;
}

int valid_tile(int tile, int dflt)
{
    switch (tile) {
    case kTileMarch8: case kTileMarch16: case kTileMarch32: case kTileWave2: case kTileWave4: case kTileWave8:
        return tile;
    default:
        return dflt;
    }
}

// Workgroups that fit on the whole device at once for one kernel (for the
// precision the context iterates in).  A launch sized to this runs as a single
// wave of workgroups with no tail.
int resident_blocks(const pot3d_ctx *c, int mode, int tile)
{
    const int per_cu = (c->precision == POT3D_FP32_REFINED) ? stencil_blocks_per_cu<float>(mode, tile)
                                                            : stencil_blocks_per_cu<double>(mode, tile);
    return std::max(1, per_cu) * std::max(1, c->num_cu);
}

// Default shapes (measured on MI355X at 151 x 301 x 601).  The p update runs
// on 16-row LDS-plane tiles (it reads r and p_old over a halo ring, and a
// taller tile reads fewer halo rows per cell), about 3 workgroups per CU in
// long radial chunks: fewer, longer chunks repeat fewer boundary layers, and
// a launch that fits the resident slots runs as one wave of workgroups with
// no tail.  The FP64 r/x update, whose x update comes once per pair of
// iterations, runs on the four-row wavefront kernel with about 4096
// workgroups: two-pass solve 1.906 s against 2.025 s on 8-row LDS-plane
// tiles, phi-line solve 0.966 s against 0.998 s.
// FP32 passes move half the bytes per cell, so a workgroup keeps fewer bytes
// in flight and more are needed: the p update about 6 per CU, the r/x update
// on the two-row wavefront kernel with about 4096 workgroups.  (The 8-row
// LDS-plane FP32 r/x update is as fast in a single solve, but ran 18 % slower
// in the batched launches of the server; the wavefront kernel 3 %.)  The
// 16-row p update took the FP64 two-pass iteration, with x in every r/x
// update, from 368 us on 8-row tiles for both passes to 346 us.
// POT3D_TILE[_P|_R] and POT3D_TARGET_BLOCKS[_P|_R] override.
void default_tiles(int precision, int *tile_p, int *tile_r)
{
    const int all = valid_tile(env_int("POT3D_TILE", 0), 0);
    const int dflt_p = kTileMarch16;
    const int dflt_r = precision == POT3D_FP32_REFINED ? kTileWave2 : kTileWave4;
    *tile_p = valid_tile(env_int("POT3D_TILE_P", all ? all : dflt_p), dflt_p);
    *tile_r = valid_tile(env_int("POT3D_TILE_R", all ? all : dflt_r), dflt_r);
}

// Grids whose vectors stream from HBM (FP64 vectors of at least 512 MiB, so
// the four of an iteration are 8x the 256 MB memory-side cache) run both
// passes on the two-row wavefront kernel in 16-layer chunks: many short
// workgroups that sweep the grid.  Measured at 301 x 641 x 1281: FP64 3.72 ms
// per iteration against 4.14 ms with whole-radius chunks of the LDS-plane
// kernel, FP32 1.89 ms against 2.10 ms.  Smaller grids get much of their
// traffic from that cache, where long chunks in the LDS-plane kernel win.
// Serving contexts keep the server's shapes.
bool streams_from_hbm(const pot3d_ctx *c)
{
    return (double)c->npad * sizeof(double) >= 512.0 * 1024 * 1024;
}

// The one-sweep kernel addresses a vector with 32-bit byte offsets; it runs
// the iterations of single solves (FP64, or the FP32 inner iterations of the
// refined mode) and of the server's one-sweep batches.
bool sweep_capable(const pot3d_ctx *c)
{
    const double vb = c->precision == POT3D_FP32_REFINED ? sizeof(float) : sizeof(double);
    return (double)c->npad * vb < 4294967296.0;
}

// Single solves iterate in one sweep unless set otherwise.
bool one_sweep(const pot3d_ctx *c)
{
    return (c->precision == POT3D_FP32_REFINED ? c->graph32s != nullptr : c->graph_s != nullptr) &&
           c->iteration == POT3D_ITER_ONE_SWEEP;
}

void choose_launch(pot3d_ctx *c)
{
    const bool fp32 = c->precision == POT3D_FP32_REFINED;
    const int all = valid_tile(env_int("POT3D_TILE", 0), 0);
    default_tiles(c->precision, &c->tile_p, &c->tile_r);
    const bool env_tiles = all || env_int("POT3D_TILE_P", 0) || env_int("POT3D_TILE_R", 0);
    const bool hbm_shape = !c->serving && !env_tiles && streams_from_hbm(c);
    if (hbm_shape) c->tile_p = c->tile_r = kTileWave2;
    c->tile_o = all ? all : kTileWave2;
    const int tb = env_int("POT3D_TARGET_BLOCKS", 0);
    const int tp = env_int("POT3D_TARGET_BLOCKS_P", tb), tr = env_int("POT3D_TARGET_BLOCKS_R", tb);
    auto dflt_target = [&](int mode, int tile) {
        if (tile_is_wave(tile)) return 4096;
        return std::min(resident_blocks(c, mode, tile), (fp32 ? 6 : 3) * c->num_cu);
    };
    const int hbm_ci = (hbm_shape && env_int("POT3D_CI", 0) <= 0 && tb <= 0) ? 16 : 0;
    c->grid_p = make_grid(c, c->tile_p, tp > 0 ? tp : dflt_target(kUpdateP, c->tile_p), tp > 0 ? 0 : hbm_ci);
    c->grid_r = make_grid(c, c->tile_r, tr > 0 ? tr : dflt_target(kUpdateR, c->tile_r), tr > 0 ? 0 : hbm_ci);
    c->grid_o = make_grid(c, c->tile_o, tb > 0 ? tb : 2048, 0);
    // The r/x update walks the tiles in the opposite order to the p update, so
    // each pass starts on the tiles the previous pass touched last, while their
    // lines may still sit in the 256 MB memory-side cache.
    c->grid_p.reverse = env_int("POT3D_REVERSE_P", 0) != 0;
    c->grid_r.reverse = env_int("POT3D_REVERSE_R", 1) != 0;
    c->max_blocks = std::max(c->grid_p.nblocks, std::max(c->grid_r.nblocks, c->grid_o.nblocks));
    if (sweep_capable(c)) {
        // one-sweep kernel: about one resident set of workgroups
        const int rows = env_int("POT3D_SWEEP_ROWS", 4);
        c->sweep_rows = valid_sweep_rows(rows) ? rows : 4;
        const int ts = env_int("POT3D_TARGET_BLOCKS_S", 0);
        const int per_cu = fp32 ? sweep_blocks_per_cu<float>(c->sweep_rows) : sweep_blocks_per_cu<double>(c->sweep_rows);
        const int resident = std::max(1, per_cu) * std::max(1, c->num_cu);
        c->grid_s = make_sweep_grid(c, c->sweep_rows, ts > 0 ? ts : resident);
        c->grid_s.reverse = env_int("POT3D_REVERSE_S", 0) != 0;
        c->max_blocks = std::max(c->max_blocks, c->grid_s.nblocks);
    }
}

void fill_shape(const pot3d_ctx *c, pot3d_stats &st)
{
    st.tile_p = c->tile_p;
    st.tile_r = c->tile_r;
    st.chunk_p = c->grid_p.ci;
    st.chunk_r = c->grid_r.ci;
    st.blocks_p = c->grid_p.nblocks;
    st.blocks_r = c->grid_r.nblocks;
    st.iteration = one_sweep(c) ? POT3D_ITER_ONE_SWEEP : POT3D_ITER_TWO_PASS;
    st.sweep_rows = c->sweep_rows;
    st.chunk_s = c->grid_s.ci;
    st.blocks_s = c->grid_s.nblocks;
    st.precond = c->precond;
    st.blocks_l = c->precond == POT3D_PC_PHI_LINE ? c->line_blocks : 0;
    if (c->precond == POT3D_PC_PHI_LINE) st.iteration = POT3D_ITER_TWO_PASS;
}

void set_tables(pot3d_ctx *c)
{
    for (GridArgs *g : {&c->grid_p, &c->grid_r, &c->grid_o, &c->grid_s}) {
        g->rows = c->rows;
        g->dphi = c->dphi;
        g->ih = c->ih;
    }
}

StencilVecs<double> base_vecs(pot3d_ctx *c)
{
    StencilVecs<double> v{};
    v.sc = c->sc;
    v.partial = c->partial;
    return v;
}

// Capture m PCG iterations (update-p, alpha, update-r, beta/convergence) on the
// idle context stream.  V is the vector type; the scalars stay FP64.
template <typename V>
int capture_iterations(pot3d_ctx *c, V *r, V *p0, V *p1, V *x, DevScalars *sc, hipGraphExec_t *out)
{
    hipStream_t s = c->stream;
    HIP_TRY(c, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    V *pb[2] = {p0, p1};
    for (int it = 0; it < c->graph_m && e == hipSuccess; ++it) {
        StencilVecs<V> a{};
        a.sc = sc;
        a.partial = c->partial;
        a.in = r;
        a.pold = pb[it & 1];
        a.pnew = pb[(it + 1) & 1];
        e = launch_stencil<V>(kUpdateP, c->tile_p, c->grid_p, a, s);
        if (e == hipSuccess) e = launch_finish(kFinSigma, sc, c->partial, c->grid_p.nblocks, s);
        if (e == hipSuccess) {
            StencilVecs<V> bv{};
            bv.sc = sc;
            bv.partial = c->partial;
            bv.in = pb[(it + 1) & 1];
            bv.pold = pb[it & 1];   // p_{k-1}, for the odd r/x update of a pair
            bv.r = r;
            bv.x = x;
            e = launch_stencil<V>(update_r_mode(it, c->graph_m), c->tile_r, c->grid_r, bv, s);
        }
        if (e == hipSuccess) e = launch_finish(kFinRho, sc, c->partial, c->grid_r.nblocks, s);
    }
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(s, &graph);
    if (e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(c, POT3D_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    }
    if (e2 != hipSuccess) return fail(c, POT3D_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e2));
    hipError_t e3 = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e3 != hipSuccess) return fail(c, POT3D_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e3));
    return POT3D_OK;
}

// x update of the one-sweep iteration for sweep `it` of a graph (even count,
// starting at an even sweep): once per pair of sweeps by default,
// POT3D_SWEEP_X=1 for every sweep.
int sweep_xmode(int it)
{
    if (env_int("POT3D_SWEEP_X", 2) == 1) return 0;
    return (it & 1) ? 2 : 1;
}

// HBM bytes per unknown per iteration of the one-sweep form: read r, p_old
// and write r, p in every sweep, read and write x in every other one
// (every one with POT3D_SWEEP_X=1).
double sweep_bytes(bool fp32)
{
    const double b = env_int("POT3D_SWEEP_X", 2) == 1 ? 48.0 : 40.0;
    return fp32 ? b / 2 : b;
}

// The two-pass form pairs its iterations the same way: the even r/x update
// leaves x alone (24 N instead of 40 N), the odd one reads p_{k-1} and adds
// both increments (48 N).  Only for an even number of captured iterations, so
// that replays continue the alternation.
int update_r_mode(int it, int m)
{
    if (env_int("POT3D_SWEEP_X", 2) == 1 || (m & 1)) return kUpdateR;
    return (it & 1) ? kUpdateRPair : kUpdateRSkip;
}

double two_pass_bytes(bool fp32, int m)
{
    const double b = update_r_mode(0, m) == kUpdateR ? 64.0 : 60.0;
    return fp32 ? b / 2 : b;
}

// Capture 2 m sweeps of the one-sweep iteration (sweep, finisher) on the
// idle context stream.  Sweep j reads r and p from buffer j mod 2 and writes
// buffer (j + 1) mod 2; 2 m is even, so replays continue the alternation,
// and of the x pairing too (an even sweep leaves x to the odd one after it).
template <typename V>
int capture_sweeps(pot3d_ctx *c, V *r0, V *r1, V *p0, V *p1, V *x, DevScalars *sc, hipGraphExec_t *out)
{
    hipStream_t s = c->stream;
    HIP_TRY(c, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    V *rb[2] = {r0, r1};
    V *pb[2] = {p0, p1};
    for (int it = 0; it < 2 * c->graph_m && e == hipSuccess; ++it) {
        SweepVecs<V> v{};
        v.r_in = rb[it & 1];
        v.r_out = rb[(it + 1) & 1];
        v.p_old = pb[it & 1];
        v.p_new = pb[(it + 1) & 1];
        v.x = x;
        v.sc = sc;
        v.partial = c->partial;
        v.xmode = sweep_xmode(it);
        e = launch_sweep<V>(c->sweep_rows, c->grid_s, v, s);
        if (e == hipSuccess) e = launch_finish(kFinSweep, sc, c->partial, c->grid_s.nblocks, s);
    }
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(s, &graph);
    if (e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(c, POT3D_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    }
    if (e2 != hipSuccess) return fail(c, POT3D_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e2));
    hipError_t e3 = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e3 != hipSuccess) return fail(c, POT3D_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e3));
    return POT3D_OK;
}

// Capture m PCG iterations with the phi-line block preconditioner: the
// direction update on z (p = z + beta p_old, A p, p.Ap), alpha, the r/x
// update, the line pass (z = M^-1 r, r.z, r.r), then beta and convergence.
// V: the vector type (FP64 solves, or the FP32 inner iterations of the
// refined mode, whose scalars and sums stay FP64).
template <typename V>
int capture_line_iterations(pot3d_ctx *c, V *r, V *p0, V *p1, V *x, V *z, DevScalars *sc, hipGraphExec_t *out)
{
    hipStream_t s = c->stream;
    HIP_TRY(c, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    V *pb[2] = {p0, p1};
    for (int it = 0; it < c->graph_m && e == hipSuccess; ++it) {
        StencilVecs<V> a{};
        a.sc = sc;
        a.partial = c->partial;
        a.in = z;
        a.pold = pb[it & 1];
        a.pnew = pb[(it + 1) & 1];
        a.zin = 1;
        e = launch_stencil<V>(kUpdateP, c->tile_p, c->grid_p, a, s);
        if (e == hipSuccess) e = launch_finish(kFinSigma, sc, c->partial, c->grid_p.nblocks, s);
        if (e == hipSuccess) {
            StencilVecs<V> bv{};
            bv.sc = sc;
            bv.partial = c->partial;
            bv.in = pb[(it + 1) & 1];
            bv.pold = pb[it & 1];   // p_{k-1}, for the odd r/x update of a pair
            bv.r = r;
            bv.x = x;
            bv.zin = 1;
            e = launch_stencil<V>(update_r_mode(it, c->graph_m), c->tile_r, c->grid_r, bv, s);
        }
        if (e == hipSuccess) e = launch_line<V>(c->grid_o, r, z, c->partial, c->line_blocks, sc, 0, s);
        if (e == hipSuccess) e = launch_finish(kFinRho, sc, c->partial, c->line_blocks, s);
    }
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(s, &graph);
    if (e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(c, POT3D_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    }
    if (e2 != hipSuccess) return fail(c, POT3D_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e2));
    hipError_t e3 = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e3 != hipSuccess) return fail(c, POT3D_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e3));
    return POT3D_OK;
}

// Replay `graph` (`per_graph` iterations each) until the scalar block `sc`
// reports done, keeping one graph queued ahead of the poll.  Returns
// POT3D_OK or a HIP error status.
int replay_until_done(pot3d_ctx *c, hipGraphExec_t graph, DevScalars *sc, hipStream_t s, int maxit, int per_graph,
                      int *launches, DevScalars *final_out)
{
    int slot = 0;
    int n = 0;
    HIP_TRY(c, hipGraphLaunch(graph, s));
    ++n;
    HIP_TRY(c, hipMemcpyAsync(&c->h_sc[slot], sc, sizeof(DevScalars), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipEventRecord(c->ev_poll[slot], s));
    const long long max_launches = ((long long)maxit + 1) / per_graph + 3;
    for (;;) {
        const int nxt = slot ^ 1;
        HIP_TRY(c, hipGraphLaunch(graph, s));
        ++n;
        HIP_TRY(c, hipMemcpyAsync(&c->h_sc[nxt], sc, sizeof(DevScalars), hipMemcpyDeviceToHost, s));
        HIP_TRY(c, hipEventRecord(c->ev_poll[nxt], s));
        HIP_TRY(c, hipEventSynchronize(c->ev_poll[slot]));
        if (c->h_sc[slot].done || n > max_launches) break;
        slot = nxt;
    }
    HIP_TRY(c, hipStreamSynchronize(s));
    HIP_TRY(c, hipMemcpy(final_out, sc, sizeof(DevScalars), hipMemcpyDeviceToHost));
    *launches += n;
    if (!final_out->done) return fail(c, POT3D_EDEVICE, "iteration loop ended without the device done flag");
    return POT3D_OK;
}

void free_ctx(pot3d_ctx *c)
{
    if (!c) return;
    DeviceGuard guard(c->device);
    if (c->graph) (void)hipGraphExecDestroy(c->graph);
    if (c->graph32) (void)hipGraphExecDestroy(c->graph32);
    if (c->graph_s) (void)hipGraphExecDestroy(c->graph_s);
    if (c->graph_l) (void)hipGraphExecDestroy(c->graph_l);
    if (c->graph32l) (void)hipGraphExecDestroy(c->graph32l);
    if (c->graph32s) (void)hipGraphExecDestroy(c->graph32s);
    for (hipEvent_t *e : {&c->ev_poll[0], &c->ev_poll[1], &c->ev_t0, &c->ev_t1, &c->ev_loop0, &c->ev_loop1})
        if (*e) (void)hipEventDestroy(*e);
    if (c->stream) (void)hipStreamDestroy(c->stream);
    void *bufs[] = {c->rows, c->dphi, c->ih, c->bfac, c->x, c->r, c->r2, c->p[0], c->p[1],
                    c->bplane, c->br, c->partial, c->poles, c->vr, c->vt, c->bcs, c->ftab, c->sc,
                    c->r32, c->r32b, c->p32[0], c->p32[1], c->e32, c->sc32, c->z, c->z32};
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

// b from Br and the starting x (phi0, or zero).
int prepare_solve(pot3d_ctx *c, const double *br_dev, const double *phi0, hipMemcpyKind kind_in, hipStream_t s)
{
    const size_t rowb = (size_t)c->np * sizeof(double), pitchb = (size_t)c->pitch * sizeof(double);
    const size_t nrows = (size_t)c->nr * c->nt;
    c->have_solution = false;
    c->field_ready = false;
    const bool closed = c->upper_bc == POT3D_UPPER_CLOSED_WALL;
    if (closed) HIP_TRY(c, launch_monopole(br_dev, c->bfac, c->dphi, c->nt, c->np, c->bcs, s));
    HIP_TRY(c, launch_rhs(br_dev, c->bfac, c->dphi, c->nt, c->np, c->pitch, closed ? c->bcs : nullptr, c->bplane, s));
    if (phi0 && kind_in == hipMemcpyHostToDevice && c->pitch != c->np) {
        // one contiguous host copy into r (free until the solve starts), then
        // the padded layout on the device
        HIP_TRY(c, hipMemcpyAsync(c->r, phi0, (size_t)c->n * sizeof(double), kind_in, s));
        HIP_TRY(c, launch_repack(c->r, c->x, (long long)nrows, c->np, c->pitch, false, s));
    } else if (phi0) {
        HIP_TRY(c, copy_rows(c->x, pitchb, phi0, rowb, rowb, nrows, kind_in, s));
    }
    else HIP_TRY(c, launch_fill<double>(c->x, c->npad, 0.0, s));
    return POT3D_OK;
}

// FP64 start: scalars, p_old = 0, r = b - A x0 and the first residual test.
int start_fp64(pot3d_ctx *c, hipStream_t s, double tol, int maxit)
{
    DevScalars init{};
    init.tol = tol;
    init.maxit = maxit;
    c->h_sc[0] = init;
    HIP_TRY(c, hipMemcpyAsync(c->sc, &c->h_sc[0], sizeof(DevScalars), hipMemcpyHostToDevice, s));
    HIP_TRY(c, launch_fill<double>(c->p[0], c->npad, 0.0, s));
    StencilVecs<double> rv = base_vecs(c);
    rv.in = c->x;
    rv.r = c->r;
    rv.bplane = c->bplane;
    rv.store_r = 1;
    rv.ignore_done = 1;
    HIP_TRY(c, launch_stencil<double>(kResidual, c->tile_o, c->grid_o, rv, s));
    HIP_TRY(c, launch_finish(kFinInit, c->sc, c->partial, c->grid_o.nblocks, s));
    if (c->precond == POT3D_PC_PHI_LINE) {
        // z = M^-1 r of the starting residual and rho = r.z (the first
        // direction update then forms p = z)
        HIP_TRY(c, launch_line<double>(c->grid_o, c->r, c->z, c->partial, c->line_blocks, c->sc, 1, s));
        HIP_TRY(c, launch_finish(kFinLineInit, c->sc, c->partial, c->line_blocks, s));
    }
    return POT3D_OK;
}

// FP64 PCG: start, then graph replays (one-sweep, two-pass, or with the
// phi-line preconditioner) until done.
int run_fp64(pot3d_ctx *c, double *phi_out, hipMemcpyKind kind_out, hipStream_t s, double tol, int maxit, int *iters,
             double *relres_true)
{
    int rc = start_fp64(c, s, tol, maxit);
    if (rc != POT3D_OK) return rc;
    HIP_TRY(c, hipEventRecord(c->ev_loop0, s));
    int launches = 0;
    DevScalars fin{};
    const bool line = c->precond == POT3D_PC_PHI_LINE;
    const bool sweep = !line && one_sweep(c);
    hipGraphExec_t graph = line ? c->graph_l : (sweep ? c->graph_s : c->graph);
    rc = replay_until_done(c, graph, c->sc, s, maxit, sweep ? 2 * c->graph_m : c->graph_m, &launches, &fin);
    if (rc != POT3D_OK) return rc;
    // the increment of x the last sweep or r/x update may have left to a next one
    HIP_TRY(c, launch_x_catchup<double>(c->x, c->sc, c->nr, c->nt, c->np, c->pitch, s));
    HIP_TRY(c, hipEventRecord(c->ev_loop1, s));
    return finish_solve(c, phi_out, kind_out, s, fin, launches, fin.k, 1, line ? two_pass_bytes(false, c->graph_m) + 16.0 : (sweep ? sweep_bytes(false) : two_pass_bytes(false, c->graph_m)), iters,
                        relres_true);
}

// Refinement, outer step: r = b - A x in FP64, then the outer test.  The
// scalar block must already hold tol (set once per solve).  Waits for the
// result and returns it in *out.
int refined_outer_check(pot3d_ctx *c, hipStream_t s, DevScalars *out)
{
    StencilVecs<double> rv = base_vecs(c);
    rv.in = c->x;
    rv.r = c->r;
    rv.bplane = c->bplane;
    rv.store_r = 1;
    rv.ignore_done = 1;
    HIP_TRY(c, launch_stencil<double>(kResidual, c->tile_o, c->grid_o, rv, s));
    HIP_TRY(c, launch_finish(kFinOuter, c->sc, c->partial, c->grid_o.nblocks, s));
    HIP_TRY(c, hipMemcpyAsync(&c->h_sc[0], c->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    *out = c->h_sc[0];
    return POT3D_OK;
}

// Refinement, inner start.  The FP32 residual becomes r / ||r|| (the true
// residual just computed in FP64) and the correction e restarts from zero.
// Restart mode: p = 0, a fresh PCG.  Reliable-update mode, after a segment that
// converged: the last search direction is kept, rescaled to the new
// normalisation, and beta continues from the previous r.z, so the Krylov
// process is not thrown away (residual replacement as in the reliable-update
// CG of Sleijpen and van der Vorst).  An inner segment goes no further than the
// outer target needs: a reduction of tol / relres (with a factor 2 margin)
// already meets it.  prev: the scalars of the segment just finished (NULL
// before the first); scale_prev: the normalisation it ran in.
// The inner tolerance: as set, or the measured default of the mode (reliable
// updates every factor 10 of residual reduction; restarts every 1e-4).  Longer
// stretches between replacements let the FP32 recursion drift: at
// 151 x 301 x 601 a reliable update every 1e-3 took 34x the iterations.
double inner_tolerance(const pot3d_ctx *c)
{
    if (c->inner_tol > 0.0) return c->inner_tol;
    return c->refine_mode == POT3D_REFINE_RELIABLE ? 0.1 : 1e-4;
}

int refined_start_inner(pot3d_ctx *c, hipStream_t s, double tol, int maxit_left, const DevScalars &outer,
                        const DevScalars *prev, double scale_prev)
{
    const int nb_dots = std::max(1, std::min(c->max_blocks, c->nr * c->nt));
    const bool resume = c->refine_mode == POT3D_REFINE_RELIABLE && prev && prev->done && prev->status == POT3D_OK &&
                        prev->k > 0 &&
                        std::isfinite(prev->rho) && prev->rho > 0.0 && scale_prev > 0.0 &&
                        std::isfinite(outer.scale) && outer.scale > 0.0;
    DevScalars in{};
    in.tol = std::max(inner_tolerance(c), 0.5 * tol / outer.relres);
    in.maxit = maxit_left;
    if (resume) {
        // A continued segment that runs far longer than the one before it has
        // lost the recurrence (FP32 drift between replacements): cap it, and
        // a capped segment (status ENOCONV) makes the next one a restart.
        in.maxit = (int)std::min<long long>(maxit_left, 2LL * prev->k + 64);
        const double f = outer.scale / scale_prev;   // new units per old unit
        HIP_TRY(c, launch_resume_residual(c->r, c->r32, c->e32, c->p32[prev->k & 1], c->p32[0], c->npad, c->sc,
                                          (float)f, s));
        in.scale = 1.0 / (f * f * prev->rho);   // 1 / rho_prev in the new units
    } else {
        HIP_TRY(c, launch_cast_residual(c->r, c->r32, c->e32, c->p32[0], c->npad, c->sc, s));
    }
    c->h_sc[1] = in;
    HIP_TRY(c, hipMemcpyAsync(c->sc32, &c->h_sc[1], sizeof(DevScalars), hipMemcpyHostToDevice, s));
    if (c->precond == POT3D_PC_PHI_LINE) {
        // z = M^-1 r of the new FP32 residual, with r.z and r.r
        HIP_TRY(c, launch_line<float>(c->grid_o, c->r32, c->z32, c->partial, c->line_blocks, c->sc32, 1, s));
        HIP_TRY(c, launch_finish(resume ? kFinResume : kFinInner, c->sc32, c->partial, c->line_blocks, s));
        return POT3D_OK;
    }
    HIP_TRY(c, launch_dots_rz(c->grid_o, c->r32, c->partial, nb_dots, s));
    HIP_TRY(c, launch_finish(resume ? kFinResume : kFinInner, c->sc32, c->partial, nb_dots, s));
    return POT3D_OK;
}

int refined_correct(pot3d_ctx *c, hipStream_t s)
{
    HIP_TRY(c, launch_add_correction(c->x, c->e32, c->npad, c->sc, s));
    return POT3D_OK;
}

// FP32-refined: outer FP64 defect correction around FP32 Jacobi-PCG solves.
//   repeat: r = b - A x (FP64); stop if ||r||/||b|| <= tol
//           solve A e = r / ||r|| with FP32 PCG (FP64 dots) to inner_tol
//           x += ||r|| e (FP64)
// maxit caps the total number of inner iterations.
int run_refined(pot3d_ctx *c, double *phi_out, hipMemcpyKind kind_out, hipStream_t s, double tol, int maxit,
                int *iters, double *relres_true)
{
    DevScalars init{};
    init.tol = tol;
    init.maxit = maxit;
    c->h_sc[0] = init;
    HIP_TRY(c, hipMemcpyAsync(c->sc, &c->h_sc[0], sizeof(DevScalars), hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipEventRecord(c->ev_loop0, s));
    int launches = 0, total = 0, outer = 0;
    DevScalars out{}, inner{};
    double scale_prev = 0.0;
    for (;;) {
        int rc = refined_outer_check(c, s, &out);
        if (rc != POT3D_OK) return rc;
        if (out.done) break;
        if (outer >= c->max_outer || total >= maxit) {
            out.status = POT3D_ENOCONV;
            break;
        }
        rc = refined_start_inner(c, s, tol, maxit - total, out, outer > 0 ? &inner : nullptr, scale_prev);
        if (rc != POT3D_OK) return rc;
        scale_prev = out.scale;
        const bool line = c->precond == POT3D_PC_PHI_LINE;
        const bool sweep = !line && one_sweep(c);
        rc = replay_until_done(c, line ? c->graph32l : (sweep ? c->graph32s : c->graph32), c->sc32, s, maxit - total,
                               sweep ? 2 * c->graph_m : c->graph_m, &launches, &inner);
        if (rc != POT3D_OK) return rc;
        HIP_TRY(c, launch_x_catchup<float>(c->e32, c->sc32, c->nr, c->nt, c->np, c->pitch, s));
        total += inner.k;
        ++outer;
        if (inner.status == POT3D_EBREAKDOWN) {
            out.status = POT3D_EBREAKDOWN;
            break;
        }
        rc = refined_correct(c, s);
        if (rc != POT3D_OK) return rc;
    }
    HIP_TRY(c, hipEventRecord(c->ev_loop1, s));
    const double per = c->precond == POT3D_PC_PHI_LINE ? two_pass_bytes(true, c->graph_m) + 8.0
                                                       : (one_sweep(c) ? sweep_bytes(true) : two_pass_bytes(true, c->graph_m));
    return finish_solve(c, phi_out, kind_out, s, out, launches, total, outer, per, iters, relres_true);
}

// The solve proper.  br_dev: device Br (nt*np); phi0: initial guess or NULL
// (host or device per `kind_in`); phi_out: destination (host or device).
int run_solve(pot3d_ctx *c, const double *br_dev, const double *phi0, hipMemcpyKind kind_in, double *phi_out,
              hipMemcpyKind kind_out, hipStream_t s, double tol, int maxit, int *iters, double *relres_true)
{
    HIP_TRY(c, hipEventRecord(c->ev_t0, s));
    int rc = prepare_solve(c, br_dev, phi0, kind_in, s);
    if (rc != POT3D_OK) return rc;
    if (c->precision == POT3D_FP32_REFINED) return run_refined(c, phi_out, kind_out, s, tol, maxit, iters, relres_true);
    return run_fp64(c, phi_out, kind_out, s, tol, maxit, iters, relres_true);
}

// Common tail: true residual (FP64), pole values, Phi out, statistics.
int finish_solve(pot3d_ctx *c, double *phi_out, hipMemcpyKind kind_out, hipStream_t s, DevScalars fin, int launches,
                 int total_iters, int outer, double bytes_per_unknown, int *iters, double *relres_true)
{
    const size_t rowb = (size_t)c->np * sizeof(double), pitchb = (size_t)c->pitch * sizeof(double);
    const size_t nrows = (size_t)c->nr * c->nt;
    StencilVecs<double> tv = base_vecs(c);
    tv.in = c->x;
    tv.bplane = c->bplane;
    tv.store_r = 0;
    tv.ignore_done = 1;
    if (fin.zero_solution) HIP_TRY(c, launch_fill<double>(c->x, c->npad, 0.0, s));
    else if (c->upper_bc == POT3D_UPPER_CLOSED_WALL)
        HIP_TRY(c, launch_gauge(c->x, c->vr, c->vt, c->dphi, c->nr, c->nt, c->np, c->pitch, c->inv_volume, c->partial,
                                c->max_blocks, c->bcs + 2, s));
    HIP_TRY(c, launch_stencil<double>(kResidual, c->tile_o, c->grid_o, tv, s));
    HIP_TRY(c, launch_finish(kFinTrue, c->sc, c->partial, c->grid_o.nblocks, s));
    HIP_TRY(c, launch_poles(c->x, c->dphi, c->nr, c->nt, c->np, c->pitch, kTwoPi, c->poles, s));
    if (kind_out == hipMemcpyDeviceToHost && c->pitch != c->np) {
        // packed on the device into r (no longer needed), then one contiguous copy
        HIP_TRY(c, launch_repack(c->x, c->r, (long long)nrows, c->np, c->pitch, true, s));
        HIP_TRY(c, hipMemcpyAsync(phi_out, c->r, (size_t)c->n * sizeof(double), kind_out, s));
    } else {
        HIP_TRY(c, copy_rows(phi_out, rowb, c->x, pitchb, rowb, nrows, kind_out, s));
    }
    HIP_TRY(c, hipMemcpyAsync(&c->h_sc[0], c->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipEventRecord(c->ev_t1, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    const double true_rel = c->h_sc[0].relres_true;

    float ms_total = 0.f, ms_loop = 0.f;
    (void)hipEventElapsedTime(&ms_total, c->ev_t0, c->ev_t1);
    (void)hipEventElapsedTime(&ms_loop, c->ev_loop0, c->ev_loop1);
    pot3d_stats &st = c->stats;
    st.iters = total_iters;
    st.outer = outer;
    st.status = fin.status;
    st.graph_launches = launches;
    st.relres = fin.relres;
    st.relres_true = fin.zero_solution ? 0.0 : true_rel;
    st.solve_ms = ms_total;
    st.loop_ms = ms_loop;
    st.bytes_per_iter = bytes_per_unknown * (double)c->n;
    st.n = c->n;
    st.pitch = c->pitch;
    fill_shape(c, st);
    if (const unsigned line = take_oob_line(s))
        return fail(c, POT3D_EDEVICE, "checked build: out-of-range index at kernels.hip line " + std::to_string(line));
    c->have_solution = true;
    c->field_ready = true;
    if (iters) *iters = total_iters;
    if (relres_true) *relres_true = st.relres_true;
    if (fin.status == POT3D_EBREAKDOWN) return fail(c, POT3D_EBREAKDOWN, "breakdown: non-finite data or p.Ap <= 0");
    if (fin.status == POT3D_ENOCONV) return fail(c, POT3D_ENOCONV, "iteration cap reached before tol");
    return fin.status;
}

// Average duration of the two iteration kernels as they run in a solve: a
// graph of `reps` iterations in the solve's order (p update, alpha, r/x
// update, beta), replayed twice back to back (warm-up, then timed).  In this
// graph each stencil launch records, on the device wall clock, its first
// workgroup's start and its last workgroup's end; host events around the
// timed replay set the clock's scale.  (Host events on single launches are no
// substitute: a launch that signals an event to the host runs longer, and the
// r/x update starts on the tiles the p update touched last, whose lines are
// then still in the memory-side cache, so it is timed in that sequence.)  The
// stencil kernels ignore the done flag.  FP64: a fixed-count PCG from x = 0
// on the context's right-hand side; FP32: fixed scalars.  Runs on (and
// overwrites) the context's vectors.
template <typename V>
int time_pair(pot3d_ctx *ctx, V *r, V *p0, V *p1, V *x, DevScalars *sc, int reps, double *ms_p, double *ms_r)
{
    hipStream_t s = ctx->stream;
    const int m = std::max(2, reps + (reps & 1));   // even: the r/x updates pair up, across the two replays too
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, ctx->device) != hipSuccess || khz <= 0)
        return fail(ctx, POT3D_EDEVICE, "device wall-clock rate unavailable");
    if constexpr (std::is_same<V, double>::value) {
        // a real fixed-count PCG from x = 0 on the context's right-hand side
        HIP_TRY(ctx, launch_fill<double>(ctx->x, ctx->npad, 0.0, s));
        const int rc = start_fp64(ctx, s, 0.0, 1 << 30);
        if (rc != POT3D_OK) return rc;
    } else {
        DevScalars st{};
        st.alpha = 1e-3;
        st.beta = 0.5;
        st.rho = 1.0;
        st.bnorm = 1.0;
        st.tol = 0.0;
        st.maxit = 1 << 30;
        ctx->h_sc[0] = st;
        HIP_TRY(ctx, hipMemcpyAsync(sc, &ctx->h_sc[0], sizeof(DevScalars), hipMemcpyHostToDevice, s));
    }
    // per iteration: p update start, end; r/x update start, end
    std::vector<unsigned long long> init(4 * (size_t)m), stamps(4 * (size_t)m);
    for (int q = 0; q < 2 * m; ++q) {
        init[2 * q] = ~0ull;
        init[2 * q + 1] = 0ull;
    }
    unsigned long long *d_ts = nullptr;
    HIP_TRY(ctx, hipMalloc(reinterpret_cast<void **>(&d_ts), init.size() * sizeof(unsigned long long)));
    V *pb[2] = {p0, p1};
    hipGraphExec_t exec = nullptr;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    for (int it = 0; it < m && e == hipSuccess; ++it) {
        StencilVecs<V> a{};
        a.sc = sc;
        a.partial = ctx->partial;
        a.in = r;
        a.pold = pb[it & 1];
        a.pnew = pb[(it + 1) & 1];
        a.ignore_done = 1;
        a.tstamp = d_ts + 4 * it;
        StencilVecs<V> bv{};
        bv.sc = sc;
        bv.partial = ctx->partial;
        bv.in = pb[(it + 1) & 1];
        bv.pold = pb[it & 1];
        bv.r = r;
        bv.x = x;
        bv.ignore_done = 1;
        bv.tstamp = d_ts + 4 * it + 2;
        e = launch_stencil<V>(kUpdateP, ctx->tile_p, ctx->grid_p, a, s);
        if (e == hipSuccess) e = launch_finish(kFinSigma, sc, ctx->partial, ctx->grid_p.nblocks, s);
        if (e == hipSuccess) e = launch_stencil<V>(update_r_mode(it, m), ctx->tile_r, ctx->grid_r, bv, s);
        if (e == hipSuccess) e = launch_finish(kFinRho, sc, ctx->partial, ctx->grid_r.nblocks, s);
    }
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(s, &graph);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    double tp = 0.0, tr = 0.0;
    const int timed = m;
    if (e == hipSuccess) e = hipGraphLaunch(exec, s);   // warm-up
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_ts, init.data(), init.size() * sizeof(unsigned long long), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(ctx->ev_t0, s);
    if (e == hipSuccess) e = hipGraphLaunch(exec, s);
    if (e == hipSuccess) e = hipEventRecord(ctx->ev_t1, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(stamps.data(), d_ts, stamps.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    // device ticks -> ms: the replay's span on the device clock (first p
    // update start to last r/x update end) against the same replay between
    // host events
    float span_ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&span_ms, ctx->ev_t0, ctx->ev_t1);
    const double span_ticks = (double)(stamps[4 * (size_t)(m - 1) + 3] - stamps[0]);
    const double ms_per_tick = (span_ticks > 0.0 && span_ms > 0.f) ? span_ms / span_ticks : 1.0 / khz;
    for (int it = 0; it < m && e == hipSuccess; ++it) {
        tp += (double)(stamps[4 * it + 1] - stamps[4 * it]) * ms_per_tick;
        tr += (double)(stamps[4 * it + 3] - stamps[4 * it + 2]) * ms_per_tick;
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    (void)hipFree(d_ts);
    if (e != hipSuccess) return fail(ctx, POT3D_EDEVICE, std::string("kernel timing: ") + hipGetErrorString(e));
    *ms_p = tp / timed;
    *ms_r = tr / timed;
    return POT3D_OK;
}

// Average duration of the one-sweep kernel as it runs in a solve: as
// time_pair, with a graph of `reps` sweeps (sweep, finisher) of a fixed-count
// FP64 PCG from x = 0 on the context's right-hand side.  ms_even, ms_odd: the
// even sweeps (x left to the next sweep) and the odd ones (x of the pair).
template <typename V>
int time_sweeps(pot3d_ctx *ctx, V *r0, V *r1, V *p0, V *p1, V *x, DevScalars *sc, int reps, double *ms_even,
                double *ms_odd)
{
    hipStream_t s = ctx->stream;
    const int m = std::max(2, reps + (reps & 1));   // even: the buffers alternate across the two replays
    if constexpr (std::is_same<V, double>::value) {
        HIP_TRY(ctx, launch_fill<double>(ctx->x, ctx->npad, 0.0, s));
        const int rc = start_fp64(ctx, s, 0.0, 1 << 30);
        if (rc != POT3D_OK) return rc;
    } else {
        // fixed scalars on whatever the FP32 vectors hold
        DevScalars st{};
        st.alpha = 1e-3;
        st.beta = 0.5;
        st.rho = 1.0;
        st.bnorm = 1.0;
        st.tol = 0.0;
        st.maxit = 1 << 30;
        ctx->h_sc[0] = st;
        HIP_TRY(ctx, hipMemcpyAsync(sc, &ctx->h_sc[0], sizeof(DevScalars), hipMemcpyHostToDevice, s));
    }
    // per sweep: start, end
    std::vector<unsigned long long> init(2 * (size_t)m), stamps(2 * (size_t)m);
    for (int q = 0; q < m; ++q) {
        init[2 * q] = ~0ull;
        init[2 * q + 1] = 0ull;
    }
    unsigned long long *d_ts = nullptr;
    HIP_TRY(ctx, hipMalloc(reinterpret_cast<void **>(&d_ts), init.size() * sizeof(unsigned long long)));
    V *rb[2] = {r0, r1};
    V *pb[2] = {p0, p1};
    hipGraphExec_t exec = nullptr;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    for (int it = 0; it < m && e == hipSuccess; ++it) {
        SweepVecs<V> v{};
        v.r_in = rb[it & 1];
        v.r_out = rb[(it + 1) & 1];
        v.p_old = pb[it & 1];
        v.p_new = pb[(it + 1) & 1];
        v.x = x;
        v.sc = sc;
        v.partial = ctx->partial;
        v.ignore_done = 1;
        v.tstamp = d_ts + 2 * it;
        v.xmode = sweep_xmode(it);
        e = launch_sweep<V>(ctx->sweep_rows, ctx->grid_s, v, s);
        if (e == hipSuccess) e = launch_finish(kFinSweep, sc, ctx->partial, ctx->grid_s.nblocks, s);
    }
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(s, &graph);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e == hipSuccess) e = hipGraphLaunch(exec, s);   // warm-up
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_ts, init.data(), init.size() * sizeof(unsigned long long), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(ctx->ev_t0, s);
    if (e == hipSuccess) e = hipGraphLaunch(exec, s);
    if (e == hipSuccess) e = hipEventRecord(ctx->ev_t1, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(stamps.data(), d_ts, stamps.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    // device ticks -> ms from the replay's span on the device clock and between host events
    float span_ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&span_ms, ctx->ev_t0, ctx->ev_t1);
    int khz = 0;
    (void)hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, ctx->device);
    const double span_ticks = (double)(stamps[2 * (size_t)(m - 1) + 1] - stamps[0]);
    const double ms_per_tick = (span_ticks > 0.0 && span_ms > 0.f) ? span_ms / span_ticks : 1.0 / std::max(1, khz);
    double t[2] = {0.0, 0.0};
    for (int it = 0; it < m && e == hipSuccess; ++it)
        t[it & 1] += (double)(stamps[2 * it + 1] - stamps[2 * it]) * ms_per_tick;
    if (exec) (void)hipGraphExecDestroy(exec);
    (void)hipFree(d_ts);
    if (e != hipSuccess) return fail(ctx, POT3D_EDEVICE, std::string("kernel timing: ") + hipGetErrorString(e));
    *ms_even = t[0] / (m / 2);
    *ms_odd = t[1] / (m / 2);
    return POT3D_OK;
}

int create_context(const double *r_faces, int nr, const double *t_faces, int nt, const double *p_faces, int np,
                   int upper_bc, int precision, int device, bool serving, pot3d_ctx **out)
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
    c->serving = serving;
    c->nr = nr;
    c->nt = nt;
    c->np = np;
    c->precision = precision;
    c->upper_bc = upper_bc;
    // rows padded to an even length at least, so two-cell (16-byte) accesses stay in the row
    int align = std::max(2, env_int("POT3D_PITCH_ALIGN", 8));
    align += align & 1;
    c->pitch = ((np + align - 1) / align) * align;
    c->n = (long long)nr * nt * np;
    c->npad = (long long)nr * nt * c->pitch;
    c->graph_m = std::max(2, env_int("POT3D_GRAPH_ITERS", 16));
    c->graph_m += c->graph_m & 1;   // even, so the p buffers alternate consistently across replays
    // Default form: one sweep, except for the FP32 inner iterations of grids
    // whose vectors stream from HBM, where the two FP32 passes in their
    // streaming shape are faster (301 x 641 x 1281: 2.08 against 2.35 ms per
    // inner iteration; 151 x 301 x 601: 201 against 197 us).
    const int it_env = env_int("POT3D_ITERATION", -1);
    if (it_env == POT3D_ITER_TWO_PASS || it_env == POT3D_ITER_ONE_SWEEP)
        c->iteration = it_env;
    else
        c->iteration = (precision == POT3D_FP32_REFINED && streams_from_hbm(c)) ? POT3D_ITER_TWO_PASS
                                                                                : POT3D_ITER_ONE_SWEEP;
    c->rf.assign(r_faces, r_faces + nr + 1);
    c->tf.assign(t_faces, t_faces + nt + 1);
    c->pf.assign(p_faces, p_faces + np + 1);
    build_tables(c);
    hipDeviceProp_t prop{};
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        c->num_cu = prop.multiProcessorCount;
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
    CREATE_TRY(dalloc(&c->partial, (size_t)kMaxPartials * c->max_blocks));
    CREATE_TRY(dalloc(&c->poles, (size_t)2 * nr));
    CREATE_TRY(dalloc(&c->vr, (size_t)nr));
    CREATE_TRY(dalloc(&c->vt, (size_t)nt));
    CREATE_TRY(dalloc(&c->bcs, 4));
    CREATE_TRY(dalloc(&c->ftab, c->ftab_h.size()));
    CREATE_TRY(dalloc(&c->sc, 1));
    CREATE_TRY(hipHostMalloc(reinterpret_cast<void **>(&c->h_sc), 2 * sizeof(DevScalars), hipHostMallocDefault));
    CREATE_TRY(hipMemcpyAsync(c->rows, c->rows_h.data(), c->rows_h.size() * sizeof(RowCoef), hipMemcpyHostToDevice, c->stream));
    CREATE_TRY(hipMemcpyAsync(c->dphi, c->dphi_h.data(), np * sizeof(double), hipMemcpyHostToDevice, c->stream));
    CREATE_TRY(hipMemcpyAsync(c->ih, c->ih_h.data(), np * sizeof(double), hipMemcpyHostToDevice, c->stream));
    CREATE_TRY(hipMemcpyAsync(c->bfac, c->bfac_h.data(), nt * sizeof(double), hipMemcpyHostToDevice, c->stream));
    CREATE_TRY(hipMemcpyAsync(c->vr, c->vr_h.data(), nr * sizeof(double), hipMemcpyHostToDevice, c->stream));
    CREATE_TRY(hipMemcpyAsync(c->vt, c->vt_h.data(), nt * sizeof(double), hipMemcpyHostToDevice, c->stream));
    CREATE_TRY(launch_fill<double>(c->bcs, 4, 0.0, c->stream));
    CREATE_TRY(hipMemcpyAsync(c->ftab, c->ftab_h.data(), c->ftab_h.size() * sizeof(double), hipMemcpyHostToDevice,
                              c->stream));
    for (double *b : {c->x, c->r, c->p[0], c->p[1]}) CREATE_TRY(launch_fill<double>(b, c->npad, 0.0, c->stream));
    CREATE_TRY(launch_fill<double>(c->bplane, (long long)nt * c->pitch, 0.0, c->stream));
    CREATE_TRY(launch_fill<double>(c->poles, 2LL * nr, 0.0, c->stream));
    CREATE_TRY(hipMemsetAsync(c->sc, 0, sizeof(DevScalars), c->stream));
    if (sweep_capable(c) && precision == POT3D_FP64) {
        CREATE_TRY(dalloc(&c->r2, (size_t)c->npad));
        CREATE_TRY(launch_fill<double>(c->r2, c->npad, 0.0, c->stream));
    }
    CREATE_TRY(hipStreamSynchronize(c->stream));
    set_tables(c);
    if (precision == POT3D_FP32_REFINED) {
        CREATE_TRY(dalloc(&c->r32, (size_t)c->npad));
        CREATE_TRY(dalloc(&c->p32[0], (size_t)c->npad));
        CREATE_TRY(dalloc(&c->p32[1], (size_t)c->npad));
        CREATE_TRY(dalloc(&c->e32, (size_t)c->npad));
        CREATE_TRY(dalloc(&c->sc32, 1));
        if (sweep_capable(c)) CREATE_TRY(dalloc(&c->r32b, (size_t)c->npad));
        for (float *b : {c->r32, c->r32b, c->p32[0], c->p32[1], c->e32})
            if (b) CREATE_TRY(launch_fill<float>(b, c->npad, 0.0f, c->stream));
        CREATE_TRY(hipMemsetAsync(c->sc32, 0, sizeof(DevScalars), c->stream));
        CREATE_TRY(hipStreamSynchronize(c->stream));
    }
#undef CREATE_TRY
    // The iteration graphs are captured once, on the idle context stream
    // (serving slots iterate inside the server's batched graph instead).
    int gc = serving ? POT3D_OK : capture_iterations<double>(c, c->r, c->p[0], c->p[1], c->x, c->sc, &c->graph);
    if (gc == POT3D_OK && c->r2 && !serving)
        gc = capture_sweeps<double>(c, c->r, c->r2, c->p[0], c->p[1], c->x, c->sc, &c->graph_s);
    if (gc == POT3D_OK && c->r32b && !serving)
        gc = capture_sweeps<float>(c, c->r32, c->r32b, c->p32[0], c->p32[1], c->e32, c->sc32, &c->graph32s);
    if (gc == POT3D_OK && precision == POT3D_FP32_REFINED && !serving)
        gc = capture_iterations<float>(c, c->r32, c->p32[0], c->p32[1], c->e32, c->sc32, &c->graph32);
    if (gc != POT3D_OK) {
        std::string m = c->err;
        free_ctx(c);
        return fail(nullptr, POT3D_EDEVICE, m);
    }
    *out = c;
    return POT3D_OK;
}

size_t context_bytes(const pot3d_ctx *c)
{
    size_t b = (size_t)c->npad * sizeof(double) * (c->r2 ? 5 : 4) + (size_t)c->nt * c->pitch * sizeof(double) +
               (size_t)c->nt * c->np * sizeof(double) + c->rows_h.size() * sizeof(RowCoef) +
               (size_t)kMaxPartials * c->max_blocks * sizeof(double) + (size_t)2 * c->nr * sizeof(double);
    if (c->precision == POT3D_FP32_REFINED) b += (size_t)c->npad * sizeof(float) * (c->r32b ? 5 : 4);
    return b;
}

}  // namespace host
}  // namespace pot3d

using namespace pot3d;
using namespace pot3d::host;

extern "C" {

const char *pot3d_version(void)
{
    return checked_build() ? "pot3d-mi355x 0.2 (gfx950, FP64 and FP32-refined Jacobi-PCG, checked indices)"
                           : "pot3d-mi355x 0.2 (gfx950, FP64 and FP32-refined Jacobi-PCG)";
}

int pot3d_set_refinement_mode(pot3d_ctx *ctx, int mode)
{
    if (!ctx) return fail(nullptr, POT3D_EINVAL, "ctx is NULL");
    if (ctx->precision != POT3D_FP32_REFINED) return fail(ctx, POT3D_EINVAL, "context is not FP32-refined");
    if (mode != POT3D_REFINE_RESTART && mode != POT3D_REFINE_RELIABLE) return fail(ctx, POT3D_EINVAL, "unknown mode");
    ctx->refine_mode = mode;
    return POT3D_OK;
}

int pot3d_set_refinement(pot3d_ctx *ctx, double inner_tol, int max_outer)
{
    if (!ctx) return fail(nullptr, POT3D_EINVAL, "ctx is NULL");
    if (ctx->precision != POT3D_FP32_REFINED) return fail(ctx, POT3D_EINVAL, "context is not FP32-refined");
    if (!(inner_tol > 0.0 && inner_tol < 1.0)) return fail(ctx, POT3D_EINVAL, "inner_tol must be in (0, 1)");
    if (max_outer < 1) return fail(ctx, POT3D_EINVAL, "max_outer must be >= 1");
    ctx->inner_tol = inner_tol;
    ctx->max_outer = max_outer;
    return POT3D_OK;
}

const char *pot3d_last_error(const pot3d_ctx *ctx)
{
    if (ctx) return ctx->err.c_str();
    return g_thread_error.c_str();
}

int pot3d_create(const double *r_faces, int nr, const double *t_faces, int nt, const double *p_faces, int np,
                 int upper_bc, int precision, int device, pot3d_ctx **out)
{
    return create_context(r_faces, nr, t_faces, nt, p_faces, np, upper_bc, precision, device, false, out);
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
    HIP_TRY(ctx, launch_stencil<double>(kApply, ctx->tile_o, ctx->grid_o, a, s));
    HIP_TRY(ctx, copy_rows(d_y, rowb, ctx->r, pitchb, rowb, nrows, hipMemcpyDeviceToDevice, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (const unsigned line = take_oob_line(s))
        return fail(ctx, POT3D_EDEVICE, "checked build: out-of-range index at kernels.hip line " + std::to_string(line));
    return POT3D_OK;
}

int pot3d_precondition_device(pot3d_ctx *ctx, const double *d_r, double *d_z, void *stream)
{
    if (!ctx) return fail(nullptr, POT3D_EINVAL, "ctx is NULL");
    if (!d_r || !d_z) return fail(ctx, POT3D_EINVAL, "r or z is NULL");
    if (d_r == d_z) return fail(ctx, POT3D_EINVAL, "r and z must be distinct");
    if (ctx->precision != POT3D_FP64) return fail(ctx, POT3D_EINVAL, "FP64 contexts only");
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return fail(ctx, POT3D_EDEVICE, "hipSetDevice failed");
    hipStream_t s = stream ? reinterpret_cast<hipStream_t>(stream) : ctx->stream;
    const size_t rowb = (size_t)ctx->np * sizeof(double), pitchb = (size_t)ctx->pitch * sizeof(double);
    const size_t nrows = (size_t)ctx->nr * ctx->nt;
    HIP_TRY(ctx, copy_rows(ctx->r, pitchb, d_r, rowb, rowb, nrows, hipMemcpyDeviceToDevice, s));
    double *zpad = ctx->p[1];
    if (ctx->precond == POT3D_PC_PHI_LINE) {
        zpad = ctx->z;
        HIP_TRY(ctx, launch_line<double>(ctx->grid_o, ctx->r, zpad, ctx->partial, ctx->line_blocks, ctx->sc, 1, s));
    } else {
        HIP_TRY(ctx, launch_jacobi(ctx->grid_o, ctx->r, zpad, s));
    }
    HIP_TRY(ctx, copy_rows(d_z, rowb, zpad, pitchb, rowb, nrows, hipMemcpyDeviceToDevice, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (const unsigned line = take_oob_line(s))
        return fail(ctx, POT3D_EDEVICE, "checked build: out-of-range index at kernels.hip line " + std::to_string(line));
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
    const bool closed = ctx->upper_bc == POT3D_UPPER_CLOSED_WALL;
    ctx->field_ready = false;   // the b plane no longer holds the last solve's
    if (closed) HIP_TRY(ctx, launch_monopole(d_br, ctx->bfac, ctx->dphi, ctx->nt, ctx->np, ctx->bcs, s));
    HIP_TRY(ctx, launch_rhs(d_br, ctx->bfac, ctx->dphi, ctx->nt, ctx->np, ctx->pitch, closed ? ctx->bcs : nullptr,
                            ctx->bplane, s));
    HIP_TRY(ctx, launch_fill<double>(d_b, ctx->n, 0.0, s));
    HIP_TRY(ctx, copy_rows(d_b, rowb, ctx->bplane, pitchb, rowb, (size_t)ctx->nt, hipMemcpyDeviceToDevice, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    return POT3D_OK;
}

int pot3d_field_device(pot3d_ctx *ctx, double *d_br, double *d_bt, double *d_bp, void *stream)
{
    if (!ctx) return fail(nullptr, POT3D_EINVAL, "ctx is NULL");
    if (!d_br || !d_bt || !d_bp) return fail(ctx, POT3D_EINVAL, "output pointers are required");
    if (!ctx->field_ready) return fail(ctx, POT3D_EINVAL, "no solution to take the field of (solve first)");
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return fail(ctx, POT3D_EDEVICE, "hipSetDevice failed");
    hipStream_t s = stream ? reinterpret_cast<hipStream_t>(stream) : ctx->stream;
    const double *fr = ctx->ftab, *ft = fr + ctx->nr + 1, *rinv = ft + ctx->nt + 1, *sinv = rinv + ctx->nr;
    HIP_TRY(ctx, launch_field(ctx->x, ctx->bplane, ctx->bfac, ctx->dphi, ctx->ih, fr, ft, rinv, sinv, ctx->nr, ctx->nt,
                              ctx->np, ctx->pitch, d_br, d_bt, d_bp, s));
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
    fill_shape(ctx, *out);
    const bool fp32 = ctx->precision == POT3D_FP32_REFINED;
    const double per = ctx->precond == POT3D_PC_PHI_LINE ? two_pass_bytes(fp32, ctx->graph_m) + (fp32 ? 8.0 : 16.0)
                       : one_sweep(ctx) ? sweep_bytes(fp32) : two_pass_bytes(fp32, ctx->graph_m);
    out->bytes_per_iter = per * (double)ctx->n;
    return POT3D_OK;
}

int pot3d_time_kernels(pot3d_ctx *ctx, int reps, double *ms_update_p, double *ms_update_r)
{
    if (!ctx) return fail(nullptr, POT3D_EINVAL, "ctx is NULL");
    if (reps <= 0 || !ms_update_p || !ms_update_r) return fail(ctx, POT3D_EINVAL, "reps > 0 and outputs required");
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return fail(ctx, POT3D_EDEVICE, "hipSetDevice failed");
    int rc;
    if (one_sweep(ctx) && ctx->precision == POT3D_FP32_REFINED) {
        rc = time_sweeps<float>(ctx, ctx->r32, ctx->r32b, ctx->p32[0], ctx->p32[1], ctx->e32, ctx->sc32, reps,
                                ms_update_p, ms_update_r);
    } else if (ctx->precision == POT3D_FP32_REFINED) {
        rc = time_pair<float>(ctx, ctx->r32, ctx->p32[0], ctx->p32[1], ctx->e32, ctx->sc32, reps, ms_update_p, ms_update_r);
    } else if (one_sweep(ctx)) {
        rc = time_sweeps<double>(ctx, ctx->r, ctx->r2, ctx->p[0], ctx->p[1], ctx->x, ctx->sc, reps, ms_update_p,
                                 ms_update_r);
    } else {
        rc = time_pair<double>(ctx, ctx->r, ctx->p[0], ctx->p[1], ctx->x, ctx->sc, reps, ms_update_p, ms_update_r);
    }
    ctx->have_solution = false;
    ctx->field_ready = false;
    if (rc == POT3D_OK) {
        if (const unsigned line = take_oob_line(ctx->stream))
            return fail(ctx, POT3D_EDEVICE, "checked build: out-of-range index at kernels.hip line " + std::to_string(line));
    }
    return rc;
}

int pot3d_set_iteration(pot3d_ctx *ctx, int iteration)
{
    if (!ctx) return fail(nullptr, POT3D_EINVAL, "ctx is NULL");
    if (iteration != POT3D_ITER_TWO_PASS && iteration != POT3D_ITER_ONE_SWEEP)
        return fail(ctx, POT3D_EINVAL, "iteration must be POT3D_ITER_TWO_PASS or POT3D_ITER_ONE_SWEEP");
    if (iteration == POT3D_ITER_ONE_SWEEP && !ctx->graph_s && !ctx->graph32s)
        return fail(ctx, POT3D_EINVAL, "the one-sweep iteration needs vectors under 4 GiB");
    ctx->iteration = iteration;
    return POT3D_OK;
}

int pot3d_set_preconditioner(pot3d_ctx *ctx, int pc)
{
    if (!ctx) return fail(nullptr, POT3D_EINVAL, "ctx is NULL");
    if (pc != POT3D_PC_JACOBI && pc != POT3D_PC_PHI_LINE)
        return fail(ctx, POT3D_EINVAL, "pc must be POT3D_PC_JACOBI or POT3D_PC_PHI_LINE");
    if (pc == POT3D_PC_JACOBI) {
        ctx->precond = pc;
        return POT3D_OK;
    }
    if (ctx->serving) return fail(ctx, POT3D_EINVAL, "the phi-line preconditioner runs single solves only");
    if (ctx->np > kMaxLineCells)
        return fail(ctx, POT3D_EINVAL, "the phi-line preconditioner takes at most 2048 azimuthal cells");
    const double h = kTwoPi / ctx->np;
    for (int k = 0; k < ctx->np; ++k)
        if (std::fabs(ctx->dphi_h[k] - h) > 1e-12 * h)
            return fail(ctx, POT3D_EINVAL, "the phi-line preconditioner needs uniform phi faces");
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return fail(ctx, POT3D_EDEVICE, "hipSetDevice failed");
    const long long rows = (long long)ctx->nr * ctx->nt;
    // one wave of resident workgroups, each wavefront walking rows with the
    // grid's stride (wider grids measured slower at 151 x 301 x 601)
    const int per_cu = ctx->precision == POT3D_FP64 ? line_blocks_per_cu<double>(ctx->np)
                                                    : line_blocks_per_cu<float>(ctx->np);
    ctx->line_blocks = (int)std::max<long long>(
        1, std::min<long long>({(rows + kWaves - 1) / kWaves, (long long)ctx->max_blocks,
                                (long long)std::max(1, per_cu) * ctx->num_cu}));
    if (const int lb = env_int("POT3D_LINE_BLOCKS", 0); lb > 0)   // launch-width experiments
        ctx->line_blocks = std::min(lb, ctx->line_blocks);
    if (ctx->precision == POT3D_FP64) {
        if (!ctx->z) {
            HIP_TRY(ctx, dalloc(&ctx->z, (size_t)ctx->npad));
            HIP_TRY(ctx, launch_fill<double>(ctx->z, ctx->npad, 0.0, ctx->stream));
            HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        }
        if (!ctx->graph_l) {
            const int rc = capture_line_iterations<double>(ctx, ctx->r, ctx->p[0], ctx->p[1], ctx->x, ctx->z, ctx->sc,
                                                           &ctx->graph_l);
            if (rc != POT3D_OK) return rc;
        }
    } else {
        // FP32-refined: the inner FP32 iterations take the line preconditioner
        if (!ctx->z32) {
            HIP_TRY(ctx, dalloc(&ctx->z32, (size_t)ctx->npad));
            HIP_TRY(ctx, launch_fill<float>(ctx->z32, ctx->npad, 0.0f, ctx->stream));
            HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        }
        if (!ctx->graph32l) {
            const int rc = capture_line_iterations<float>(ctx, ctx->r32, ctx->p32[0], ctx->p32[1], ctx->e32, ctx->z32,
                                                          ctx->sc32, &ctx->graph32l);
            if (rc != POT3D_OK) return rc;
        }
    }
    ctx->precond = pc;
    return POT3D_OK;
}

void pot3d_destroy(pot3d_ctx *ctx) { free_ctx(ctx); }

}  // extern "C"
