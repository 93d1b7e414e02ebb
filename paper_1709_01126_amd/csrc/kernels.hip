// kernels.hip -- gfx950 kernels of the Jacobi-PCG iteration for the
// volume-scaled spherical Laplacian (arXiv:1709.01126, Sec. 2.2-2.3).
//
// One marching kernel serves every pass over the 7-point stencil:
//   apply       y = A x
//   residual    r = b - A x, with partial sums r.z, r.r, b.b   (z = D^-1 r)
//   update-p    p = D^-1 r + beta p_old (stored), q = A p, partial p.q
//   update-r    q = A p again, r -= alpha q, x += alpha p, partial r.z, r.r
// update-p and update-r are the two HBM passes of one PCG iteration: they
// read r, p_old and write p (24 bytes per unknown), then read p, r, x and write
// r, x (40 bytes per unknown).  A p is never stored; recomputing it is free
// next to the memory traffic.
//
// A workgroup (4 wavefronts) owns a TJ x 64 (theta x phi) tile of the grid and
// walks a chunk of radial layers i0..i1-1.  It keeps the operand at layers
// i-1, i, i+1 of its own points in registers, and layer i with a one-point
// halo ring in LDS for the theta and phi neighbours (3 LDS slots rotate, so
// there is one barrier per layer).  Every wavefront reads one 64-wide,
// phi-contiguous row segment per access.  Periodic phi wraps inside the row;
// pole and radial boundary rows carry zero weights in the row table, so the
// kernel has no boundary branches beyond the tile edges.
//
// Reductions are deterministic: wavefront butterfly, then the 4 waves in
// fixed order, one partial per workgroup, then a single-workgroup finisher
// that sums partials in a fixed order.
#include "kernels.hpp"

#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

namespace pot3d {

// Checked builds (-DPOT3D_CHECKED, libpot3d_checked.so) test every global
// index of the stencil kernels against its array size.  An index out of range
// is replaced by 0 and the source line is recorded in g_oob_line, which the
// host reads after each solve.  Normal builds compile CHK(i, n) to i.
#ifdef POT3D_CHECKED
__device__ unsigned int g_oob_line = 0;
__device__ __forceinline__ long long chk_index(long long i, long long n, unsigned line)
{
    if (i < 0 || i >= n) {
        g_oob_line = line;
        return 0;
    }
    return i;
}
#define CHK(i, n) chk_index((long long)(i), (long long)(n), __LINE__)
#else
#define CHK(i, n) (i)
#endif

template <typename V> __device__ __forceinline__ V vfma(V a, V b, V c);
template <> __device__ __forceinline__ double vfma<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }
template <> __device__ __forceinline__ float vfma<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Pointer to global memory, typed as such.
template <typename T>
using GPtr = __attribute__((address_space(1))) T *;
template <typename T>
__device__ __forceinline__ GPtr<T> to_global(T *p)
{
    return (GPtr<T>)p;
}

// Streaming accesses: vectors that a pass reads or writes once per cell use
// the non-temporal policy, so they do not displace the lines that are read
// again soon (the operand's halo rows and layers, and the tiles the next pass
// starts on).  Measured: 393 -> 369 us per FP64 iteration at 151 x 301 x 601,
// 3.72 -> 3.48 ms at 301 x 641 x 1281, FP32-refined solve 1.28 -> 1.23 s.
template <typename P>
__device__ __forceinline__ auto stream_load(P p)
{
    return __builtin_nontemporal_load(p);
}
template <typename P, typename T>
__device__ __forceinline__ void stream_store(P p, T v)
{
    __builtin_nontemporal_store(v, p);
}

// Pointer to memory that no kernel writes while this one runs (row tables,
// the scalar block): uniform loads through it become scalar loads.
template <typename T>
using CPtr = __attribute__((address_space(4))) T *;
template <typename T>
__device__ __forceinline__ CPtr<T> to_const(T *p)
{
    return (CPtr<T>)p;
}

__device__ __forceinline__ RowCoef load_row(CPtr<const RowCoef> rows, long long idx)
{
    RowCoef r;
    r.rm = rows[idx].rm;
    r.rp = rows[idx].rp;
    r.tm = rows[idx].tm;
    r.tp = rows[idx].tp;
    r.s = rows[idx].s;
    r.pq = rows[idx].pq;
    r.pad0 = r.pad1 = 0.0;
    return r;
}

// Diagonal of A at one point (the Jacobi preconditioner).
template <typename V>
__device__ __forceinline__ V diag_at(const RowCoef &rc, V dph, V ihm, V ihk)
{
    return vfma<V>(dph, (V)rc.s, (V)rc.pq * (ihm + ihk));
}

// The r/x update in pairs of iterations: the even one records the increment
// x still lacks (alpha_k p_k: the scalar and the buffer of p_k), which a
// catch-up adds if the solve ends after it; the other r/x updates clear it.
template <int MODE, typename V>
__device__ __forceinline__ void record_x_lag(const DevScalars *sc, CPtr<const DevScalars> csc, const V *p, int b)
{
    if (is_update_r(MODE) && b == 0 && threadIdx.x == 0) {
        DevScalars *w = const_cast<DevScalars *>(sc);
        w->x_lag = MODE == kUpdateRSkip ? csc->alpha : 0.0;
        w->x_lag_p = MODE == kUpdateRSkip ? (unsigned long long)p : 0ull;
    }
}

// The LDS-plane marching pass for one workgroup; b is the workgroup's index
// within its own launch shape (blockIdx.x for a single solve, the index inside
// the slot for a batched launch).
template <int TJ, int MODE, typename V>
__device__ __forceinline__ void march_body(const GridArgs &g, const StencilVecs<V> &v, const RowCoef *__restrict__ rows,
                                           const V *__restrict__ vin, const V *__restrict__ vpold, V *__restrict__ vout,
                                           V *__restrict__ vout2, const int b)
{
    static_assert(TJ % kWaves == 0 && 2 * TJ <= kWave, "tile rows");
    constexpr int M = TJ / kWaves;   // rows per wavefront
    constexpr int TK = kWave;
    __shared__ V lds[3][TJ + 2][TK + 2];
    __shared__ double red[kWaves][3];

    const CPtr<const DevScalars> csc = to_const(v.sc);
    const CPtr<const RowCoef> crows = to_const(rows);
    if (!v.ignore_done && csc->done) return;   // uniform over the workgroup
    if (v.tstamp && threadIdx.x == 0) atomicMin(&v.tstamp[0], wall_clock64());

    // Element accesses go through global-address-space pointers.  A batched
    // launch reads its pointers from the slot table, and the compiler would
    // otherwise use flat accesses there, which share a wait counter with the
    // LDS traffic of the plane pipeline.
    const GPtr<const V> gin = to_global(vin), gpold = to_global(vpold);
    const GPtr<V> gout = to_global(vout), gout2 = to_global(vout2);
    const GPtr<const double> gdphi = to_global(g.dphi), gih = to_global(g.ih), gbp = to_global(v.bplane);
    const GPtr<double> gpart = to_global(v.partial);

    // Workgroup -> tile.  Hardware hands consecutive workgroup ids to the 8
    // XCDs in turn; renumber so that each XCD works on a contiguous range of
    // logical tiles and shares their halos in its L2.  The phi tile varies
    // fastest: the phi-halo cells of a tile sit in 128-byte lines owned by its
    // phi neighbours, which then run beside it on the same XCD.
    const int per = g.nblocks / kXcds;
    int L = (b < per * kXcds) ? (b % kXcds) * per + b / kXcds : b;
    if (g.reverse) L = g.nblocks - 1 - L;
    const int kt = L % g.ntk;
    L /= g.ntk;
    const int ic = L % g.nchunk;
    const int jt = L / g.nchunk;
    const int i0 = ic * g.ci;
    const int i1 = min(i0 + g.ci, g.nr);
    const int j0 = jt * TJ;
    const int k0 = kt * TK;

    const int nt = g.nt, np = g.np, nr = g.nr;
    const int lane = threadIdx.x & (kWave - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int k = k0 + lane;
    const bool kval = k < np;
    const int kc = kval ? k : np - 1;          // in-row address for every lane
    const V mk = kval ? V(1) : V(0);
    // LDS column of the k+1 neighbour: the last cell of a row wraps to k = 0,
    // which the right halo column holds.
    const int kp_col = (k == np - 1) ? TK + 1 : lane + 2;

    const V dph = kval ? (V)gdphi[CHK(kc, np)] : V(0);
    const V ihm = kval ? (V)gih[CHK(kc == 0 ? np - 1 : kc - 1, np)] : V(0);
    const V ihk = kval ? (V)gih[CHK(kc, np)] : V(0);

    // Halo ring of the tile in one layer: wave 0 the row below (j0-1), wave 1
    // the row above (j0+TJ), wave 2 the left and right columns (wrapped in phi).
    int hrow = -1, hcol = 0, hj = 0, hk = 0;
    bool hval = false;
    if (w < 2) {
        hrow = (w == 0) ? 0 : TJ + 1;
        hcol = lane + 1;
        hj = (w == 0) ? j0 - 1 : j0 + TJ;
        hk = kc;
        hval = kval && hj >= 0 && hj < nt;
    } else if (w == 2 && lane < 2 * TJ) {
        const bool left = lane < TJ;
        hrow = (left ? lane : lane - TJ) + 1;
        hcol = left ? 0 : TK + 1;
        hj = j0 + hrow - 1;
        hk = left ? (k0 == 0 ? np - 1 : k0 - 1) : (k0 + TK >= np ? 0 : k0 + TK);
        hval = hj < nt;
    }
    const int hjc = min(max(hj, 0), nt - 1);   // clamped halo address
    const V mh = hval ? V(1) : V(0);
    V hdph = 0, hihm = 0, hihk = 0;
    if (MODE == kUpdateP) {
        hdph = (V)gdphi[CHK(hk, np)];
        hihm = (V)gih[CHK(hk == 0 ? np - 1 : hk - 1, np)];
        hihk = (V)gih[CHK(hk, np)];
    }

    V beta = 0, alpha = 0, alpha_p = 0;
    if (MODE == kUpdateP) beta = (V)csc->beta;
    if (is_update_r(MODE)) alpha = (V)csc->alpha;
    if (MODE == kUpdateRPair) alpha_p = (V)csc->alpha_prev;
    record_x_lag<MODE>(v.sc, csc, vin, b);

    auto offs = [&](int ip, int j, int kk) -> long long {
        return (long long)ip * g.plane + (long long)j * g.pitch + kk;
    };
    // Operand from raw loads: update-p forms z + beta p_old, otherwise the
    // loaded value.  Masked by multiplication (clamped data are finite).
    auto eval = [&](V a, V bold, const RowCoef &rc, V pdph, V pihm, V pihk, V mask) -> V {
        if constexpr (MODE == kUpdateP) {
            // z = D^-1 r, or the operand itself when it is z already (block preconditioner)
            const V z = v.zin ? a : a / diag_at<V>(rc, pdph + (V(1) - mask), pihm, pihk);
            return vfma<V>(beta, bold, z) * mask;
        } else {
            return a * mask;
        }
    };

    V q0[M], q1[M], q2[M];
    // Layer ip: the own rows into dst (and LDS slot `slot` if to_lds, with the
    // halo ring), storing the new direction when asked.  All loads first.
    auto produce = [&](int ip_in, bool ip_on, int slot, V (&dst)[M], bool to_lds, bool store) {
        const int ip = min(max(ip_in, 0), nr - 1);   // the layer below the first chunk is -1
        V ra[M], rb[M];
        RowCoef rcs[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int jc = min(j0 + w + kWaves * m, nt - 1);
            const long long o = offs(ip, jc, kc);
            if constexpr (MODE == kUpdateP) {
                // r and p_old of the own rows: read once here (neighbours read
                // their halo copies)
                ra[m] = stream_load(gin + CHK(o, g.npad));
                rb[m] = stream_load(gpold + CHK(o, g.npad));
                rcs[m] = load_row(crows, CHK(ip * nt + jc, nr * nt));
            } else {
                ra[m] = gin[CHK(o, g.npad)];
                rb[m] = 0;
            }
        }
        V ha = 0, hb = 0;
        RowCoef hrc{};
        if (to_lds) {
            const long long o = offs(ip, hjc, hk);
            ha = gin[CHK(o, g.npad)];
            if constexpr (MODE == kUpdateP) {
                hb = gpold[CHK(o, g.npad)];
                hrc = load_row(crows, CHK(ip * nt + hjc, nr * nt));
            }
        }
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int row = w + kWaves * m;
            const int j = j0 + row;
            const V mrow = (ip_on && j < nt) ? mk : V(0);
            const V val = eval(ra[m], rb[m], rcs[m], dph, ihm, ihk, mrow);
            dst[m] = val;
            if constexpr (MODE == kUpdateP) {
                if (store && kval && j < nt) stream_store(gout + CHK(offs(ip, j, k), g.npad), val);
            }
            if (to_lds) lds[slot][row + 1][lane + 1] = val;
        }
        if (to_lds && hrow >= 0) lds[slot][hrow][hcol] = eval(ha, hb, hrc, hdph, hihm, hihk, ip_on ? mh : V(0));
    };

    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;

    produce(i0 - 1, i0 > 0, 0, q0, false, false);
    produce(i0, true, i0 % 3, q1, true, MODE == kUpdateP);

    for (int i = i0; i < i1; ++i) {
        // this layer's r and x (update-r), issued with the next layer's operand
        V rv[M], xv[M], pv[M];
        RowCoef rc[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int jc = min(j0 + w + kWaves * m, nt - 1);
            rc[m] = load_row(crows, CHK(i * nt + jc, nr * nt));
            if constexpr (is_update_r(MODE)) {
                const long long o = CHK(offs(i, jc, kc), g.npad);
                rv[m] = stream_load(gout + o);
                if constexpr (MODE != kUpdateRSkip) xv[m] = stream_load(gout2 + o);
                if constexpr (MODE == kUpdateRPair) pv[m] = stream_load(gpold + o);   // p_{k-1}
            }
        }
        produce(i + 1, i + 1 < nr, (i + 1) % 3, q2, true, MODE == kUpdateP && i + 1 < i1);
        __syncthreads();
        const int s = i % 3;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int row = w + kWaves * m;
            const int j = j0 + row;
            const bool on = kval && j < nt;
            const RowCoef &r_ = rc[m];
            const V pc = q1[m];
            const V pjm = lds[s][row][lane + 1];
            const V pjp = lds[s][row + 2][lane + 1];
            const V pkm = lds[s][row + 1][lane];
            const V pkp = lds[s][row + 1][kp_col];
            // (A p) = dphi_k (s pc - rm p_{i-1} - rp p_{i+1} - tm p_{j-1} - tp p_{j+1})
            //       + pq (ih_{k-1} (pc - p_{k-1}) + ih_k (pc - p_{k+1}))
            V t = (V)r_.s * pc;
            t = vfma<V>(-(V)r_.rm, q0[m], t);
            t = vfma<V>(-(V)r_.rp, q2[m], t);
            t = vfma<V>(-(V)r_.tm, pjm, t);
            t = vfma<V>(-(V)r_.tp, pjp, t);
            V u = ihm * (pc - pkm);
            u = vfma<V>(ihk, pc - pkp, u);
            const V ap = vfma<V>(dph, t, (V)r_.pq * u);
            const long long idx = on ? CHK(offs(i, j, k), g.npad) : 0;
            if constexpr (MODE == kApply) {
                if (on) gout[idx] = ap;
            } else if constexpr (MODE == kResidual) {
                if (on) {
                    const double bval = (i == 0) ? gbp[CHK((long long)j * g.pitch + k, (long long)nt * g.pitch)] : 0.0;
                    const V res = (V)(bval - (double)ap);
                    if (v.store_r) gout[idx] = res;
                    const V z = res / diag_at<V>(r_, dph, ihm, ihk);
                    acc0 += (double)res * (double)z;
                    acc1 += (double)res * (double)res;
                    acc2 += bval * bval;
                }
            } else if constexpr (MODE == kUpdateP) {
                if (on) acc0 += (double)pc * (double)ap;
            } else {  // kUpdateR
                if (on) {
                    const V rn = vfma<V>(-alpha, ap, rv[m]);
                    stream_store(gout + idx, rn);
                    if constexpr (MODE == kUpdateR) stream_store(gout2 + idx, vfma<V>(alpha, pc, xv[m]));
                    if constexpr (MODE == kUpdateRPair)
                        stream_store(gout2 + idx, vfma<V>(alpha, pc, vfma<V>(alpha_p, pv[m], xv[m])));
                    if (!v.zin) {   // with a block preconditioner the line pass takes r.z and r.r
                        const V z = rn / diag_at<V>(r_, dph, ihm, ihk);
                        acc0 += (double)rn * (double)z;
                        acc1 += (double)rn * (double)rn;
                    }
                }
            }
        }
#pragma unroll
        for (int m = 0; m < M; ++m) {
            q0[m] = q1[m];
            q1[m] = q2[m];
        }
    }

    if constexpr (MODE != kApply) {
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) {
            acc0 += __shfl_xor(acc0, off, kWave);
            acc1 += __shfl_xor(acc1, off, kWave);
            acc2 += __shfl_xor(acc2, off, kWave);
        }
        if (lane == 0) {
            red[w][0] = acc0;
            red[w][1] = acc1;
            red[w][2] = acc2;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
            for (int q = 0; q < kWaves; ++q) {
                s0 += red[q][0];
                s1 += red[q][1];
                s2 += red[q][2];
            }
            gpart[CHK(b, g.nblocks)] = s0;
            gpart[CHK(g.nblocks + b, 3LL * g.nblocks)] = s1;
            gpart[CHK(2 * g.nblocks + b, 3LL * g.nblocks)] = s2;
        }
    }
    if (v.tstamp) {   // timing runs: this workgroup's end
        __syncthreads();
        if (threadIdx.x == 0) atomicMax(&v.tstamp[1], wall_clock64());
    }
}

template <int TJ, int MODE, typename V>
__global__ void __launch_bounds__(kThreads)
stencil_march(GridArgs g, StencilVecs<V> v, const RowCoef *__restrict__ rows, const V *__restrict__ vin,
              const V *__restrict__ vpold, V *__restrict__ vout, V *__restrict__ vout2)
{
    march_body<TJ, MODE, V>(g, v, rows, vin, vpold, vout, vout2, blockIdx.x);
}

// Index of the slot that owns workgroup bid of a batched launch, or -1.
template <typename S>
__device__ __forceinline__ int batch_slot(const S *__restrict__ slots, int nslots, int bid)
{
    int s = -1;
    for (int q = 0; q < nslots; ++q) {
        const S &sl = slots[q];
        if (sl.active && bid >= sl.offset && bid < sl.offset + sl.g.nblocks) s = q;
    }
    return s;
}

// Batched pass: one launch covers every active slot of a slot table.  Slot q
// owns workgroups [offset, offset + nblocks) of the grid (offsets are
// multiples of 8, so the XCD-aware tile order inside a slot is unchanged), and
// each slot runs exactly the arithmetic of its single-solve launch.
template <int TJ, int MODE, typename V>
__global__ void __launch_bounds__(kThreads)
stencil_march_batch(const BatchSlot<V> *__restrict__ slots, int nslots)
{
    const int bid = blockIdx.x;
    const int s = batch_slot(slots, nslots, bid);
    if (s < 0) return;
    const BatchSlot<V> sl = slots[s];
    march_body<TJ, MODE, V>(sl.g, sl.v, sl.g.rows, sl.v.in, sl.v.pold, sl.out, sl.v.x, bid - sl.offset);
}

// ---------------------------------------------------------------------------
// Wavefront-level marching kernel (no LDS, no barriers in the sweep).
//
// A task is one wavefront's column of the grid: M consecutive polar rows j0..j0+M-1
// times a 128-cell azimuthal segment (two consecutive cells per lane, moved with
// 16-byte accesses), over a chunk of radial layers.  The wavefront holds the
// operand at layers i-1, i, i+1 of its own rows in registers.  Theta neighbours
// are the neighbouring own rows; the two rows just outside the run are loaded
// per layer.  Phi neighbours cross lanes with DPP wavefront shifts, and the
// segment ends take the cells just outside it (wrapped in phi).
//
// The loads of a layer do not depend on each other and sit in one basic block:
// out-of-range rows, layers and lanes read a clamped in-range address, and their
// values are masked afterwards.  One layer therefore costs about one memory round
// trip per wavefront, and the wavefronts never wait for each other until the
// final reduction.
// ---------------------------------------------------------------------------
// Two consecutive cells moved as one 16-byte (FP64) or 8-byte (FP32) access
// (the compiler's own vector type, which loads and stores through
// address-space-qualified pointers).
template <typename V> struct Pair;
template <> struct Pair<double> { typedef double T __attribute__((ext_vector_type(2))); };
template <> struct Pair<float> { typedef float T __attribute__((ext_vector_type(2))); };

// Lane l receives the value of lane l-1 (lane 0 receives 0).
__device__ __forceinline__ double lane_from_left(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
// Lane l receives the value of lane l+1 (lane 63 receives 0).
__device__ __forceinline__ double lane_from_right(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane_from_left(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, false));
}
__device__ __forceinline__ float lane_from_right(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, false));
}

__device__ __forceinline__ double wave_uniform(double v)
{
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float wave_uniform(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

template <int M, int MODE, typename V>
__device__ __forceinline__ void wave_body(const GridArgs &g, const StencilVecs<V> &v, const RowCoef *__restrict__ rows,
                                          const V *__restrict__ vin, const V *__restrict__ vpold, V *__restrict__ vout,
                                          V *__restrict__ vout2, const int b)
{
    using P2 = typename Pair<V>::T;
    constexpr int SEG = 2 * kWave;   // azimuthal cells per task
    __shared__ double red[kWaves][3];

    const CPtr<const DevScalars> csc = to_const(v.sc);
    const CPtr<const RowCoef> crows = to_const(rows);
    if (!v.ignore_done && csc->done) return;   // uniform over the workgroup
    if (v.tstamp && threadIdx.x == 0) atomicMin(&v.tstamp[0], wall_clock64());
    record_x_lag<MODE>(v.sc, csc, vin, b);
    const GPtr<const V> gin = to_global(vin), gpold = to_global(vpold);
    const GPtr<V> gout = to_global(vout), gout2 = to_global(vout2);
    const GPtr<const double> gdphi = to_global(g.dphi), gih = to_global(g.ih), gbp = to_global(v.bplane);
    const GPtr<double> gpart = to_global(v.partial);

    const int lane = threadIdx.x & (kWave - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int per = g.nblocks / kXcds;
    int L = (b < per * kXcds) ? (b % kXcds) * per + b / kXcds : b;
    if (g.reverse) L = g.nblocks - 1 - L;
    const int task = L * kWaves + w;
    const int ntask = g.ntj * g.ntk * g.nchunk;
    const int nt = g.nt, np = g.np, nr = g.nr;

    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;

    if (task < ntask) {
        const int ks = task % g.ntk;
        const int rest = task / g.ntk;
        const int jr = rest % g.ntj;
        const int ic = rest / g.ntj;
        const int i0 = ic * g.ci;
        const int i1 = min(i0 + g.ci, nr);
        const int j0 = jr * M;
        const int k0 = ks * SEG;
        const int kb = k0 + 2 * lane;            // this lane's first cell
        const bool lane_on = kb < g.pitch;       // both cells inside the padded row
        const int kc = lane_on ? kb : 0;         // in-row address for every lane
        const bool v0 = kb < np, v1 = kb + 1 < np;
        const int kl = (k0 == 0) ? np - 1 : k0 - 1;          // cell left of the segment
        const int kr = (k0 + SEG >= np) ? 0 : k0 + SEG;      // cell right of the segment
        const bool last0 = kb == np - 1, last1 = kb + 1 == np - 1;
        const int jlo = max(j0 - 1, 0), jhi = min(j0 + M, nt - 1);       // clamped halo rows
        const bool hlo_on = j0 > 0, hhi_on = j0 + M < nt;

        const int kc0 = v0 ? kb : 0, kc1 = v1 ? kb + 1 : 0;
        const V mv0 = v0 ? V(1) : V(0), mv1 = v1 ? V(1) : V(0);
        const V dph0 = v0 ? (V)gdphi[CHK(kc0, np)] : V(0), dph1 = v1 ? (V)gdphi[CHK(kc1, np)] : V(0);
        const V ihk0 = v0 ? (V)gih[CHK(kc0, np)] : V(0), ihk1 = v1 ? (V)gih[CHK(kc1, np)] : V(0);
        const V ihm0 = v0 ? (V)gih[CHK(kc0 == 0 ? np - 1 : kc0 - 1, np)] : V(0), ihm1 = ihk0;
        const V dphl = (V)gdphi[CHK(kl, np)], ihml = (V)gih[CHK(kl == 0 ? np - 1 : kl - 1, np)], ihkl = (V)gih[CHK(kl, np)];
        const V dphr = (V)gdphi[CHK(kr, np)], ihmr = (V)gih[CHK(kr == 0 ? np - 1 : kr - 1, np)], ihkr = (V)gih[CHK(kr, np)];
        const V beta = (MODE == kUpdateP) ? (V)csc->beta : V(0);
        const V alpha = is_update_r(MODE) ? (V)csc->alpha : V(0);
        const V alpha_p = (MODE == kUpdateRPair) ? (V)csc->alpha_prev : V(0);

        auto rowoff = [&](int ip, int j) -> long long { return (long long)ip * g.plane + (long long)j * g.pitch; };
        auto ld2 = [&](GPtr<const V> p, long long off) -> P2 { return *(GPtr<const P2>)(p + CHK(off, g.npad - 1)); };
        // a vector read once per cell in this pass (see stream_load)
        auto ld2_stream = [&](GPtr<const V> p, long long off) -> P2 {
            return stream_load((GPtr<const P2>)(p + CHK(off, g.npad - 1)));
        };

        // Raw loads of the operand on a row segment, and their evaluation.
        struct Raw { P2 a, b; };
        // own: one of this wavefront's rows (update-p reads r and p_old there
        // once; the halo rows are read again by the neighbouring task)
        auto raw_row = [&](int ip, int j, bool own) -> Raw {
            const long long off = rowoff(ip, j) + kc;
            Raw q;
            if constexpr (MODE == kUpdateP) {
                q.a = own ? ld2_stream(gin, off) : ld2(gin, off);
                q.b = own ? ld2_stream(gpold, off) : ld2(gpold, off);
            } else {
                q.a = ld2(gin, off);
            }
            return q;
        };
        // Evaluate a raw row segment with the row's coefficients (update-p: the
        // new direction z + beta p_old; otherwise the loaded value), masked.
        auto eval_row = [&](const Raw &q, const RowCoef &rc, bool on, V &a0, V &a1) {
            V e0, e1;
            if constexpr (MODE == kUpdateP) {
                const V z0 = v.zin ? q.a.x : q.a.x / diag_at<V>(rc, dph0 + (V)(!v0), ihm0, ihk0);
                const V z1 = v.zin ? q.a.y : q.a.y / diag_at<V>(rc, dph1 + (V)(!v1), ihm1, ihk1);
                e0 = vfma<V>(beta, q.b.x, z0);
                e1 = vfma<V>(beta, q.b.y, z1);
            } else {
                e0 = q.a.x;
                e1 = q.a.y;
            }
            // masked by multiplication: a select would let the compiler sink the
            // loads into a branch; clamped data are finite, so x * 0 = 0
            const V mon = on ? V(1) : V(0);
            a0 = e0 * (mon * mv0);
            a1 = e1 * (mon * mv1);
        };
        // Raw loads of the operand at one cell (same address on every lane).
        struct RawCell { V a, b; };
        // (made wave-uniform so that the load is issued with the others, not
        // sunk into the lanes that use it)
        auto raw_cell = [&](int ip, int j, int kk) -> RawCell {
            const long long off = rowoff(ip, j) + kk;
            RawCell q;
            q.a = wave_uniform(gin[CHK(off, g.npad)]);
            if constexpr (MODE == kUpdateP) q.b = wave_uniform(gpold[CHK(off, g.npad)]);
            else q.b = 0;
            return q;
        };
        auto eval_cell = [&](const RawCell &q, const RowCoef &rc, V cdph, V cihm, V cihk) -> V {
            if constexpr (MODE == kUpdateP)
                return vfma<V>(beta, q.b, v.zin ? q.a : q.a / diag_at<V>(rc, cdph, cihm, cihk));
            else return q.a;
        };
        auto store2 = [&](GPtr<V> dst, int ip, int j, V a0, V a1) {
            P2 o;
            o.x = v0 ? a0 : V(0);
            o.y = v1 ? a1 : V(0);
            GPtr<P2> to = (GPtr<P2>)(dst + CHK(rowoff(ip, j) + kc, g.npad - 1));
            if constexpr (MODE == kUpdateP || is_update_r(MODE)) {
                if (lane_on) stream_store(to, o);
            } else {
                if (lane_on) *to = o;
            }
        };

        V q0[M][2], q1[M][2], q2[M][2];
        // own rows of layer ip (clamped loads, masked values); store p if asked
        auto produce_own = [&](int ip, bool ip_on, V (&dst)[M][2], bool store) {
            const int ipc = min(ip, nr - 1);
            Raw raw[M];
            RowCoef rcs[M];
#pragma unroll
            for (int m = 0; m < M; ++m) {
                raw[m] = raw_row(ipc, min(j0 + m, nt - 1), true);
                if constexpr (MODE == kUpdateP) rcs[m] = load_row(crows, CHK(ipc * nt + min(j0 + m, nt - 1), nr * nt));
            }
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int j = j0 + m;
                eval_row(raw[m], rcs[m], ip_on && j < nt, dst[m][0], dst[m][1]);
                if constexpr (MODE == kUpdateP) {
                    if (store && j < nt) store2(gout, ip, j, dst[m][0], dst[m][1]);
                }
            }
        };

        produce_own(i0 - 1 < 0 ? 0 : i0 - 1, i0 > 0, q0, false);
        produce_own(i0, true, q1, MODE == kUpdateP);

        for (int i = i0; i < i1; ++i) {
            // ---- every load of this layer, unconditionally, from clamped addresses ----
            const int ipn = min(i + 1, nr - 1);
            Raw nxt[M], hraw[2];
            RawCell cl[M], cr[M];
            RowCoef rc[M], rcn[M], rch[2];
            P2 rv[M], xv[M], pv[M];
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int jc = min(j0 + m, nt - 1);
                rc[m] = load_row(crows, CHK(i * nt + jc, nr * nt));
                nxt[m] = raw_row(ipn, jc, true);
                if constexpr (MODE == kUpdateP) rcn[m] = load_row(crows, CHK(ipn * nt + jc, nr * nt));
                cl[m] = raw_cell(i, jc, kl);
                cr[m] = raw_cell(i, jc, kr);
                if constexpr (is_update_r(MODE)) {
                    rv[m] = ld2_stream(gout, rowoff(i, jc) + kc);
                    if constexpr (MODE != kUpdateRSkip) xv[m] = ld2_stream(gout2, rowoff(i, jc) + kc);
                    if constexpr (MODE == kUpdateRPair) pv[m] = ld2_stream(gpold, rowoff(i, jc) + kc);   // p_{k-1}
                }
            }
            hraw[0] = raw_row(i, jlo, false);
            hraw[1] = raw_row(i, jhi, false);
            if constexpr (MODE == kUpdateP) {
                rch[0] = load_row(crows, CHK(i * nt + jlo, nr * nt));
                rch[1] = load_row(crows, CHK(i * nt + jhi, nr * nt));
            }
            // ---- next layer's operand (stored as the new direction in update-p) ----
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int j = j0 + m;
                eval_row(nxt[m], rcn[m], i + 1 < nr && j < nt, q2[m][0], q2[m][1]);
                if constexpr (MODE == kUpdateP) {
                    if (i + 1 < i1 && j < nt) store2(gout, i + 1, j, q2[m][0], q2[m][1]);
                }
            }
            V hlo0, hlo1, hhi0, hhi1;
            eval_row(hraw[0], rch[0], hlo_on, hlo0, hlo1);
            eval_row(hraw[1], rch[1], hhi_on, hhi0, hhi1);
            // ---- stencil on the own rows of layer i ----
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int j = j0 + m;
                const bool row_on = j < nt;          // uniform: rows past the pole are masked
                const double wrow = row_on ? 1.0 : 0.0;
                const V kL = eval_cell(cl[m], rc[m], dphl, ihml, ihkl);
                const V kR = eval_cell(cr[m], rc[m], dphr, ihmr, ihkr);
                const V c0 = q1[m][0], c1 = q1[m][1];
                const V jm0 = (m > 0) ? q1[m - 1][0] : hlo0, jm1 = (m > 0) ? q1[m - 1][1] : hlo1;
                const V jp0 = (m + 1 < M) ? q1[m + 1][0] : hhi0, jp1 = (m + 1 < M) ? q1[m + 1][1] : hhi1;
                const V from_left = lane_from_left(c1);     // second cell of lane-1
                const V from_right = lane_from_right(c0);   // first cell of lane+1
                const V km0 = (lane == 0) ? kL : from_left;
                const V kp0 = last0 ? kR : c1;
                const V km1 = c0;
                const V kp1 = (last1 || lane == kWave - 1) ? kR : from_right;
                const V cc[2] = {c0, c1}, ii[2] = {q0[m][0], q0[m][1]}, ipv[2] = {q2[m][0], q2[m][1]};
                const V jm[2] = {jm0, jm1}, jp[2] = {jp0, jp1}, km[2] = {km0, km1}, kp[2] = {kp0, kp1};
                const V dph[2] = {dph0, dph1}, ihm[2] = {ihm0, ihm1}, ihk[2] = {ihk0, ihk1};
                const bool ve[2] = {v0, v1};
                const RowCoef &r_ = rc[m];
                V ap[2];
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    V t = (V)r_.s * cc[e];
                    t = vfma<V>(-(V)r_.rm, ii[e], t);
                    t = vfma<V>(-(V)r_.rp, ipv[e], t);
                    t = vfma<V>(-(V)r_.tm, jm[e], t);
                    t = vfma<V>(-(V)r_.tp, jp[e], t);
                    V u = ihm[e] * (cc[e] - km[e]);
                    u = vfma<V>(ihk[e], cc[e] - kp[e], u);
                    ap[e] = ve[e] ? vfma<V>(dph[e], t, (V)r_.pq * u) : V(0);
                }
                if constexpr (MODE == kApply) {
                    if (row_on) store2(gout, i, j, ap[0], ap[1]);
                } else if constexpr (MODE == kResidual) {
                    V res[2];
#pragma unroll
                    for (int e = 0; e < 2; ++e) {
                        const double bval = (i == 0 && ve[e] && row_on) ? gbp[CHK((long long)min(j, nt - 1) * g.pitch + (e ? kc1 : kc0), (long long)nt * g.pitch)] : 0.0;
                        res[e] = ve[e] ? (V)(bval - (double)ap[e]) : V(0);
                        const V z = res[e] / diag_at<V>(r_, dph[e] + (V)(!ve[e]), ihm[e], ihk[e]);
                        acc0 += wrow * ((double)res[e] * (double)z);
                        acc1 += wrow * ((double)res[e] * (double)res[e]);
                        acc2 += bval * bval;
                    }
                    if (v.store_r && row_on) store2(gout, i, j, res[0], res[1]);
                } else if constexpr (MODE == kUpdateP) {
                    acc0 += wrow * ((double)c0 * (double)ap[0] + (double)c1 * (double)ap[1]);
                } else {  // the r/x update modes
                    const V rr[2] = {rv[m].x, rv[m].y};
                    V xx[2] = {V(0), V(0)};
                    if constexpr (MODE != kUpdateRSkip) {
                        xx[0] = xv[m].x;
                        xx[1] = xv[m].y;
                    }
                    if constexpr (MODE == kUpdateRPair) {   // alpha_{k-1} p_{k-1} first
                        xx[0] = vfma<V>(alpha_p, pv[m].x, xx[0]);
                        xx[1] = vfma<V>(alpha_p, pv[m].y, xx[1]);
                    }
                    V rn[2], xn[2];
#pragma unroll
                    for (int e = 0; e < 2; ++e) {
                        rn[e] = ve[e] ? vfma<V>(-alpha, ap[e], rr[e]) : V(0);
                        xn[e] = ve[e] ? vfma<V>(alpha, cc[e], xx[e]) : V(0);
                        if (!v.zin) {   // with a block preconditioner the line pass takes the sums
                            const V z = rn[e] / diag_at<V>(r_, dph[e] + (V)(!ve[e]), ihm[e], ihk[e]);
                            acc0 += wrow * ((double)rn[e] * (double)z);
                            acc1 += wrow * ((double)rn[e] * (double)rn[e]);
                        }
                    }
                    if (row_on) {
                        store2(gout, i, j, rn[0], rn[1]);
                        if constexpr (MODE != kUpdateRSkip) store2(gout2, i, j, xn[0], xn[1]);
                    }
                }
            }
#pragma unroll
            for (int m = 0; m < M; ++m) {
                q0[m][0] = q1[m][0];
                q0[m][1] = q1[m][1];
                q1[m][0] = q2[m][0];
                q1[m][1] = q2[m][1];
            }
        }
    }

    if constexpr (MODE != kApply) {
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) {
            acc0 += __shfl_xor(acc0, off, kWave);
            acc1 += __shfl_xor(acc1, off, kWave);
            acc2 += __shfl_xor(acc2, off, kWave);
        }
        if (lane == 0) {
            red[w][0] = acc0;
            red[w][1] = acc1;
            red[w][2] = acc2;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
            for (int q = 0; q < kWaves; ++q) {
                s0 += red[q][0];
                s1 += red[q][1];
                s2 += red[q][2];
            }
            gpart[CHK(b, g.nblocks)] = s0;
            gpart[CHK(g.nblocks + b, 3LL * g.nblocks)] = s1;
            gpart[CHK(2 * g.nblocks + b, 3LL * g.nblocks)] = s2;
        }
    }
    if (v.tstamp) {   // timing runs: this workgroup's end
        __syncthreads();
        if (threadIdx.x == 0) atomicMax(&v.tstamp[1], wall_clock64());
    }
}

template <int M, int MODE, typename V>
__global__ void __launch_bounds__(kThreads)
stencil_wave(GridArgs g, StencilVecs<V> v, const RowCoef *__restrict__ rows, const V *__restrict__ vin,
             const V *__restrict__ vpold, V *__restrict__ vout, V *__restrict__ vout2)
{
    wave_body<M, MODE, V>(g, v, rows, vin, vpold, vout, vout2, blockIdx.x);
}

template <int M, int MODE, typename V>
__global__ void __launch_bounds__(kThreads)
stencil_wave_batch(const BatchSlot<V> *__restrict__ slots, int nslots)
{
    const int bid = blockIdx.x;
    const int s = batch_slot(slots, nslots, bid);
    if (s < 0) return;
    const BatchSlot<V> sl = slots[s];
    wave_body<M, MODE, V>(sl.g, sl.v, sl.g.rows, sl.v.in, sl.v.pold, sl.out, sl.v.x, bid - sl.offset);
}

// ---------------------------------------------------------------------------
// One-sweep PCG iteration: the Jacobi-PCG of Sec. 2.3 rearranged so that one
// pass over memory does one iteration (the same iterates in exact arithmetic).
//
// Sweep j (j = 0, 1, ...) computes
//   r_j = r_{j-1} - alpha_{j-1} A p_{j-1}    (r_{j-1} and r_j in two buffers)
//   x_j = x_{j-1} + alpha_{j-1} p_{j-1}      (in place)
//   z_j = D^-1 r_j,   p_j = z_j + beta_j p_{j-1}
//   w_j = A p_j                              (not stored)
// and per-workgroup partial sums of r_j.z_j, r_j.r_j, p_j.w_j, z_j.w_j and
// w_j.D^-1 w_j.  The finisher then has alpha_j = r_j.z_j / p_j.w_j, and as
// r_{j+1} = r_j - alpha_j w_j,
//   r_{j+1}.z_{j+1} = r_j.z_j - 2 alpha_j z_j.w_j + alpha_j^2 w_j.D^-1 w_j,
// which gives beta_{j+1} before r_{j+1} exists.  Sweep 0 runs with
// alpha = beta = 0 and p_{-1} = 0.  Traffic: 48 bytes per unknown per
// iteration (read r, p_old, x; write r, p, x) against 64 for the two passes,
// and one stencil launch and one finisher instead of two of each.
//
// x is needed only at the end, so sweeps can run in pairs that touch it once:
// an even sweep j leaves x_{j-1} as it is, and the odd sweep j + 1 adds both
// increments, alpha_{j-1} p_{j-1} + alpha_j p_j.  It has p_j (its p_old) and
// r_j, hence z_j, and p_j = z_j + beta_j p_{j-1} gives
// p_{j-1} = (p_j - z_j) / beta_j without reading it: 32 + 48 bytes per
// unknown per pair of sweeps instead of 2 x 48, with r and p bitwise as
// before.  z_j is recomputed bitwise (same r_j, same 1/diag), and the
// rebuilt increment carries a rounding error of about
// alpha_{j-1} |p_j| eps / beta_j, so the pairing is kept to
// beta_j >= 1/64; otherwise (and for the restarts, beta = 0) the even sweep
// updates x itself.  After the last sweep of a solve, x may still lack
// alpha_{j-1} p_{j-1}; p_{j-1} is then intact in its buffer, and the first
// workgroup of each sweep records which increment is owed (x_lag).
//
// p_j feeds A p_j on a one-cell ring around each cell, and A p_{j-1} is
// needed on that ring too, so p_{j-1} is read with a two-cell ring.  A
// workgroup owns tj x tk interior (theta, phi) cells over a chunk of radial
// layers and holds them with the ring as a box of 4R rows x 64 lanes
// (tj <= 4R - 4, tk <= 60).  Box row e is polar row j0 - 2 + e; lane c is
// azimuthal cell (k0 - 2 + c) mod np, so periodic phi needs no special case
// and phi neighbours are the neighbouring lanes (DPP shifts).  Wavefront w
// holds box rows [wR, wR + R).  For each layer a of the chunk, and one layer
// beyond each end:
//   stage A, layer a, on the box less its outer ring: A p_{j-1}, r_j, z_j,
//     p_j (p_{j-1} of layers a-1, a, a+1 from LDS planes);
//   stage B, layer a - 1, interior: w_j = A p_j and the dot products (p_j of
//     layers a-2, a-1 from LDS planes, of layer a from registers).
// Each vector has three LDS layer slots in rotation: one barrier per layer.
// The row coefficients of three layers are staged in LDS too, and r, x and
// p_{j-1} of the next layers are loaded one layer ahead.  The coefficients
// are loaded a step before they are written to LDS: a vector-memory wait
// covers every load issued before it, so writing them in the step that loads
// them would wait for that step's other loads too.
// ---------------------------------------------------------------------------
// Reciprocal of a positive normal value: the hardware estimate refined by
// two Newton steps y <- y + y (1 - d y), each of which squares the relative
// error (within about an ulp of 1/d).
__device__ __forceinline__ double recip(double d)
{
    double y = __builtin_amdgcn_rcp(d);
    double e = __builtin_fma(-d, y, 1.0);
    y = __builtin_fma(y, e, y);
    e = __builtin_fma(-d, y, 1.0);
    return __builtin_fma(y, e, y);
}
// FP32: the estimate and one Newton step (about an ulp; the IEEE division
// is three times the instructions).  Both sweeps of a pair use it, so the
// odd sweep recomputes the even sweep's z bitwise.
__device__ __forceinline__ float recip(float d)
{
    const float y = __builtin_amdgcn_rcpf(d);
    return __builtin_fmaf(y, __builtin_fmaf(-d, y, 1.0f), y);
}

// Lane l receives lane l-1 (shr) or l+1 (shl); the lane past the wavefront's
// end receives 0 (DPP bound control: no initialised destination needed).
__device__ __forceinline__ double shr1(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x138, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x138, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double shl1(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x130, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x130, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float shr1(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ float shl1(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xF, 0xF, true));
}

// Element at a 32-bit byte offset from a vector's base: the access takes the
// base in scalar registers and a 32-bit offset per lane.  (The one-sweep
// path is used for vectors under 4 GiB.)
template <typename T>
__device__ __forceinline__ GPtr<T> at_byte(GPtr<T> base, unsigned boff)
{
    using C = typename std::conditional<std::is_const<T>::value, const char, char>::type;
    return (GPtr<T>)((__attribute__((address_space(1))) C *)base + boff);
}
#ifdef POT3D_CHECKED
#define SWEEP_AT(base, boff) ((base) + CHK((boff) / sizeof(V), g.npad))
#else
#define SWEEP_AT(base, boff) at_byte((base), (boff))
#endif

// Whether an even sweep running with alpha_{j-1}, beta_j leaves its x
// increment to the odd sweep after it (which tests the same values).
__device__ __forceinline__ bool defer_x(double alpha_prev, double beta)
{
    return alpha_prev == 0.0 || (beta >= 1.0 / 64.0 && isfinite(beta));
}

// LDS of the sweep, one object per (R, V): kernels that inline the body
// twice (the two x modes of an even sweep) share it.
template <int R, typename V>
struct alignas(16) SweepLds {   // 16: the coefficient rows are read 16 bytes at a time
    alignas(16) V lp[3][kWaves * R][kWave];     // p_{j-1} of three layers
    alignas(16) V lq[3][kWaves * R][kWave];     // p_j of three layers
    alignas(16) V lc[3][kWaves * R][8];         // row coefficients of three layers, converted to V
    double red[kWaves][5];
};
template <int R, typename V>
__device__ __forceinline__ SweepLds<R, V> &sweep_lds()
{
    __shared__ SweepLds<R, V> lds;
    return lds;
}

template <int R, typename V, int XM>
__device__ __forceinline__ void sweep_body(const GridArgs &g, const SweepVecs<V> &v, const RowCoef *__restrict__ rows,
                                           const V *__restrict__ rin, V *__restrict__ rout, const V *__restrict__ pold,
                                           V *__restrict__ pnew, V *__restrict__ xvec, const int b)
{
    constexpr int ER = kWaves * R;
    SweepLds<R, V> &lds = sweep_lds<R, V>();
    auto &lp = lds.lp;
    auto &lq = lds.lq;
    auto &lc = lds.lc;
    auto &red = lds.red;
    static_assert(ER * 8 <= kThreads, "coefficient staging");

    const CPtr<const DevScalars> csc = to_const(v.sc);
    if (!v.ignore_done && csc->done) return;   // uniform over the workgroup
    if (v.tstamp && threadIdx.x == 0) atomicMin(&v.tstamp[0], wall_clock64());

    const GPtr<const V> grin = to_global(rin), gpold = to_global(pold);
    const GPtr<V> grout = to_global(rout), gpnew = to_global(pnew), gx = to_global(xvec);
    const GPtr<const double> gdphi = to_global(g.dphi), gih = to_global(g.ih);
    const GPtr<double> gpart = to_global(v.partial);

    // Workgroup -> tile, XCD-aware as in march_body, with the radial chunk
    // outermost: an XCD's range of workgroups then covers twice as many polar
    // tile rows of one chunk, so fewer tiles have their polar neighbours (whose
    // rings they read) in another XCD's L2.
    const int per = g.nblocks / kXcds;
    int L = (b < per * kXcds) ? (b % kXcds) * per + b / kXcds : b;
    if (g.reverse) L = g.nblocks - 1 - L;
    const int kt = L % g.ntk;
    L /= g.ntk;
    const int jt = L % g.ntj;
    const int ic = L / g.ntj;
    const int nt = g.nt, np = g.np, nr = g.nr;
    const int i0 = ic * g.ci;
    const int i1 = min(i0 + g.ci, nr);
    const int j0 = jt * g.tj;
    const int k0 = kt * g.tk;
    const int tjn = min(g.tj, nt - j0);   // interior rows of this tile
    const int tkn = min(g.tk, np - k0);   // interior cells of a row

    const int lane = threadIdx.x & (kWave - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    // This lane's azimuthal cell; lanes past the box's right ring repeat its
    // last cell (their values are never used).
    int kk = (k0 - 2 + min(lane, tkn + 3)) % np;
    if (kk < 0) kk += np;
    const bool col_in = lane >= 2 && lane < tkn + 2;    // interior cell
    const V dph = (V)gdphi[CHK(kk, np)];
    const V ihm = (V)gih[CHK(kk == 0 ? np - 1 : kk - 1, np)];
    const V ihk = (V)gih[CHK(kk, np)];
    const V ihs = ihm + ihk;   // the phi part of the diagonal, / pq
    const V alpha = (V)csc->alpha, beta = (V)csc->beta;
    // x pairing: an even sweep leaves x alone (xskip; the kernel has chosen
    // this body only if defer_x holds); the odd sweep after it adds
    // xc (p_{j-1} - z_{j-1}) with xc = alpha_{j-2} / beta_{j-1}.
    constexpr bool xskip = XM == 1;
    V xc = V(0);
    if (XM == 2) {
        const double ap = csc->alpha_prev, bp = csc->beta_prev;
        if (ap != 0.0 && defer_x(ap, bp)) xc = (V)(ap / bp);
    }
    if (b == 0 && threadIdx.x == 0) {   // the increment x lacks if this is the last sweep
        v.sc->x_lag = xskip ? csc->alpha : 0.0;
        v.sc->x_lag_p = xskip ? (unsigned long long)pold : 0ull;
    }

    // Per lane: the byte offset of the cell within a layer for each of this
    // wavefront's box rows (rows outside the grid read the nearest grid row),
    // and whether the row is interior.  Values read outside the grid, or
    // computed from such values, only ever meet zero weights: the pole rows
    // have no theta coupling across the pole and the radial boundary rows none
    // outside the shell, so they need no masking.
    const int e0 = w * R;
    unsigned vrow[R];
    bool oki[R];
#pragma unroll
    for (int m = 0; m < R; ++m) {
        const int e = e0 + m;
        vrow[m] = (unsigned)(min(max(j0 - 2 + e, 0), nt - 1) * g.pitch + kk) * (unsigned)sizeof(V);
        oki[m] = e >= 2 && e < tjn + 2;
    }
    const unsigned planeb = (unsigned)g.plane * (unsigned)sizeof(V);
    auto layer_b = [&](int a) { return (unsigned)min(max(a, 0), nr - 1) * planeb; };
    auto slot = [](int a) { return (a + 3) % 3; };
    auto load_p = [&](int a, V (&dst)[R]) {
        const unsigned lb = layer_b(a);
#pragma unroll
        for (int m = 0; m < R; ++m) dst[m] = *SWEEP_AT(gpold, lb + vrow[m]);
    };
    // r_{j-1} of layer a; x_{j-1} on the interior of the chunk's own layers
    auto load_rx = [&](int a, V (&rdst)[R], V (&xdst)[R]) {
        const bool own = a >= i0 && a < i1;
        const unsigned lb = layer_b(a);
#pragma unroll
        for (int m = 0; m < R; ++m) {
            rdst[m] = V(0);   // the box's outer ring needs no r
            if (e0 + m >= 1 && e0 + m < tjn + 3) rdst[m] = *SWEEP_AT(grin, lb + vrow[m]);
            xdst[m] = V(0);
            if (!xskip && own && oki[m] && col_in) xdst[m] = stream_load(SWEEP_AT(gx, lb + vrow[m]));
        }
    };
    // Row coefficients of the box rows of one layer, staged in LDS (three
    // layers in rotation) and read back as broadcasts: rm rp tm tp s pq.
    // load_coef returns this thread's value; put_coef writes it a step later,
    // converted once to the vectors' type (FP32 sweeps then read floats and
    // convert nothing per cell).
    auto load_coef = [&](int a) -> double {
        const int t = threadIdx.x;
        double v = 0.0;
        if (t < ER * 8) {
            const int e = t >> 3, f = t & 7;
            const int jc = min(max(j0 - 2 + e, 0), nt - 1);
            const int ac = min(max(a, 0), nr - 1);
            const GPtr<const double> src = to_global(reinterpret_cast<const double *>(rows));
            v = src[CHK(((long long)ac * nt + jc) * 8 + f, 8LL * nr * nt)];
        }
        return v;
    };
    auto put_coef = [&](int a, double v) {
        const int t = threadIdx.x;
        if (t < ER * 8) lc[slot(a)][t >> 3][t & 7] = (V)v;
    };
    struct Coef {
        V rm, rp, tm, tp, s, pq;
    };
    auto coef = [&](int sl, int e) -> Coef {
        return Coef{lc[sl][e][0], lc[sl][e][1], lc[sl][e][2], lc[sl][e][3], lc[sl][e][4], lc[sl][e][5]};
    };
    // 7-point operator at one cell from the centre, radial and theta
    // neighbours; the phi neighbours come from the adjacent lanes.
    auto apply = [&](const Coef &rc, V pc, V pim, V pip, V pjm, V pjp) -> V {
        const V pkm = shr1(pc), pkp = shl1(pc);
        V t = rc.s * pc;
        t = vfma<V>(-rc.rm, pim, t);
        t = vfma<V>(-rc.rp, pip, t);
        t = vfma<V>(-rc.tm, pjm, t);
        t = vfma<V>(-rc.tp, pjp, t);
        V u = ihm * (pc - pkm);
        u = vfma<V>(ihk, pc - pkp, u);
        return vfma<V>(dph, t, rc.pq * u);
    };

    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0, acc4 = 0.0;
    // One layer step: stage A at layer a, stage B at layer a - 1.  rv, xo:
    // r_{j-1}, x_{j-1} of layer a (loaded one step ahead; the next layer's go
    // to rv_n, xo_n).  z1, i1: z_j and 1/diag of layer a - 1 (stage B); this
    // step's go to za, ia.  Each wavefront reads its own rows of the LDS
    // planes at any time (it alone writes them) and other rows only across a
    // barrier.  cq: this thread's coefficient of layer a + 1 (loaded in the
    // step before, written to LDS at this step's end); cq_n receives layer a + 2's.
    // FP32 sweeps load p_{j-1} two layers ahead (pc_: layer a + 2, loaded in
    // the step before; pn2 receives layer a + 3): 2 % off the FP32-refined
    // solve.  FP64 sweeps load it one layer ahead, which measured 1.3 % faster
    // for them (more registers in flight cost them more).
    constexpr bool kPTwoAhead = std::is_same<V, float>::value;
    auto step = [&](int a, V (&rv)[R], V (&xo)[R], V (&rv_n)[R], V (&xo_n)[R], V (&z1)[R], V (&i1_)[R], V (&za)[R],
                    V (&ia)[R], double cq, double &cq_n, V (&pc_)[R], V (&pn2)[R]) {
        const bool own = a >= i0 && a < i1;
        const unsigned lb = layer_b(a);
        const int sa = slot(a), sa1 = slot(a + 1), sb = slot(a - 1), sb2 = slot(a - 2);
        // The next layers' loads are issued at raised wavefront priority, so
        // the SIMD schedules a wavefront that can put requests in flight
        // before those that only compute (FP64 sweeps 221.5 / 298.9 ->
        // 211.1 / 282.1 us at 151 x 301 x 601).
        V pn[R];
        __builtin_amdgcn_s_setprio(3);
        if constexpr (kPTwoAhead) load_p(a + 3, pn2);
        else load_p(a + 2, pn);
        load_rx(a + 1, rv_n, xo_n);
        cq_n = load_coef(a + 2);
        __builtin_amdgcn_s_setprio(0);
        V qa[R];
#pragma unroll
        for (int m = 0; m < R; ++m) {
            const int e = e0 + m;
            const Coef rc = coef(sa, e);
            const V pc = lp[sa][e][lane];
            const V ap = apply(rc, pc, lp[sb][e][lane], lp[sa1][e][lane], lp[sa][max(e - 1, 0)][lane],
                               lp[sa][min(e + 1, ER - 1)][lane]);
            const V rn = vfma<V>(-alpha, ap, rv[m]);
            const V inv = recip(vfma<V>(dph, rc.s, rc.pq * ihs));
            const V zn = rn * inv;
            const V qn = vfma<V>(beta, pc, zn);
            qa[m] = qn;
            za[m] = zn;
            ia[m] = inv;
            lq[sa][e][lane] = qn;
            if (own && oki[m] && col_in) {
                stream_store(SWEEP_AT(grout, lb + vrow[m]), rn);
                stream_store(SWEEP_AT(gpnew, lb + vrow[m]), qn);
                if (!xskip) {
                    V xn = xo[m];
                    if (XM == 2) xn = vfma<V>(xc, pc - rv[m] * inv, xn);   // alpha_{j-2} p_{j-2}
                    stream_store(SWEEP_AT(gx, lb + vrow[m]), vfma<V>(alpha, pc, xn));
                }
                acc0 = __builtin_fma((double)rn, (double)zn, acc0);
                acc1 = __builtin_fma((double)rn, (double)rn, acc1);
            }
        }
        if (a - 1 >= i0) {
#pragma unroll
            for (int m = 0; m < R; ++m) {
                if (!oki[m]) continue;   // uniform
                const int e = e0 + m;
                const Coef rc = coef(sb, e);
                const V qc = lq[sb][e][lane];
                const V wv = apply(rc, qc, lq[sb2][e][lane], qa[m], lq[sb][e - 1][lane], lq[sb][e + 1][lane]);
                if (col_in) {
                    acc2 = __builtin_fma((double)qc, (double)wv, acc2);
                    acc3 = __builtin_fma((double)z1[m], (double)wv, acc3);
                    acc4 = __builtin_fma((double)wv * (double)i1_[m], (double)wv, acc4);
                }
            }
        }
#pragma unroll
        for (int m = 0; m < R; ++m) lp[slot(a + 2)][e0 + m][lane] = kPTwoAhead ? pc_[m] : pn[m];
        put_coef(a + 1, cq);   // slot(a + 1) held layer a - 2, which no stage reads in this step
        __syncthreads();
    };

    V rvA[R], xoA[R], rvB[R], xoB[R], zA[R], iA[R], zB[R], iB[R], pA[R], pB[R];
    put_coef(i0 - 1, load_coef(i0 - 1));
    double cA = load_coef(i0), cB = 0.0;
    load_rx(i0 - 1, rvA, xoA);
    {
        V t0[R], t1[R], t2[R];
        load_p(i0 - 2, t0);
        load_p(i0 - 1, t1);
        load_p(i0, t2);
        if constexpr (kPTwoAhead) load_p(i0 + 1, pA);
#pragma unroll
        for (int m = 0; m < R; ++m) {
            lp[slot(i0 - 2)][e0 + m][lane] = t0[m];
            lp[slot(i0 - 1)][e0 + m][lane] = t1[m];
            lp[slot(i0)][e0 + m][lane] = t2[m];
            zA[m] = iA[m] = V(0);
        }
    }
    __syncthreads();
    int a = i0 - 1;
    for (; a + 1 <= i1; a += 2) {
        step(a, rvA, xoA, rvB, xoB, zA, iA, zB, iB, cA, cB, pA, pB);
        step(a + 1, rvB, xoB, rvA, xoA, zB, iB, zA, iA, cB, cA, pB, pA);
    }
    if (a <= i1) step(a, rvA, xoA, rvB, xoB, zA, iA, zB, iB, cA, cB, pA, pB);

#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        acc0 += __shfl_xor(acc0, off, kWave);
        acc1 += __shfl_xor(acc1, off, kWave);
        acc2 += __shfl_xor(acc2, off, kWave);
        acc3 += __shfl_xor(acc3, off, kWave);
        acc4 += __shfl_xor(acc4, off, kWave);
    }
    if (lane == 0) {
        red[w][0] = acc0;
        red[w][1] = acc1;
        red[w][2] = acc2;
        red[w][3] = acc3;
        red[w][4] = acc4;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        const int q = threadIdx.x;
        double s = 0.0;
#pragma unroll
        for (int u = 0; u < kWaves; ++u) s += red[u][q];
        gpart[CHK((long long)q * g.nblocks + b, 5LL * g.nblocks)] = s;
    }
    if (v.tstamp) {   // timing runs: this workgroup's end
        __syncthreads();
        if (threadIdx.x == 0) atomicMax(&v.tstamp[1], wall_clock64());
    }
}
#undef SWEEP_AT

// An even sweep (XM = 1) whose alpha_{j-1}, beta_j do not allow the
// deferral runs the body that updates x itself.  The choice is made once, at
// the top, between two inlined bodies, so that each keeps exact memory-wait
// counts (loads under a run-time condition would make the compiler's waits
// conservative).
template <int R, typename V, int XM>
__global__ void __launch_bounds__(kThreads)
stencil_sweep(GridArgs g, SweepVecs<V> v, const RowCoef *__restrict__ rows, const V *__restrict__ rin,
              V *__restrict__ rout, const V *__restrict__ pold, V *__restrict__ pnew, V *__restrict__ x)
{
    if (XM == 1) {
        const CPtr<const DevScalars> csc = to_const(v.sc);
        if (!defer_x(csc->alpha, csc->beta)) {
            sweep_body<R, V, 0>(g, v, rows, rin, rout, pold, pnew, x, blockIdx.x);
            return;
        }
    }
    sweep_body<R, V, XM>(g, v, rows, rin, rout, pold, pnew, x, blockIdx.x);
}

// Batched sweeps: slot q owns workgroups [offset, offset + nblocks) of the
// grid and runs exactly the arithmetic of its single-solve launch.
template <int R, typename V, int XM>
__global__ void __launch_bounds__(kThreads)
stencil_sweep_batch(const BatchSweep<V> *__restrict__ slots, int nslots)
{
    const int bid = blockIdx.x;
    const int s = batch_slot(slots, nslots, bid);
    if (s < 0) return;
    const BatchSweep<V> sl = slots[s];
    if (XM == 1) {   // as in stencil_sweep
        const CPtr<const DevScalars> csc = to_const(sl.v.sc);
        if (!defer_x(csc->alpha, csc->beta)) {
            sweep_body<R, V, 0>(sl.g, sl.v, sl.g.rows, sl.v.r_in, sl.v.r_out, sl.v.p_old, sl.v.p_new, sl.v.x,
                                bid - sl.offset);
            return;
        }
    }
    sweep_body<R, V, XM>(sl.g, sl.v, sl.g.rows, sl.v.r_in, sl.v.r_out, sl.v.p_old, sl.v.p_new, sl.v.x, bid - sl.offset);
}

// ---------------------------------------------------------------------------
// Finishers: one workgroup sums the per-workgroup partials in a fixed order
// and advances the scalar state of the iteration.
// ---------------------------------------------------------------------------
constexpr int kFinThreads = 256;

__device__ __forceinline__ void block_sums(const double *partial, int nb, int ncomp, double out[kMaxPartials])
{
    // Fixed order: each thread sums its strided partials, a wavefront
    // butterfly combines the 64 lanes, then the 4 wavefronts in order.  The
    // partials were written by workgroups on every XCD, so each read misses
    // this XCD's L2: a thread issues the loads of kFinLoads strides of every
    // component together and only then adds them, in the same order (the
    // padding zeros leave a sum that starts at +0 unchanged).
    constexpr int kFinLoads = 4;
    __shared__ double sh[kFinThreads / kWave][kMaxPartials];
    const int t = threadIdx.x;
    double acc[kMaxPartials];
#pragma unroll
    for (int c = 0; c < kMaxPartials; ++c) acc[c] = 0.0;
    for (int q0 = t; q0 < nb; q0 += kFinThreads * kFinLoads) {
        double v[kMaxPartials][kFinLoads];
#pragma unroll
        for (int c = 0; c < kMaxPartials; ++c)
#pragma unroll
            for (int u = 0; u < kFinLoads; ++u) {
                const int q = q0 + u * kFinThreads;
                v[c][u] = (c < ncomp && q < nb) ? partial[(long long)c * nb + q] : 0.0;
            }
#pragma unroll
        for (int c = 0; c < kMaxPartials; ++c)
#pragma unroll
            for (int u = 0; u < kFinLoads; ++u) acc[c] += v[c][u];
    }
#pragma unroll
    for (int c = 0; c < kMaxPartials; ++c)
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) acc[c] += __shfl_xor(acc[c], off, kWave);
    if ((t & (kWave - 1)) == 0)
#pragma unroll
        for (int c = 0; c < kMaxPartials; ++c) sh[t / kWave][c] = acc[c];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kMaxPartials; ++c) {
        double v = 0.0;
#pragma unroll
        for (int w = 0; w < kFinThreads / kWave; ++w) v += sh[w][c];
        out[c] = v;
    }
}

__device__ __forceinline__ void finish_body(int which, DevScalars *sc, const double *partial, int nb)
{
    // the start-of-solve and end-of-solve finishers run whatever the done flag says
    const bool always = which == kFinInit || which == kFinTrue || which == kFinOuter || which == kFinInner ||
                        which == kFinResume;
    // The flag is read before the sums (whose loads then need not wait for
    // it) and tested after them; the sums of a finished solve are not used.
    const int done = sc->done;
    double s[kMaxPartials] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const int ncomp = (which == kFinSigma) ? 1
                      : (which == kFinSweep) ? 5
                      : ((which == kFinInit || which == kFinOuter) ? 3 : 2);   // kFinLineInit: 2
    block_sums(partial, nb, ncomp, s);
    if (!always && done) return;
    if (threadIdx.x != 0) return;
    if (which == kFinInit) {
        // After r = b - A x0: rho = r.z, ||b||, first residual check.
        const double bnorm = sqrt(s[2]);
        sc->bb = s[2];
        sc->bnorm = bnorm;
        sc->rr = s[1];
        sc->rho = s[0];
        sc->alpha = 0.0;
        sc->beta = 0.0;
        sc->k = 0;
        sc->sweep = 0;
        sc->zero_solution = 0;
        sc->done = 0;
        sc->status = POT3D_ENOCONV;
        if (!isfinite(bnorm)) {
            sc->relres = NAN;
            sc->status = POT3D_EBREAKDOWN;
            sc->done = 1;
        } else if (bnorm == 0.0) {
            sc->relres = 0.0;
            sc->zero_solution = 1;
            sc->status = POT3D_OK;
            sc->done = 1;
        } else {
            const double rel = sqrt(s[1]) / bnorm;
            sc->relres = rel;
            if (!isfinite(rel)) {
                sc->status = POT3D_EBREAKDOWN;
                sc->done = 1;
            } else if (rel <= sc->tol) {
                sc->status = POT3D_OK;
                sc->done = 1;
            } else if (sc->maxit <= 0) {
                sc->status = POT3D_ENOCONV;
                sc->done = 1;
            }
        }
    } else if (which == kFinSigma) {
        // alpha = rho / p.Ap; a non-positive or non-finite curvature ends the solve.
        // The previous alpha is kept for the r/x update that pairs two iterations.
        const double sigma = s[0];
        sc->sigma = sigma;
        if (!(sigma > 0.0) || !isfinite(sigma)) {
            sc->status = POT3D_EBREAKDOWN;
            sc->done = 1;
        } else {
            sc->alpha_prev = sc->alpha;
            sc->alpha = sc->rho / sigma;
        }
    } else if (which == kFinRho) {
        // After the r update: convergence test, then beta for the next direction.
        const int k = sc->k + 1;
        sc->k = k;
        sc->rr = s[1];
        const double rel = sqrt(s[1]) / sc->bnorm;
        sc->relres = rel;
        if (!isfinite(rel)) {
            sc->status = POT3D_EBREAKDOWN;
            sc->done = 1;
        } else if (rel <= sc->tol) {
            sc->status = POT3D_OK;
            sc->done = 1;
        } else {
            sc->beta = s[0] / sc->rho;
            sc->rho = s[0];
            if (k >= sc->maxit) {
                sc->status = POT3D_ENOCONV;
                sc->done = 1;
            }
        }
    } else if (which == kFinSweep) {
        // After sweep j of the one-sweep iteration (partials: r_j.z_j, r_j.r_j,
        // p_j.w_j, z_j.w_j, w_j.D^-1 w_j).  For j > 0, r_j is the residual of
        // iteration j: convergence test.  Then alpha_j, and beta_{j+1} from the
        // predicted r_{j+1}.z_{j+1}; a prediction that rounding made
        // non-positive restarts the recurrence (beta = 0, a steepest-descent
        // step, which the next sweep's true r.z then corrects).
        const int j = sc->sweep;
        sc->sweep = j + 1;
        bool stop = false;
        if (j > 0) {
            sc->k = j;
            sc->rr = s[1];
            const double rel = sqrt(s[1]) / sc->bnorm;
            sc->relres = rel;
            if (!isfinite(rel)) {
                sc->status = POT3D_EBREAKDOWN;
                stop = true;
            } else if (rel <= sc->tol) {
                sc->status = POT3D_OK;
                stop = true;
            } else if (j >= sc->maxit) {
                sc->status = POT3D_ENOCONV;
                stop = true;
            }
        }
        if (!stop) {
            const double rho = s[0], sigma = s[2];
            sc->rho = rho;
            sc->sigma = sigma;
            if (!(sigma > 0.0) || !isfinite(sigma)) {
                sc->status = POT3D_EBREAKDOWN;
                stop = true;
            } else {
                const double alpha = rho / sigma;
                const double rho_next = fma(alpha * alpha, s[4], fma(-2.0 * alpha, s[3], rho));
                sc->alpha_prev = sc->alpha;
                sc->beta_prev = sc->beta;
                sc->alpha = alpha;
                sc->beta = (rho_next > 0.0 && isfinite(rho_next)) ? rho_next / rho : 0.0;
            }
        }
        if (stop) sc->done = 1;
    } else if (which == kFinLineInit) {
        // Block preconditioner: the start's rho is r.z with z = M^-1 r from the
        // line pass (kFinInit took ||b|| and the first residual test).
        sc->rho = s[0];
    } else if (which == kFinTrue) {  // ||b - A x|| / ||b|| from a residual pass with store_r = 0
        sc->relres_true = (sc->bnorm > 0.0) ? sqrt(s[1]) / sc->bnorm : 0.0;
    } else if (which == kFinOuter) {
        // Outer step of the refinement, after r = b - A x in FP64: test the true
        // residual, and the scale that normalises the FP32 copy of r.
        const double bnorm = sqrt(s[2]);
        const double rnorm = sqrt(s[1]);
        sc->bb = s[2];
        sc->bnorm = bnorm;
        sc->rr = s[1];
        sc->zero_solution = 0;
        sc->done = 0;
        if (!isfinite(bnorm) || !isfinite(rnorm)) {
            sc->relres = NAN;
            sc->status = POT3D_EBREAKDOWN;
            sc->done = 1;
        } else if (bnorm == 0.0) {
            sc->relres = 0.0;
            sc->zero_solution = 1;
            sc->status = POT3D_OK;
            sc->done = 1;
        } else {
            sc->relres = rnorm / bnorm;
            sc->relres_true = sc->relres;
            sc->scale = 1.0 / rnorm;
            if (sc->relres <= sc->tol) {
                sc->status = POT3D_OK;
                sc->done = 1;
            } else {
                sc->status = POT3D_ENOCONV;
            }
        }
    } else {
        // kFinInner: PCG start on the normalised FP32 residual (e = 0, p = 0,
        // r = r32).  kFinResume: the same residual replacement, but the last
        // search direction is kept (rescaled to the new normalisation), and
        // beta = rho_new / rho_prev continues the recurrence; the host leaves
        // 1 / rho_prev (in the new units) in sc->scale.
        const double rnorm = sqrt(s[1]);
        const double beta = (which == kFinResume) ? s[0] * sc->scale : 0.0;
        sc->rho = s[0];
        sc->rr = s[1];
        sc->bb = s[1];
        sc->bnorm = rnorm;
        sc->alpha = 0.0;
        sc->beta = beta;
        sc->k = 0;
        sc->sweep = 0;
        sc->zero_solution = 0;
        sc->relres = 1.0;
        sc->status = POT3D_ENOCONV;
        sc->done = (!(rnorm > 0.0) || !isfinite(rnorm) || sc->maxit <= 0) ? 1 : 0;
        if (!isfinite(rnorm)) sc->status = POT3D_EBREAKDOWN;
    }
}

__global__ void __launch_bounds__(kFinThreads)
finish_kernel(int which, DevScalars *sc, const double *partial, int nb)
{
    finish_body(which, sc, partial, nb);
}

// Batched finisher: workgroup q advances the scalars of slot q.
__global__ void __launch_bounds__(kFinThreads)
finish_batch(int which, const BatchFin *__restrict__ fins, int nslots)
{
    const int q = blockIdx.x;
    if (q >= nslots || !fins[q].active) return;
    finish_body(which, fins[q].sc, fins[q].partial, fins[q].nb);
}

// ---------------------------------------------------------------------------
// phi-line block preconditioner: z = M^-1 r, where M keeps, for every (i, j)
// row, the diagonal of A and its two periodic azimuthal weights, and drops
// every coupling between rows (a stronger preconditioner than the point
// Jacobi of Sec. 2.3: near the poles the azimuthal weights, which carry
// 1 / sin(theta), dominate the diagonal).
//
// On a uniform phi grid the block of row (i, j) is the circulant
//     d I - w (S + S^-1),   w = pq / dphi,   d = dphi s + 2 w
// (S: the periodic shift by one cell), which factors as
//     (w / mu) (I - mu S) (I - mu S^-1),   mu + 1/mu = d / w,  0 < mu < 1.
// So z = (mu / w) v with two first-order periodic recurrences
//     u_k = r_k + mu u_{k-1},     v_k = u_k + mu v_{k+1}        (k mod np).
// With d / (2 w) = 1 + e, mu = 1 / (1 + e + sqrt(e (2 + e))), free of
// cancellation for small e (pole rows) and large e alike.
//
// One wavefront solves one row.  Lane l owns the run of cells
// [l NB, l NB + n_l), n_l = min(NB, max(0, np - l NB)): the row moves through
// LDS from the coalesced layout (cell 64 q + lane) to these runs and back.
// Each recurrence runs within a lane's run from a zero start, then an
// inclusive scan across the 64 lanes joins the runs: a run is the affine map
// c -> mu^n_l c + E_l (E_l its end value from a zero start), and maps compose
// as (M1, E1) then (M2, E2) = (M1 M2, E1 M2 + E2).  The carry into run l then
// enters its cell t with mu^(t + 1) (forward; mu^(n_l - t) backward).  The
// periodic wrap is closed afterwards: the value that comes round the row is
// the non-periodic end value divided by 1 - mu^np, and it enters every cell
// with its own power of mu (the scan's products give mu^(l NB) and
// mu^(np - (l + 1) NB)).  Every value is FP64; each row reads r once and
// writes z once (16 bytes per unknown in FP64 storage).  Per-workgroup
// partial sums of r.z and r.r follow in fixed order.
// ---------------------------------------------------------------------------
// m^e for an integer e >= 0 by binary powering.
__device__ __forceinline__ double powi(double m, int e)
{
    double r = 1.0;
    while (e > 0) {
        if (e & 1) r *= m;
        m *= m;
        e >>= 1;
    }
    return r;
}

// Orders one wavefront's LDS accesses across lanes (a row moving between
// layouts): release and acquire fences at wavefront scope around a wave barrier.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A double moved across lanes by a DPP row shift (row_shr:n is 0x110 + n,
// row_shl:n is 0x100 + n; rows are 16 lanes).  Lanes whose source lies
// outside their row receive 0.
template <int CTRL>
__device__ __forceinline__ double row_shift(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

// The value of v in lane l (uniform l), as a wave-uniform double.
__device__ __forceinline__ double lane_value(double v, int l)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}

// Inclusive scans of affine maps c -> M c + E across the 64 lanes, without
// LDS: DPP shifts by 1, 2, 4, 8 inside each 16-lane row, then the rows are
// chained through their composites read out of one lane each.  UP: lane l
// ends with the composite of lanes 0..l applied in order, (M1, E1) then
// (M2, E2) = (M1 M2, E1 M2 + E2).  Down: the composite of lanes l..63 with
// the lanes to the right applied first, (M, F) of l then the rest R =
// (M Mr, F + M Fr).
template <bool UP>
__device__ __forceinline__ void affine_scan(double &M, double &E, int lane)
{
    // Branch-free: a DPP read of a lane that is switched off returns 0, so the
    // shifts must run with every lane on.  A source outside the row reads
    // (0, 0), which the step turns into the identity (1, 0) by adding 1 to M.
    const int rl = lane & 15, row = lane >> 4;
    auto step = [&](double Mo, double Eo, bool ok) {
        E = __builtin_fma(Eo, M, E);
        M = (Mo + (ok ? 0.0 : 1.0)) * M;
    };
    if (UP) {
        { const double Mo = row_shift<0x111>(M), Eo = row_shift<0x111>(E); step(Mo, Eo, rl >= 1); }
        { const double Mo = row_shift<0x112>(M), Eo = row_shift<0x112>(E); step(Mo, Eo, rl >= 2); }
        { const double Mo = row_shift<0x114>(M), Eo = row_shift<0x114>(E); step(Mo, Eo, rl >= 4); }
        { const double Mo = row_shift<0x118>(M), Eo = row_shift<0x118>(E); step(Mo, Eo, rl >= 8); }
        // rows: prefix composites of rows 0, 0-1, 0-2 from lanes 15, 31, 47
        const double m0 = lane_value(M, 15), e0 = lane_value(E, 15);
        const double m1 = lane_value(M, 31), e1 = lane_value(E, 31);
        const double m2 = lane_value(M, 47), e2 = lane_value(E, 47);
        const double p1m = m0 * m1, p1e = __builtin_fma(e0, m1, e1);     // rows 0-1
        const double p2m = p1m * m2, p2e = __builtin_fma(p1e, m2, e2);   // rows 0-2
        const double pm = row == 0 ? 1.0 : row == 1 ? m0 : row == 2 ? p1m : p2m;
        const double pe = row == 0 ? 0.0 : row == 1 ? e0 : row == 2 ? p1e : p2e;
        E = __builtin_fma(pe, M, E);
        M = pm * M;
    } else {
        { const double Mo = row_shift<0x101>(M), Eo = row_shift<0x101>(E); step(Mo, Eo, rl + 1 < 16); }
        { const double Mo = row_shift<0x102>(M), Eo = row_shift<0x102>(E); step(Mo, Eo, rl + 2 < 16); }
        { const double Mo = row_shift<0x104>(M), Eo = row_shift<0x104>(E); step(Mo, Eo, rl + 4 < 16); }
        { const double Mo = row_shift<0x108>(M), Eo = row_shift<0x108>(E); step(Mo, Eo, rl + 8 < 16); }
        // rows: suffix composites of rows 3, 2-3, 1-3 from lanes 48, 32, 16
        const double m3 = lane_value(M, 48), e3 = lane_value(E, 48);
        const double m2 = lane_value(M, 32), e2 = lane_value(E, 32);
        const double m1 = lane_value(M, 16), e1 = lane_value(E, 16);
        const double s2m = m2 * m3, s2e = __builtin_fma(m2, e3, e2);     // rows 2-3
        const double s1m = m1 * s2m, s1e = __builtin_fma(m1, s2e, e1);   // rows 1-3
        const double sm = row == 3 ? 1.0 : row == 2 ? m3 : row == 1 ? s2m : s1m;
        const double se = row == 3 ? 0.0 : row == 2 ? e3 : row == 1 ? s2e : s1e;
        E = __builtin_fma(se, M, E);
        M = sm * M;
    }
}

// The value at position n - 1 of a register array (0 for n = 0), by a
// chain of selects (the index is per lane).
template <int NB>
__device__ __forceinline__ double t_end(const double (&u)[NB], int n)
{
    double v = 0.0;
#pragma unroll
    for (int t = 0; t < NB; ++t) v = (t == n - 1) ? u[t] : v;
    return v;
}

// NB = cells per lane's run, ceil(np / 64) (np in (64 (NB - 1), 64 NB]).  V is
// the storage type of r and z (FP64, or FP32 for the inner iterations of the
// refined mode); the recurrences always run in FP64.  LDS: one row per
// wavefront, cell k at k + k / NB (one slot of padding per run, so that the
// lanes' strided run accesses spread over the banks).
template <int NB, typename V>
__global__ void __launch_bounds__(kThreads)
line_solve_kernel(GridArgs g, const V *__restrict__ rin, V *__restrict__ zout, double *__restrict__ partial,
                  const DevScalars *__restrict__ sc, int ignore_done)
{
    const CPtr<const DevScalars> csc = to_const(sc);
    if (!ignore_done && csc->done) return;   // uniform over the workgroup
    constexpr int kRowSlots = NB * kWave + kWave;
    __shared__ double rowbuf[kWaves][kRowSlots];
    __shared__ double red[kWaves][2];
    const GPtr<const V> gr = to_global(rin);
    const GPtr<V> gz = to_global(zout);
    const CPtr<const RowCoef> crows = to_const(g.rows);
    const int np = g.np;
    const int lane = threadIdx.x & (kWave - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    double *const row = rowbuf[w];
    const int n_l = min(NB, max(0, np - lane * NB));   // cells of this lane's run
    const int run0 = lane * (NB + 1);                  // LDS slot of the run's first cell
    const int last_lane = (np - 1) / NB;               // the lane that holds cell np - 1
    const double dph = to_global(g.dphi)[0];           // uniform phi: every width is 2 pi / np
    const double ih = to_global(g.ih)[0];
    const long long nrows = (long long)g.nr * g.nt;
    double acc_rz = 0.0, acc_rr = 0.0;

    // r of a row, coalesced (cell 64 q + lane), into registers (storage type)
    auto load_r = [&](long long rw, V (&rq)[NB]) {
        const long long base = rw * g.pitch;
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int k = q * kWave + lane;
            rq[q] = k < np ? stream_load(gr + CHK(base + k, g.npad)) : V(0);
        }
    };
    // FP32 storage: the next row's r is loaded under this row's work (the
    // registers it takes leave the occupancy unchanged there; in FP64 they
    // would cost a wavefront per SIMD at 601 cells)
    constexpr bool kPrefetch = sizeof(V) == 4;
    const long long rstride = (long long)gridDim.x * kWaves;
    V rq[NB];
    long long rw = (long long)blockIdx.x * kWaves + w;
    if (kPrefetch && rw < nrows) load_r(rw, rq);
    for (; rw < nrows; rw += rstride) {
        const RowCoef rc = load_row(crows, CHK(rw, nrows));
        const long long base = rw * g.pitch;
        if (!kPrefetch) load_r(rw, rq);
        // r into LDS, then each lane's run into registers
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int k = q * kWave + lane;
            if (k < np) row[CHK(k + k / NB, kRowSlots)] = (double)rq[q];
        }
        if (kPrefetch && rw + rstride < nrows) load_r(rw + rstride, rq);
        wave_sync();
        double rv[NB], u[NB];
#pragma unroll
        for (int t = 0; t < NB; ++t) rv[t] = t < n_l ? row[CHK(run0 + t, kRowSlots)] : 0.0;
        wave_sync();

        const double wgt = rc.pq * ih;                       // azimuthal weight w
        const double e = dph * rc.s / (2.0 * wgt);           // d / (2 w) - 1 > 0
        const double mu = 1.0 / (1.0 + e + sqrt(e * (2.0 + e)));
        const double inv_wrap = 1.0 / (1.0 - powi(mu, np)); // 1 / (1 - mu^np)
        const double m_run = powi(mu, n_l);                  // mu^n_l (1 for an empty run)

        // forward: u_k = r_k + mu u_{k-1}; the run from a zero start
        double acc = 0.0;
#pragma unroll
        for (int t = 0; t < NB; ++t) {
            acc = __builtin_fma(mu, acc, rv[t]);
            u[t] = acc;
        }
        double M = m_run, E = t_end(u, n_l);
        affine_scan<true>(M, E, lane);
        // carry into this run (u at cell l NB - 1, non-periodic) and mu^(l NB)
        // (lane 0 reads 0 for both; branch-free, as in affine_scan)
        const double C = shr1(E);
        const double B = shr1(M) + (lane == 0 ? 1.0 : 0.0);
        const double ulast = lane_value(E, last_lane);      // u_{np-1}, non-periodic
        {
            const double cin = __builtin_fma(B, ulast * inv_wrap, C);   // carry plus the wrap
            double pw = mu;
#pragma unroll
            for (int t = 0; t < NB; ++t) {
                u[t] = t < n_l ? __builtin_fma(pw, cin, u[t]) : 0.0;
                pw *= mu;
            }
        }
        // backward: v_k = u_k + mu v_{k+1}; the run from a zero end
        acc = 0.0;
#pragma unroll
        for (int t = NB - 1; t >= 0; --t) {
            acc = __builtin_fma(mu, acc, u[t]);
            u[t] = acc;
        }
        M = m_run;
        double F = u[0];
        affine_scan<false>(M, F, lane);
        // v at cell (l + 1) NB (non-periodic) and mu^(np - (l + 1) NB)
        // (lane 63 reads 0 for both; branch-free)
        const double D = shl1(F);
        const double T = shl1(M) + (lane == kWave - 1 ? 1.0 : 0.0);
        const double v0 = lane_value(F, 0);                 // v_0, non-periodic
        const double scale = mu / wgt;
        {
            const double din = __builtin_fma(T, v0 * inv_wrap, D);   // carry plus the wrap
            double pw = mu;
#pragma unroll
            for (int t = NB - 1; t >= 0; --t) {
                if (t < n_l) {
                    const double z = scale * __builtin_fma(pw, din, u[t]);
                    u[t] = z;
                    acc_rz = __builtin_fma(rv[t], z, acc_rz);
                    acc_rr = __builtin_fma(rv[t], rv[t], acc_rr);
                    pw *= mu;
                }
            }
        }
        // z back through LDS to the coalesced layout
#pragma unroll
        for (int t = 0; t < NB; ++t)
            if (t < n_l) row[CHK(run0 + t, kRowSlots)] = u[t];
        wave_sync();
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int k = q * kWave + lane;
            if (k < np) stream_store(gz + CHK(base + k, g.npad), (V)row[CHK(k + k / NB, kRowSlots)]);
        }
        wave_sync();
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        acc_rz += __shfl_xor(acc_rz, off, kWave);
        acc_rr += __shfl_xor(acc_rr, off, kWave);
    }
    if (lane == 0) {
        red[w][0] = acc_rz;
        red[w][1] = acc_rr;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < kWaves; ++q) t += red[q][threadIdx.x];
        to_global(partial)[CHK((long long)threadIdx.x * gridDim.x + blockIdx.x, 2LL * gridDim.x)] = t;
    }
}

// Point Jacobi, z = D^-1 r over the padded layout (padding stays zero).
__global__ void __launch_bounds__(256)
jacobi_kernel(GridArgs g, const double *__restrict__ r, double *__restrict__ z)
{
    const long long nrows = (long long)g.nr * g.nt;
    const CPtr<const RowCoef> crows = to_const(g.rows);
    const GPtr<const double> gdphi = to_global(g.dphi), gih = to_global(g.ih);
    for (long long row = blockIdx.x; row < nrows; row += gridDim.x) {
        const RowCoef rc = load_row(crows, CHK(row, nrows));
        for (int k = threadIdx.x; k < g.np; k += blockDim.x) {
            const double d = diag_at<double>(rc, gdphi[CHK(k, g.np)], gih[CHK(k == 0 ? g.np - 1 : k - 1, g.np)],
                                             gih[CHK(k, g.np)]);
            const long long o = CHK(row * g.pitch + k, g.npad);
            z[o] = r[o] / d;
        }
    }
}

hipError_t launch_jacobi(const GridArgs &g, const double *r, double *z, hipStream_t s)
{
    const long long nrows = (long long)g.nr * g.nt;
    jacobi_kernel<<<(unsigned)std::min<long long>(nrows, 65536), 256, 0, s>>>(g, r, z);
    return hipGetLastError();
}

template <int NB, typename V>
static hipError_t launch_line_nb(int nb, const GridArgs &g, const V *r, V *z, double *partial, int nblocks,
                                 const DevScalars *sc, int ignore_done, hipStream_t s)
{
    if constexpr (NB > 1) {
        if (nb < NB) return launch_line_nb<NB - 1, V>(nb, g, r, z, partial, nblocks, sc, ignore_done, s);
    }
    line_solve_kernel<NB, V><<<nblocks, kThreads, 0, s>>>(g, r, z, partial, sc, ignore_done);
    return hipGetLastError();
}

template <typename V>
hipError_t launch_line(const GridArgs &g, const V *r, V *z, double *partial, int nblocks, const DevScalars *sc,
                       int ignore_done, hipStream_t s)
{
    const int nb = (g.np + kWave - 1) / kWave;
    if (nb < 1 || nb > kMaxLineCells / kWave) return hipErrorInvalidValue;
    return launch_line_nb<kMaxLineCells / kWave, V>(nb, g, r, z, partial, nblocks, sc, ignore_done, s);
}
template hipError_t launch_line<double>(const GridArgs &, const double *, double *, double *, int,
                                        const DevScalars *, int, hipStream_t);
template hipError_t launch_line<float>(const GridArgs &, const float *, float *, double *, int, const DevScalars *,
                                       int, hipStream_t);

template <int NB, typename V>
static int line_blocks_per_cu_nb(int nb)
{
    if constexpr (NB > 1) {
        if (nb < NB) return line_blocks_per_cu_nb<NB - 1, V>(nb);
    }
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void *>(&line_solve_kernel<NB, V>),
                                                     kThreads, 0) != hipSuccess)
        return 0;
    return n;
}

template <typename V>
int line_blocks_per_cu(int np)
{
    const int nb = (np + kWave - 1) / kWave;
    if (nb < 1 || nb > kMaxLineCells / kWave) return 0;
    return line_blocks_per_cu_nb<kMaxLineCells / kWave, V>(nb);
}
template int line_blocks_per_cu<double>(int);
template int line_blocks_per_cu<float>(int);

// ---------------------------------------------------------------------------
// Refinement helpers (pointwise over the padded arrays; padding stays zero).
// ---------------------------------------------------------------------------
__global__ void cast_residual_kernel(const double *r64, float *r32, float *e32, float *p32, long long n,
                                     const DevScalars *sc)
{
    const double scale = sc->scale;
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
        r32[q] = (float)(r64[q] * scale);
        e32[q] = 0.0f;
        p32[q] = 0.0f;
    }
}

// Reliable update of the FP32 inner iteration: the true residual replaces the
// recursive one, the correction restarts from zero, and the last search
// direction continues in the new units (pdst = f psrc; the two may alias).
__global__ void resume_residual_kernel(const double *r64, float *r32, float *e32, const float *psrc, float *pdst,
                                       long long n, const DevScalars *sc, float f)
{
    const double scale = sc->scale;
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
        r32[q] = (float)(r64[q] * scale);
        e32[q] = 0.0f;
        pdst[q] = f * psrc[q];
    }
}

// After the last sweep of a solve in which x is updated every other sweep:
// x += x_lag p_{j-1}, if the last sweep left that increment (see the
// one-sweep iteration).  Grid cells only (k < np).
template <typename V>
__global__ void x_catchup_kernel(V *x, const DevScalars *sc, long long nrows, int np, int pitch, long long npad)
{
    const double a = sc->x_lag;
    if (a == 0.0) return;
    const V *p = reinterpret_cast<const V *>(sc->x_lag_p);
    const V av = (V)a;
    const long long n = nrows * np;
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
        const long long row = q / np;
        const long long o = row * pitch + (q - row * np);
        x[CHK(o, npad)] = vfma<V>(av, p[CHK(o, npad)], x[CHK(o, npad)]);
    }
}

__global__ void add_correction_kernel(double *x64, const float *e32, long long n, const DevScalars *sc)
{
    const double inv = 1.0 / sc->scale;
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x)
        x64[q] = fma((double)e32[q], inv, x64[q]);
}

// r.z and r.r of an FP32 vector, one workgroup per group of (i, j) rows taken
// in a fixed order, one partial per workgroup.
__global__ void __launch_bounds__(256)
dots_rz_kernel(GridArgs g, const float *r, double *partial, int nblocks)
{
    __shared__ double sh[2][256];
    const int t = threadIdx.x;
    double a0 = 0.0, a1 = 0.0;
    const int nrows = g.nr * g.nt;
    for (int row = blockIdx.x; row < nrows; row += nblocks) {
        const RowCoef rc = g.rows[row];
        const float *rp = r + (long long)row * g.pitch;
        for (int k = t; k < g.np; k += 256) {
            const float dph = (float)g.dphi[k], ihk = (float)g.ih[k];
            const float ihm = (float)g.ih[k == 0 ? g.np - 1 : k - 1];
            const float rv = rp[k];
            const float z = rv / diag_at<float>(rc, dph, ihm, ihk);
            a0 += (double)rv * (double)z;
            a1 += (double)rv * (double)rv;
        }
    }
    sh[0][t] = a0;
    sh[1][t] = a1;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (t < st) {
            sh[0][t] += sh[0][t + st];
            sh[1][t] += sh[1][t + st];
        }
        __syncthreads();
    }
    if (t == 0) {
        partial[blockIdx.x] = sh[0][0];
        partial[nblocks + blockIdx.x] = sh[1][0];
    }
}

// b on the first radial layer: dphi_k * bfac_j * Br(j, k), with
// bfac_j = sin(theta_j) dtheta_j R0^2 (the r = R0 face area over dphi_k).
// b on the first layer; mono (closed wall only, else NULL): [0] the monopole
// of Br to subtract, [1] 1, or 0 when the data are a monopole up to rounding.
__global__ void rhs_kernel(const double *br, const double *bfac, const double *dphi, int nt, int np, int pitch,
                           const double *mono, double *bplane)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (j >= nt || k >= pitch) return;
    double v = 0.0;
    if (k < np) {
        const double b = br[(long long)j * np + k];
        v = mono ? mono[1] * (dphi[k] * bfac[j] * (b - mono[0])) : dphi[k] * bfac[j] * b;
    }
    bplane[(long long)j * pitch + k] = v;
}

// Closed wall (Sec. 2.1, Br = 0 on R1): the system is singular and solvable
// only for data without net flux.  One workgroup, fixed order: the monopole
// of Br, its mean over r = R0 with the face areas dphi_k bfac_j as weights,
// into out[0]; out[1] = 0 if the weighted 2-norm of Br - mean is at most
// 1e-14 of that of Br (a monopole up to rounding: b = 0), else 1.
__global__ void __launch_bounds__(256) monopole_kernel(const double *br, const double *bfac, const double *dphi, int nt,
                                                       int np, double *out)
{
    __shared__ double sh[3][256];
    const int t = threadIdx.x;
    const long long n = (long long)nt * np;
    double num = 0.0, den = 0.0, raw = 0.0;
    for (long long q = t; q < n; q += 256) {
        const int j = (int)(q / np), k = (int)(q % np);
        const double w = dphi[k] * bfac[j];
        const double v = br[q];
        num += w * v;
        den += w;
        raw += (w * v) * (w * v);
    }
    sh[0][t] = num;
    sh[1][t] = den;
    sh[2][t] = raw;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (t < st)
            for (int c = 0; c < 3; ++c) sh[c][t] += sh[c][t + st];
        __syncthreads();
    }
    const double m = sh[0][0] / sh[1][0];
    const double raw_all = sh[2][0];
    __syncthreads();
    double rest = 0.0;
    for (long long q = t; q < n; q += 256) {
        const int j = (int)(q / np), k = (int)(q % np);
        const double w = dphi[k] * bfac[j];
        const double d = w * (br[q] - m);
        rest += d * d;
    }
    sh[0][t] = rest;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (t < st) sh[0][t] += sh[0][t + st];
        __syncthreads();
    }
    if (t == 0) {
        out[0] = m;
        out[1] = (sh[0][0] <= 1e-28 * raw_all) ? 0.0 : 1.0;
    }
}

// Closed wall: Phi is fixed up to a constant; the reported solution has zero
// mean weighted by the cell volumes vr_i vt_j dphi_k (vr = r_i^2 dr_i,
// vt = sin(theta_j) dtheta_j).  Partial sums of the weighted Phi, one
// workgroup per strided set of (i, j) rows in a fixed order.
__global__ void __launch_bounds__(256) gauge_partials_kernel(const double *x, const double *vr, const double *vt,
                                                             const double *dphi, int nr, int nt, int np, int pitch,
                                                             double *partial, int nblocks)
{
    __shared__ double sh[256];
    const int t = threadIdx.x;
    double acc = 0.0;
    const int nrows = nr * nt;
    for (int row = blockIdx.x; row < nrows; row += nblocks) {
        const double w = vr[row / nt] * vt[row % nt];
        const double *xr = x + (long long)row * pitch;
        for (int k = t; k < np; k += 256) acc += w * dphi[k] * xr[k];
    }
    sh[t] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (t < st) sh[t] += sh[t + st];
        __syncthreads();
    }
    if (t == 0) partial[blockIdx.x] = sh[0];
}

// mean = inv_volume * sum of the partials (one workgroup, fixed order) into *out
__global__ void __launch_bounds__(256) gauge_mean_kernel(const double *partial, int nb, double inv_volume, double *out)
{
    __shared__ double sh[256];
    const int t = threadIdx.x;
    double acc = 0.0;
    for (int q = t; q < nb; q += 256) acc += partial[q];
    sh[t] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (t < st) sh[t] += sh[t + st];
        __syncthreads();
    }
    if (t == 0) *out = sh[0] * inv_volume;
}

// The field B = -grad Phi on the cell faces (Sec. 2.1; output layouts
// unpadded, phi fastest), by the operator's differences:
//   Br (nr+1) x nt x np:  r = R0 the surface data (b / (dphi_k bfac_j) on the
//      first layer), inside -(Phi_i - Phi_{i-1}) fr_i, r = R1 Phi_{nr-1} fr_nr
//      (fr_nr = 0 with the closed wall);
//   Bt nr x (nt+1) x np:  -(Phi_j - Phi_{j-1}) ft_j / r_i (ft = 0 on the poles);
//   Bp nr x nt x np (faces k+1/2):  -(Phi_{k+1} - Phi_k) ih_k / (r_i sin(theta_j)).
// fr, ft: inverse centre spacings; rinv = 1 / r_i; sinv = 1 / sin(theta_j).
// One workgroup per output row (a phi row of one component); the row decode
// is uniform and the lanes stream along phi.
__global__ void __launch_bounds__(256) field_kernel(const double *x, const double *bplane, const double *bfac,
                                                    const double *dphi, const double *ih, const double *fr,
                                                    const double *ft, const double *rinv, const double *sinv, int nr,
                                                    int nt, int np, int pitch, double *bfr, double *bft, double *bfp)
{
    const long long rows_r = (long long)(nr + 1) * nt, rows_t = (long long)nr * (nt + 1);
    const long long rows = rows_r + rows_t + (long long)nr * nt;
    const int t = threadIdx.x;
    auto xrow = [&](int i, int j) { return x + ((long long)i * nt + j) * pitch; };
    for (long long row = blockIdx.x; row < rows; row += gridDim.x) {
        if (row < rows_r) {
            const int i = (int)(row / nt), j = (int)(row % nt);
            double *out = bfr + row * np;
            if (i == 0) {
                const double *bp = bplane + (long long)j * pitch;
                const double bj = bfac[j];
                for (int k = t; k < np; k += 256) out[k] = bp[k] / (dphi[k] * bj);
            } else if (i == nr) {
                const double *xa = xrow(nr - 1, j);
                const double f = fr[nr];
                for (int k = t; k < np; k += 256) out[k] = xa[k] * f;
            } else {
                const double *xa = xrow(i, j), *xb = xrow(i - 1, j);
                const double f = fr[i];
                for (int k = t; k < np; k += 256) out[k] = -(xa[k] - xb[k]) * f;
            }
        } else if (row < rows_r + rows_t) {
            const long long u = row - rows_r;
            const int i = (int)(u / (nt + 1)), j = (int)(u % (nt + 1));
            double *out = bft + u * np;
            if (j == 0 || j == nt) {
                for (int k = t; k < np; k += 256) out[k] = 0.0;
            } else {
                const double *xa = xrow(i, j), *xb = xrow(i, j - 1);
                const double f = ft[j] * rinv[i];
                for (int k = t; k < np; k += 256) out[k] = -(xa[k] - xb[k]) * f;
            }
        } else {
            const long long u = row - rows_r - rows_t;
            const int i = (int)(u / nt), j = (int)(u % nt);
            double *out = bfp + u * np;
            const double *xa = xrow(i, j);
            const double f = rinv[i] * sinv[j];
            for (int k = t; k < np; k += 256) {
                const int kp = (k == np - 1) ? 0 : k + 1;
                out[k] = -(xa[kp] - xa[k]) * ih[k] * f;
            }
        }
    }
}

// x -= *mean on the cells (the row padding stays zero)
__global__ void gauge_shift_kernel(double *x, long long nrows, int np, int pitch, const double *mean)
{
    const double m = *mean;
    const long long n = nrows * np;
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
        const long long row = q / np;
        x[row * pitch + (q - row * np)] -= m;
    }
}

template <typename V>
__global__ void fill_kernel(V *p, long long n, V val)
{
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x)
        p[q] = val;
}

// Between the padded layout (rows of `pitch`) and the packed one (rows of np):
// pack = 1: dst[row * np + k] = src[row * pitch + k]; pack = 0: the reverse.
__global__ void repack_kernel(const double *src, double *dst, long long nrows, int np, int pitch, int pack)
{
    const long long n = nrows * np;
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
        const long long row = q / np;
        const long long padded = row * pitch + (q - row * np);
        if (pack) dst[q] = src[padded];
        else dst[padded] = src[q];
    }
}

// Eq. (3) pole values: per radial layer, sum_k dphi_k Phi(i, ring, k) / (2 pi)
// on the rings j = 0 (north) and j = nt-1 (south).  One workgroup per layer.
__global__ void __launch_bounds__(256)
pole_kernel(const double *x, const double *dphi, int nr, int nt, int np, int pitch, double period, double *out)
{
    __shared__ double sh[2][256];
    const int i = blockIdx.x;
    const int t = threadIdx.x;
    double sn = 0.0, ss = 0.0;
    const long long base = (long long)i * nt * pitch;
    for (int k = t; k < np; k += 256) {
        sn += dphi[k] * x[base + k];
        ss += dphi[k] * x[base + (long long)(nt - 1) * pitch + k];
    }
    sh[0][t] = sn;
    sh[1][t] = ss;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (t < st) {
            sh[0][t] += sh[0][t + st];
            sh[1][t] += sh[1][t + st];
        }
        __syncthreads();
    }
    if (t == 0) {
        out[i] = sh[0][0] / period;
        out[nr + i] = sh[1][0] / period;
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
// The vector a pass writes: y (apply), r (residual, update-r), p_new (update-p).
// Passed to the kernels as restrict-qualified pointers with the inputs, so the
// compiler may keep row coefficients in scalar registers and reorder loads.
template <typename V>
static V *out_vector(int mode, const StencilVecs<V> &v)
{
    return mode == kApply ? v.y : (mode == kUpdateP ? v.pnew : v.r);
}

// Launch one stencil kernel; with events, through hipExtLaunchKernelGGL so
// that the events carry the dispatch's own start and end timestamps.
template <typename K, typename V>
static hipError_t launch_kernel(K kern, const GridArgs &g, const StencilVecs<V> &v, V *out, hipStream_t s,
                                hipEvent_t e0, hipEvent_t e1)
{
    const dim3 grid(g.nblocks), block(kThreads);
    if (e0 || e1)
        hipExtLaunchKernelGGL(kern, grid, block, 0, s, e0, e1, 0, g, v, g.rows, v.in, v.pold, out, v.x);
    else
        hipLaunchKernelGGL(kern, grid, block, 0, s, g, v, g.rows, v.in, v.pold, out, v.x);
    return hipGetLastError();
}

template <int TJ, typename V>
static hipError_t launch_tj(int mode, const GridArgs &g, const StencilVecs<V> &v, hipStream_t s, hipEvent_t e0,
                            hipEvent_t e1)
{
    V *out = out_vector(mode, v);
    switch (mode) {
    case kApply: return launch_kernel(stencil_march<TJ, kApply, V>, g, v, out, s, e0, e1);
    case kResidual: return launch_kernel(stencil_march<TJ, kResidual, V>, g, v, out, s, e0, e1);
    case kUpdateP: return launch_kernel(stencil_march<TJ, kUpdateP, V>, g, v, out, s, e0, e1);
    case kUpdateR: return launch_kernel(stencil_march<TJ, kUpdateR, V>, g, v, out, s, e0, e1);
    case kUpdateRSkip: return launch_kernel(stencil_march<TJ, kUpdateRSkip, V>, g, v, out, s, e0, e1);
    case kUpdateRPair: return launch_kernel(stencil_march<TJ, kUpdateRPair, V>, g, v, out, s, e0, e1);
    default: return hipErrorInvalidValue;
    }
}

template <int M, typename V>
static hipError_t launch_wave(int mode, const GridArgs &g, const StencilVecs<V> &v, hipStream_t s, hipEvent_t e0,
                              hipEvent_t e1)
{
    V *out = out_vector(mode, v);
    switch (mode) {
    case kApply: return launch_kernel(stencil_wave<M, kApply, V>, g, v, out, s, e0, e1);
    case kResidual: return launch_kernel(stencil_wave<M, kResidual, V>, g, v, out, s, e0, e1);
    case kUpdateP: return launch_kernel(stencil_wave<M, kUpdateP, V>, g, v, out, s, e0, e1);
    case kUpdateR: return launch_kernel(stencil_wave<M, kUpdateR, V>, g, v, out, s, e0, e1);
    case kUpdateRSkip: return launch_kernel(stencil_wave<M, kUpdateRSkip, V>, g, v, out, s, e0, e1);
    case kUpdateRPair: return launch_kernel(stencil_wave<M, kUpdateRPair, V>, g, v, out, s, e0, e1);
    default: return hipErrorInvalidValue;
    }
}

template <typename V>
hipError_t launch_stencil(int mode, int tile, const GridArgs &g, const StencilVecs<V> &v, hipStream_t s, hipEvent_t e0,
                          hipEvent_t e1)
{
    switch (tile) {
    case kTileMarch8: return launch_tj<8, V>(mode, g, v, s, e0, e1);
    case kTileMarch16: return launch_tj<16, V>(mode, g, v, s, e0, e1);
    case kTileMarch32: return launch_tj<32, V>(mode, g, v, s, e0, e1);
    case kTileWave2: return launch_wave<2, V>(mode, g, v, s, e0, e1);
    case kTileWave4: return launch_wave<4, V>(mode, g, v, s, e0, e1);
    case kTileWave8: return launch_wave<8, V>(mode, g, v, s, e0, e1);
    default: return hipErrorInvalidValue;
    }
}

template <typename V>
static const void *stencil_symbol(int mode, int tile)
{
#define POT3D_SYM(K, T)                                                                                 \
    switch (mode) {                                                                                      \
    case kApply: return reinterpret_cast<const void *>(&K<T, kApply, V>);                                \
    case kResidual: return reinterpret_cast<const void *>(&K<T, kResidual, V>);                          \
    case kUpdateP: return reinterpret_cast<const void *>(&K<T, kUpdateP, V>);                            \
    case kUpdateR: return reinterpret_cast<const void *>(&K<T, kUpdateR, V>);                            \
    case kUpdateRSkip: return reinterpret_cast<const void *>(&K<T, kUpdateRSkip, V>);                    \
    case kUpdateRPair: return reinterpret_cast<const void *>(&K<T, kUpdateRPair, V>);                    \
    default: return nullptr;                                                                             \
    }
    switch (tile) {
    case kTileMarch8: POT3D_SYM(stencil_march, 8)
    case kTileMarch16: POT3D_SYM(stencil_march, 16)
    case kTileMarch32: POT3D_SYM(stencil_march, 32)
    case kTileWave2: POT3D_SYM(stencil_wave, 2)
    case kTileWave4: POT3D_SYM(stencil_wave, 4)
    case kTileWave8: POT3D_SYM(stencil_wave, 8)
    default: return nullptr;
    }
#undef POT3D_SYM
}

template <typename V>
int stencil_blocks_per_cu(int mode, int tile)
{
    const void *f = stencil_symbol<V>(mode, tile);
    int n = 0;
    if (!f || hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, kThreads, 0) != hipSuccess) return 0;
    return n;
}
template int stencil_blocks_per_cu<double>(int, int);
template int stencil_blocks_per_cu<float>(int, int);

template hipError_t launch_stencil<double>(int, int, const GridArgs &, const StencilVecs<double> &, hipStream_t,
                                          hipEvent_t, hipEvent_t);
template hipError_t launch_stencil<float>(int, int, const GridArgs &, const StencilVecs<float> &, hipStream_t,
                                         hipEvent_t, hipEvent_t);

template <int R, typename V>
static void launch_sweep_x(const GridArgs &g, const SweepVecs<V> &v, hipStream_t s)
{
    const dim3 grid(g.nblocks), block(kThreads);
    if (v.xmode == 1) stencil_sweep<R, V, 1><<<grid, block, 0, s>>>(g, v, g.rows, v.r_in, v.r_out, v.p_old, v.p_new, v.x);
    else if (v.xmode == 2) stencil_sweep<R, V, 2><<<grid, block, 0, s>>>(g, v, g.rows, v.r_in, v.r_out, v.p_old, v.p_new, v.x);
    else stencil_sweep<R, V, 0><<<grid, block, 0, s>>>(g, v, g.rows, v.r_in, v.r_out, v.p_old, v.p_new, v.x);
}

template <typename V>
hipError_t launch_sweep(int rows, const GridArgs &g, const SweepVecs<V> &v, hipStream_t s)
{
    if (v.xmode < 0 || v.xmode > 2) return hipErrorInvalidValue;
    switch (rows) {
    case 4: launch_sweep_x<4, V>(g, v, s); break;
    case 6: launch_sweep_x<6, V>(g, v, s); break;
    case 8: launch_sweep_x<8, V>(g, v, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
template hipError_t launch_sweep<double>(int, const GridArgs &, const SweepVecs<double> &, hipStream_t);
template hipError_t launch_sweep<float>(int, const GridArgs &, const SweepVecs<float> &, hipStream_t);

template <typename V>
int sweep_blocks_per_cu(int rows)
{
    const void *f = rows == 4   ? reinterpret_cast<const void *>(&stencil_sweep<4, V, 2>)
                    : rows == 6 ? reinterpret_cast<const void *>(&stencil_sweep<6, V, 2>)
                    : rows == 8 ? reinterpret_cast<const void *>(&stencil_sweep<8, V, 2>)
                                : nullptr;
    int n = 0;
    if (!f || hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, kThreads, 0) != hipSuccess) return 0;
    return n;
}
template int sweep_blocks_per_cu<double>(int);
template int sweep_blocks_per_cu<float>(int);

template <int R, typename V>
static void launch_sweep_batch_x(const BatchSweep<V> *slots, int nslots, int total_blocks, int xmode, hipStream_t s)
{
    const dim3 grid(total_blocks), block(kThreads);
    if (xmode == 1) stencil_sweep_batch<R, V, 1><<<grid, block, 0, s>>>(slots, nslots);
    else if (xmode == 2) stencil_sweep_batch<R, V, 2><<<grid, block, 0, s>>>(slots, nslots);
    else stencil_sweep_batch<R, V, 0><<<grid, block, 0, s>>>(slots, nslots);
}

template <typename V>
hipError_t launch_sweep_batch(int rows, const BatchSweep<V> *slots, int nslots, int total_blocks, int xmode,
                              hipStream_t s)
{
    if (total_blocks <= 0) return hipSuccess;
    if (xmode < 0 || xmode > 2) return hipErrorInvalidValue;
    switch (rows) {
    case 4: launch_sweep_batch_x<4, V>(slots, nslots, total_blocks, xmode, s); break;
    case 6: launch_sweep_batch_x<6, V>(slots, nslots, total_blocks, xmode, s); break;
    case 8: launch_sweep_batch_x<8, V>(slots, nslots, total_blocks, xmode, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
template hipError_t launch_sweep_batch<double>(int, const BatchSweep<double> *, int, int, int, hipStream_t);
template hipError_t launch_sweep_batch<float>(int, const BatchSweep<float> *, int, int, int, hipStream_t);

template <int TJ, typename V>
hipError_t launch_march_batch(int mode, const BatchSlot<V> *slots, int nslots, dim3 grid, hipStream_t s)
{
    const dim3 block(kThreads);
    switch (mode) {
    case kUpdateP: stencil_march_batch<TJ, kUpdateP, V><<<grid, block, 0, s>>>(slots, nslots); break;
    case kUpdateR: stencil_march_batch<TJ, kUpdateR, V><<<grid, block, 0, s>>>(slots, nslots); break;
    case kUpdateRSkip: stencil_march_batch<TJ, kUpdateRSkip, V><<<grid, block, 0, s>>>(slots, nslots); break;
    case kUpdateRPair: stencil_march_batch<TJ, kUpdateRPair, V><<<grid, block, 0, s>>>(slots, nslots); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int M, typename V>
hipError_t launch_wave_batch(int mode, const BatchSlot<V> *slots, int nslots, dim3 grid, hipStream_t s)
{
    const dim3 block(kThreads);
    switch (mode) {
    case kUpdateP: stencil_wave_batch<M, kUpdateP, V><<<grid, block, 0, s>>>(slots, nslots); break;
    case kUpdateR: stencil_wave_batch<M, kUpdateR, V><<<grid, block, 0, s>>>(slots, nslots); break;
    case kUpdateRSkip: stencil_wave_batch<M, kUpdateRSkip, V><<<grid, block, 0, s>>>(slots, nslots); break;
    case kUpdateRPair: stencil_wave_batch<M, kUpdateRPair, V><<<grid, block, 0, s>>>(slots, nslots); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename V>
hipError_t launch_stencil_batch(int mode, int tile, const BatchSlot<V> *slots, int nslots, int total_blocks,
                                hipStream_t s)
{
    if (total_blocks <= 0) return hipSuccess;
    const dim3 grid(total_blocks);
    switch (tile) {
    case kTileMarch8: return launch_march_batch<8, V>(mode, slots, nslots, grid, s);
    case kTileMarch16: return launch_march_batch<16, V>(mode, slots, nslots, grid, s);
    case kTileMarch32: return launch_march_batch<32, V>(mode, slots, nslots, grid, s);
    case kTileWave2: return launch_wave_batch<2, V>(mode, slots, nslots, grid, s);
    case kTileWave4: return launch_wave_batch<4, V>(mode, slots, nslots, grid, s);
    case kTileWave8: return launch_wave_batch<8, V>(mode, slots, nslots, grid, s);
    default: return hipErrorInvalidValue;
    }
}
template hipError_t launch_stencil_batch<double>(int, int, const BatchSlot<double> *, int, int, hipStream_t);
template hipError_t launch_stencil_batch<float>(int, int, const BatchSlot<float> *, int, int, hipStream_t);

hipError_t launch_finish_batch(int which, const BatchFin *fins, int nslots, hipStream_t s)
{
    finish_batch<<<nslots, kFinThreads, 0, s>>>(which, fins, nslots);
    return hipGetLastError();
}

hipError_t launch_finish(int which, DevScalars *sc, const double *partial, int nb, hipStream_t s, hipEvent_t e0)
{
    if (e0)
        hipExtLaunchKernelGGL(finish_kernel, dim3(1), dim3(kFinThreads), 0, s, e0, nullptr, 0, which, sc, partial, nb);
    else
        finish_kernel<<<1, kFinThreads, 0, s>>>(which, sc, partial, nb);
    return hipGetLastError();
}

hipError_t launch_rhs(const double *br, const double *bfac, const double *dphi, int nt, int np, int pitch,
                      const double *mono, double *bplane, hipStream_t s)
{
    const dim3 grid((pitch + 255) / 256, nt), block(256);
    rhs_kernel<<<grid, block, 0, s>>>(br, bfac, dphi, nt, np, pitch, mono, bplane);
    return hipGetLastError();
}

hipError_t launch_field(const double *x, const double *bplane, const double *bfac, const double *dphi, const double *ih,
                        const double *fr, const double *ft, const double *rinv, const double *sinv, int nr, int nt,
                        int np, int pitch, double *bfr, double *bft, double *bfp, hipStream_t s)
{
    const long long rows = (long long)(nr + 1) * nt + (long long)nr * (nt + 1) + (long long)nr * nt;
    const unsigned grid = (unsigned)std::min<long long>(rows, 1LL << 20);
    field_kernel<<<grid, 256, 0, s>>>(x, bplane, bfac, dphi, ih, fr, ft, rinv, sinv, nr, nt, np, pitch, bfr, bft, bfp);
    return hipGetLastError();
}

hipError_t launch_monopole(const double *br, const double *bfac, const double *dphi, int nt, int np, double *out,
                           hipStream_t s)
{
    monopole_kernel<<<1, 256, 0, s>>>(br, bfac, dphi, nt, np, out);
    return hipGetLastError();
}

hipError_t launch_gauge(double *x, const double *vr, const double *vt, const double *dphi, int nr, int nt, int np,
                        int pitch, double inv_volume, double *partial, int nblocks, double *mean, hipStream_t s)
{
    const int nb = std::max(1, std::min(nblocks, nr * nt));
    gauge_partials_kernel<<<nb, 256, 0, s>>>(x, vr, vt, dphi, nr, nt, np, pitch, partial, nb);
    gauge_mean_kernel<<<1, 256, 0, s>>>(partial, nb, inv_volume, mean);
    gauge_shift_kernel<<<2048, 256, 0, s>>>(x, (long long)nr * nt, np, pitch, mean);
    return hipGetLastError();
}

template <typename V>
hipError_t launch_fill(V *p, long long n, V val, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    long long blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    fill_kernel<V><<<(unsigned)blocks, 256, 0, s>>>(p, n, val);
    return hipGetLastError();
}
template hipError_t launch_fill<double>(double *, long long, double, hipStream_t);
template hipError_t launch_fill<float>(float *, long long, float, hipStream_t);

hipError_t launch_repack(const double *src, double *dst, long long nrows, int np, int pitch, bool pack, hipStream_t s)
{
    const long long n = nrows * np;
    if (n <= 0) return hipSuccess;
    long long blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    repack_kernel<<<(unsigned)blocks, 256, 0, s>>>(src, dst, nrows, np, pitch, pack ? 1 : 0);
    return hipGetLastError();
}

unsigned take_oob_line(hipStream_t s)
{
#ifdef POT3D_CHECKED
    unsigned line = 0;
    if (hipStreamSynchronize(s) != hipSuccess) return ~0u;
    if (hipMemcpyFromSymbol(&line, HIP_SYMBOL(g_oob_line), sizeof(line)) != hipSuccess) return ~0u;
    if (line) {
        const unsigned zero = 0;
        (void)hipMemcpyToSymbol(HIP_SYMBOL(g_oob_line), &zero, sizeof(zero));
    }
    return line;
#else
    (void)s;
    return 0;
#endif
}

bool checked_build()
{
#ifdef POT3D_CHECKED
    return true;
#else
    return false;
#endif
}

static unsigned stream_blocks(long long n)
{
    long long blocks = (n + 255) / 256;
    return (unsigned)std::max<long long>(1, std::min<long long>(blocks, 8192));
}

hipError_t launch_cast_residual(const double *r64, float *r32, float *e32, float *p32, long long npad,
                                const DevScalars *sc, hipStream_t s)
{
    cast_residual_kernel<<<stream_blocks(npad), 256, 0, s>>>(r64, r32, e32, p32, npad, sc);
    return hipGetLastError();
}

hipError_t launch_resume_residual(const double *r64, float *r32, float *e32, const float *psrc, float *pdst,
                                  long long npad, const DevScalars *sc, float f, hipStream_t s)
{
    resume_residual_kernel<<<stream_blocks(npad), 256, 0, s>>>(r64, r32, e32, psrc, pdst, npad, sc, f);
    return hipGetLastError();
}

template <typename V>
hipError_t launch_x_catchup(V *x, const DevScalars *sc, int nr, int nt, int np, int pitch, hipStream_t s)
{
    const long long nrows = (long long)nr * nt, npad = nrows * pitch;
    x_catchup_kernel<V><<<stream_blocks(nrows * np), 256, 0, s>>>(x, sc, nrows, np, pitch, npad);
    return hipGetLastError();
}
template hipError_t launch_x_catchup<double>(double *, const DevScalars *, int, int, int, int, hipStream_t);
template hipError_t launch_x_catchup<float>(float *, const DevScalars *, int, int, int, int, hipStream_t);

hipError_t launch_add_correction(double *x64, const float *e32, long long npad, const DevScalars *sc, hipStream_t s)
{
    add_correction_kernel<<<stream_blocks(npad), 256, 0, s>>>(x64, e32, npad, sc);
    return hipGetLastError();
}

hipError_t launch_dots_rz(const GridArgs &g, const float *r, double *partial, int nblocks, hipStream_t s)
{
    dots_rz_kernel<<<nblocks, 256, 0, s>>>(g, r, partial, nblocks);
    return hipGetLastError();
}

hipError_t launch_poles(const double *x, const double *dphi, int nr, int nt, int np, int pitch, double period,
                        double *out, hipStream_t s)
{
    pole_kernel<<<nr, 256, 0, s>>>(x, dphi, nr, nt, np, pitch, period, out);
    return hipGetLastError();
}

}  // namespace pot3d
