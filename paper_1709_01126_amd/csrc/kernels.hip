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

#include <cmath>

namespace pot3d {

template <typename V> __device__ __forceinline__ V vfma(V a, V b, V c);
template <> __device__ __forceinline__ double vfma<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }
template <> __device__ __forceinline__ float vfma<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Diagonal of A at one point (the Jacobi preconditioner).
template <typename V>
__device__ __forceinline__ V diag_at(const RowCoef &rc, V dph, V ihm, V ihk)
{
    return vfma<V>(dph, (V)rc.s, (V)rc.pq * (ihm + ihk));
}

template <int TJ, int MODE, typename V>
__global__ void __launch_bounds__(kThreads)
stencil_march(GridArgs g, StencilVecs<V> v)
{
    static_assert(TJ % kWaves == 0 && 2 * TJ <= kWave, "tile rows");
    constexpr int M = TJ / kWaves;   // rows per wavefront
    constexpr int TK = kWave;
    __shared__ V lds[3][TJ + 2][TK + 2];
    __shared__ double red[kWaves][3];

    if (!v.ignore_done && v.sc->done) return;   // uniform over the workgroup

    // Workgroup -> tile.  Hardware hands consecutive workgroup ids to the 8
    // XCDs in turn; renumber so that each XCD works on a contiguous range of
    // logical tiles (radial chunk fastest) and shares their halos in its L2.
    const int b = blockIdx.x;
    const int per = g.nblocks / kXcds;
    int L = (b < per * kXcds) ? (b % kXcds) * per + b / kXcds : b;
    const int ic = L % g.nchunk;
    L /= g.nchunk;
    const int jt = L % g.ntj;
    const int kt = L / g.ntj;
    const int i0 = ic * g.ci;
    const int i1 = min(i0 + g.ci, g.nr);
    const int j0 = jt * TJ;
    const int k0 = kt * TK;

    const int nt = g.nt, np = g.np;
    const int lane = threadIdx.x & (kWave - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int k = k0 + lane;
    const bool kval = k < np;
    // LDS column of the k+1 neighbour: the last cell of a row wraps to k = 0,
    // which the right halo column holds.
    const int kp_col = (k == np - 1) ? TK + 1 : lane + 2;

    V dph = 0, ihm = 0, ihk = 0;
    if (kval) {
        dph = (V)g.dphi[k];
        ihm = (V)g.ih[k == 0 ? np - 1 : k - 1];
        ihk = (V)g.ih[k];
    }

    // Halo ring of the tile in one layer: wave 0 the row below (j0-1), wave 1
    // the row above (j0+TJ), wave 2 the left and right columns (wrapped in phi).
    int hrow = -1, hcol = 0, hj = 0, hk = 0;
    bool hval = false;
    if (w < 2) {
        hrow = (w == 0) ? 0 : TJ + 1;
        hcol = lane + 1;
        hj = (w == 0) ? j0 - 1 : j0 + TJ;
        hk = k;
        hval = kval && hj >= 0 && hj < nt;
    } else if (w == 2 && lane < 2 * TJ) {
        const bool left = lane < TJ;
        hrow = (left ? lane : lane - TJ) + 1;
        hcol = left ? 0 : TK + 1;
        hj = j0 + hrow - 1;
        hk = left ? (k0 == 0 ? np - 1 : k0 - 1) : (k0 + TK >= np ? 0 : k0 + TK);
        hval = hj < nt;
    }
    V hdph = 0, hihm = 0, hihk = 0;
    if (MODE == kUpdateP && hval) {
        hdph = (V)g.dphi[hk];
        hihm = (V)g.ih[hk == 0 ? np - 1 : hk - 1];
        hihk = (V)g.ih[hk];
    }

    V beta = 0, alpha = 0;
    if (MODE == kUpdateP) beta = (V)v.sc->beta;
    if (MODE == kUpdateR) alpha = (V)v.sc->alpha;

    // Stencil operand at one point: the new search direction for update-p,
    // the input vector otherwise.
    auto operand = [&](int ip, int j, int kk, V pdph, V pihm, V pihk) -> V {
        const long long idx = (long long)ip * g.plane + (long long)j * g.pitch + kk;
        if constexpr (MODE == kUpdateP) {
            const V d = diag_at<V>(g.rows[ip * nt + j], pdph, pihm, pihk);
            return vfma<V>(beta, v.pold[idx], v.in[idx] / d);
        } else {
            return v.in[idx];
        }
    };

    V q0[M], q1[M], q2[M];
    // Evaluate the operand on layer ip for the own points (into dst) and, if
    // to_lds, on the tile plus halo ring into LDS slot `slot`.
    auto produce = [&](int ip, int slot, V (&dst)[M], bool to_lds, bool store) {
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int row = w + kWaves * m;
            const int j = j0 + row;
            V val = 0;
            if (kval && j < nt) {
                val = operand(ip, j, k, dph, ihm, ihk);
                if constexpr (MODE == kUpdateP) {
                    if (store) v.pnew[(long long)ip * g.plane + (long long)j * g.pitch + k] = val;
                }
            }
            dst[m] = val;
            if (to_lds) lds[slot][row + 1][lane + 1] = val;
        }
        if (to_lds && hrow >= 0) lds[slot][hrow][hcol] = hval ? operand(ip, hj, hk, hdph, hihm, hihk) : V(0);
    };

    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;

    if (i0 > 0) {
        produce(i0 - 1, 0, q0, false, false);
    } else {
#pragma unroll
        for (int m = 0; m < M; ++m) q0[m] = 0;
    }
    produce(i0, i0 % 3, q1, true, MODE == kUpdateP);

    for (int i = i0; i < i1; ++i) {
        if (i + 1 < g.nr) {
            produce(i + 1, (i + 1) % 3, q2, true, MODE == kUpdateP && i + 1 < i1);
        } else {
#pragma unroll
            for (int m = 0; m < M; ++m) q2[m] = 0;
        }
        __syncthreads();
        const int s = i % 3;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int row = w + kWaves * m;
            const int j = j0 + row;
            if (kval && j < nt) {
                const RowCoef &rc = g.rows[i * nt + j];
                const V pc = q1[m];
                const V pjm = lds[s][row][lane + 1];
                const V pjp = lds[s][row + 2][lane + 1];
                const V pkm = lds[s][row + 1][lane];
                const V pkp = lds[s][row + 1][kp_col];
                // (A p) = dphi_k (s pc - rm p_{i-1} - rp p_{i+1} - tm p_{j-1} - tp p_{j+1})
                //       + pq (ih_{k-1} (pc - p_{k-1}) + ih_k (pc - p_{k+1}))
                V t = (V)rc.s * pc;
                t = vfma<V>(-(V)rc.rm, q0[m], t);
                t = vfma<V>(-(V)rc.rp, q2[m], t);
                t = vfma<V>(-(V)rc.tm, pjm, t);
                t = vfma<V>(-(V)rc.tp, pjp, t);
                V u = ihm * (pc - pkm);
                u = vfma<V>(ihk, pc - pkp, u);
                const V ap = vfma<V>(dph, t, (V)rc.pq * u);
                const long long idx = (long long)i * g.plane + (long long)j * g.pitch + k;
                if constexpr (MODE == kApply) {
                    v.y[idx] = ap;
                } else if constexpr (MODE == kResidual) {
                    const double bval = (i == 0) ? v.bplane[(long long)j * g.pitch + k] : 0.0;
                    const V res = (V)(bval - (double)ap);
                    if (v.store_r) v.r[idx] = res;
                    const V z = res / diag_at<V>(rc, dph, ihm, ihk);
                    acc0 += (double)res * (double)z;
                    acc1 += (double)res * (double)res;
                    acc2 += bval * bval;
                } else if constexpr (MODE == kUpdateP) {
                    acc0 += (double)pc * (double)ap;
                } else {  // kUpdateR
                    const V rn = vfma<V>(-alpha, ap, v.r[idx]);
                    v.r[idx] = rn;
                    v.x[idx] = vfma<V>(alpha, pc, v.x[idx]);
                    const V z = rn / diag_at<V>(rc, dph, ihm, ihk);
                    acc0 += (double)rn * (double)z;
                    acc1 += (double)rn * (double)rn;
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
            v.partial[b] = s0;
            v.partial[g.nblocks + b] = s1;
            v.partial[2 * g.nblocks + b] = s2;
        }
    }
}

// ---------------------------------------------------------------------------
// Finishers: one workgroup sums the per-workgroup partials in a fixed order
// and advances the scalar state of the iteration.
// ---------------------------------------------------------------------------
constexpr int kFinThreads = 256;

__device__ __forceinline__ void block_sums(const double *partial, int nb, int ncomp, double out[3])
{
    __shared__ double sh[3][kFinThreads];
    const int t = threadIdx.x;
    for (int c = 0; c < ncomp; ++c) {
        double s = 0.0;
        for (int q = t; q < nb; q += kFinThreads) s += partial[(long long)c * nb + q];
        sh[c][t] = s;
    }
    __syncthreads();
    for (int st = kFinThreads / 2; st > 0; st >>= 1) {
        if (t < st)
            for (int c = 0; c < ncomp; ++c) sh[c][t] += sh[c][t + st];
        __syncthreads();
    }
    for (int c = 0; c < ncomp; ++c) out[c] = sh[c][0];
}

__global__ void __launch_bounds__(kFinThreads)
finish_kernel(int which, DevScalars *sc, const double *partial, int nb)
{
    if (which != kFinInit && which != kFinTrue && sc->done) return;
    double s[3] = {0.0, 0.0, 0.0};
    block_sums(partial, nb, which == kFinSigma ? 1 : (which == kFinInit ? 3 : 2), s);
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
        const double sigma = s[0];
        sc->sigma = sigma;
        if (!(sigma > 0.0) || !isfinite(sigma)) {
            sc->status = POT3D_EBREAKDOWN;
            sc->done = 1;
        } else {
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
    } else {  // kFinTrue: ||b - A x|| / ||b|| from a residual pass with store_r = 0
        sc->relres_true = (sc->bnorm > 0.0) ? sqrt(s[1]) / sc->bnorm : 0.0;
    }
}

// b on the first radial layer: dphi_k * bfac_j * Br(j, k), with
// bfac_j = sin(theta_j) dtheta_j R0^2 (the r = R0 face area over dphi_k).
__global__ void rhs_kernel(const double *br, const double *bfac, const double *dphi, int nt, int np, int pitch,
                           double *bplane)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (j >= nt || k >= pitch) return;
    bplane[(long long)j * pitch + k] = (k < np) ? dphi[k] * bfac[j] * br[(long long)j * np + k] : 0.0;
}

template <typename V>
__global__ void fill_kernel(V *p, long long n, V val)
{
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x)
        p[q] = val;
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
template <int TJ, typename V>
static hipError_t launch_tj(int mode, const GridArgs &g, const StencilVecs<V> &v, hipStream_t s)
{
    const dim3 grid(g.nblocks), block(kThreads);
    switch (mode) {
    case kApply: stencil_march<TJ, kApply, V><<<grid, block, 0, s>>>(g, v); break;
    case kResidual: stencil_march<TJ, kResidual, V><<<grid, block, 0, s>>>(g, v); break;
    case kUpdateP: stencil_march<TJ, kUpdateP, V><<<grid, block, 0, s>>>(g, v); break;
    case kUpdateR: stencil_march<TJ, kUpdateR, V><<<grid, block, 0, s>>>(g, v); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename V>
hipError_t launch_stencil(int mode, int tj, const GridArgs &g, const StencilVecs<V> &v, hipStream_t s)
{
    switch (tj) {
    case 8: return launch_tj<8, V>(mode, g, v, s);
    case 16: return launch_tj<16, V>(mode, g, v, s);
    case 32: return launch_tj<32, V>(mode, g, v, s);
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_stencil<double>(int, int, const GridArgs &, const StencilVecs<double> &, hipStream_t);
template hipError_t launch_stencil<float>(int, int, const GridArgs &, const StencilVecs<float> &, hipStream_t);

hipError_t launch_finish(int which, DevScalars *sc, const double *partial, int nb, hipStream_t s)
{
    finish_kernel<<<1, kFinThreads, 0, s>>>(which, sc, partial, nb);
    return hipGetLastError();
}

hipError_t launch_rhs(const double *br, const double *bfac, const double *dphi, int nt, int np, int pitch,
                      double *bplane, hipStream_t s)
{
    const dim3 grid((pitch + 255) / 256, nt), block(256);
    rhs_kernel<<<grid, block, 0, s>>>(br, bfac, dphi, nt, np, pitch, bplane);
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

hipError_t launch_poles(const double *x, const double *dphi, int nr, int nt, int np, int pitch, double period,
                        double *out, hipStream_t s)
{
    pole_kernel<<<nr, 256, 0, s>>>(x, dphi, nr, nt, np, pitch, period, out);
    return hipGetLastError();
}

}  // namespace pot3d
