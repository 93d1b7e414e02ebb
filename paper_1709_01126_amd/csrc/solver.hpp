// solver.hpp -- internal types shared by the HIP kernels and the host driver.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pot3d {

// Tile shape of the stencil kernels: a workgroup of 4 wavefronts owns a
// TJ (polar rows) x 64 (azimuthal cells) column of the grid and walks a chunk of
// radial layers.
constexpr int kWave = 64;
constexpr int kWaves = 4;
constexpr int kThreads = kWave * kWaves;
constexpr int kXcds = 8;   // MI355X: consecutive workgroups go round-robin to 8 XCDs

// Per (i, j) row of the grid: the weights of the volume-scaled operator that
// are constant along phi, in units that the per-k factors complete:
//   W_r-  = dphi_k * rm      W_r+  = dphi_k * rp
//   W_t-  = dphi_k * tm      W_t+  = dphi_k * tp
//   W_p-  = pq / (phi_k - phi_{k-1})   W_p+ = pq / (phi_{k+1} - phi_k)
//   diag  = dphi_k * s + pq * (1/(phi_k - phi_{k-1}) + 1/(phi_{k+1} - phi_k))
// with s = rm + rp + tm + tp + (top layer) D_top / dphi_k.
struct alignas(64) RowCoef {
    double rm, rp, tm, tp, s, pq, pad0, pad1;
};

// Device-resident scalars of one PCG solve.  Kernels read them, so the
// iteration needs no host round trip and can be replayed from a graph.
struct alignas(64) DevScalars {
    double rho;        // r.z of the current residual
    double alpha;      // step length of the current iteration
    double beta;       // rho_k / rho_{k-1} for the next search direction
    double sigma;      // p.Ap
    double rr;         // r.r
    double bnorm;      // ||b||_2
    double relres;     // ||r||_2 / ||b||_2 (recursive)
    double tol;        // stopping tolerance
    double bb;         // b.b
    double relres_true;
    int k;             // iterations done
    int maxit;
    int done;          // 1: all further iteration kernels are no-ops
    int status;        // POT3D_* status once done
    int zero_solution; // ||b|| = 0: the answer is Phi = 0
    int sweep;         // one-sweep iteration: sweeps done since the start
    int pad[2];
    double scale;      // refinement: 1 / ||r64|| used to normalise the FP32 residual
    // One-sweep iteration with x updated every other sweep (SweepVecs::xmode):
    double alpha_prev; // alpha and beta that the previous sweep ran with
    double beta_prev;
    double x_lag;      // alpha of the increment x still lacks after the last sweep (0: none) ...
    unsigned long long x_lag_p;   // ... and the search direction it multiplies (device address)
};

// Launch geometry and tables common to every stencil launch.
struct GridArgs {
    int nr, nt, np, pitch;
    long long plane;      // nt * pitch elements
    int ci;               // radial layers per workgroup chunk
    int nchunk, ntj, ntk; // chunks along r, tiles along theta and phi
    int nblocks;
    int reverse;          // 1: walk the tiles in reverse order
    long long npad;       // elements of each vector (nr * nt * pitch), for checked builds
    int tj, tk;           // one-sweep kernel: interior rows and cells of a tile
    const RowCoef *rows;  // nr * nt
    const double *dphi;   // np: phi_f[k+1] - phi_f[k]
    const double *ih;     // np: 1 / (phi_{k+1} - phi_k), wrapping at k = np-1
};

enum Mode : int {
    kApply = 0,   // y = A x
    kResidual = 1,// r = b - A x (optional store); partials r.z, r.r, b.b
    kUpdateP = 2, // p = D^-1 r + beta p_old (stored); partial p.Ap
    kUpdateR = 3, // r -= alpha A p; x += alpha p; partials r.z, r.r
    // The r/x update in pairs of iterations (x once per pair): the even one
    // leaves x alone; the odd one adds both increments,
    // x += alpha_{k-1} p_{k-1} + alpha_k p_k, reading p_{k-1} (StencilVecs::pold).
    kUpdateRSkip = 4,
    kUpdateRPair = 5
};

// The modes of the r/x update.
constexpr bool is_update_r(int mode) { return mode == kUpdateR || mode == kUpdateRSkip || mode == kUpdateRPair; }

template <typename V>
struct StencilVecs {
    const V *in;      // operand: x (apply, residual), p (update-r), r (update-p)
    const V *pold;    // update-p: previous search direction; kUpdateRPair: p_{k-1}
    V *pnew;          // update-p: new search direction (stored)
    V *r;             // residual: out; update-r: in/out
    V *x;             // update-r: in/out
    V *y;             // apply: out
    const double *bplane;  // residual: b on the first radial layer (nt * pitch)
    const DevScalars *sc;
    double *partial;  // [3][nblocks] per-workgroup partial sums
    int store_r;      // residual: 1 to store r, 0 to reduce only
    int ignore_done;  // 1: run even when sc->done is set
    unsigned long long *tstamp;   // timing runs only: [0] earliest workgroup start, [1] latest
                                  // workgroup end (device wall clock); NULL otherwise
    int zin;          // block preconditioner: update-p reads z = M^-1 r (already
                      // preconditioned) instead of r; update-r leaves r.z, r.r to the line pass
};

// Vectors of one sweep of the one-sweep iteration (sweep j: r_j from r_{j-1}
// and A p_{j-1}, x_j, p_j; see fused_body).  r and p alternate between two
// buffers; x is updated in place.
template <typename V>
struct SweepVecs {
    const V *r_in;    // r_{j-1}
    V *r_out;         // r_j
    const V *p_old;   // p_{j-1}
    V *p_new;         // p_j
    V *x;             // x_{j-1} in, x_j out
    DevScalars *sc;   // alpha_{j-1}, beta_j (read); x_lag, x_lag_p (written by the first workgroup)
    double *partial;  // [5][nblocks]: r.z, r.r, p.Ap, z.Ap, Ap.D^-1 Ap
    int ignore_done;  // 1: run even when sc->done is set
    unsigned long long *tstamp;   // timing runs only, as in StencilVecs
    int xmode;        // 0: x_j = x_{j-1} + alpha p_{j-1} in every sweep.  Sweeps in pairs:
                      // 1 (even sweeps): x is left for the next sweep; 2 (odd sweeps): x
                      // takes both increments, p_{j-2} rebuilt as (p_{j-1} - z_{j-1}) / beta_{j-1}
};

// One slot of a batched stencil launch (device-resident table).  `out` is the
// pass's output vector: p_new for update-p, r for update-r (x is v.x).
template <typename V>
struct BatchSlot {
    GridArgs g;
    StencilVecs<V> v;
    V *out;
    int offset;   // first workgroup of the slot in the batched grid (multiple of 8)
    int active;
};

// One slot of a batched one-sweep launch (device-resident table).
template <typename V>
struct BatchSweep {
    GridArgs g;
    SweepVecs<V> v;
    int offset;   // first workgroup of the slot in the batched grid (multiple of 8)
    int active;
};

// One slot of a batched finisher launch.
struct BatchFin {
    DevScalars *sc;
    const double *partial;
    int nb;
    int active;
};

}  // namespace pot3d
