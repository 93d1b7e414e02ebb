// kernels.hpp -- launchers of the gfx950 kernels (defined in kernels.hip).
#pragma once

#include "pot3d.h"
#include "solver.hpp"

namespace pot3d {

enum FinWhich : int {
    kFinInit = 0,   // after the initial residual pass: rho, ||b||, first test
    kFinSigma = 1,  // after update-p: alpha = rho / p.Ap
    kFinRho = 2,    // after update-r: convergence test, beta
    kFinTrue = 3,   // after a residual pass without store: true relative residual
    kFinOuter = 4,  // refinement, after the FP64 residual pass: outer test, scale = 1/||r||
    kFinInner = 5,  // refinement, after the r.z pass on the FP32 residual: inner start
    kFinResume = 6, // refinement, reliable update: as kFinInner, keeping the direction
    kFinSweep = 7,  // one-sweep iteration: convergence test, alpha, predicted r.z, beta
    kFinLineInit = 8  // block preconditioner, after the first line pass: rho = r.z
};

// Partial sums per workgroup that a finisher may read (the one-sweep kernel
// writes five).
constexpr int kMaxPartials = 5;

// Stencil kernel shapes.  march: TJ x 64 tile per workgroup with an LDS plane;
// wave: M rows x 128 cells per wavefront, registers and lane shuffles only.
enum Tile : int {
    kTileMarch8 = 8, kTileMarch16 = 16, kTileMarch32 = 32,
    kTileWave2 = 102, kTileWave4 = 104, kTileWave8 = 108
};
inline bool tile_is_wave(int tile) { return tile > 100; }
inline int tile_rows(int tile) { return tile > 100 ? tile - 100 : tile; }
inline int tile_cols(int tile) { return tile > 100 ? 2 * kWave : kWave; }

// e0/e1 (optional): events stamped with the kernel's own start and end.
template <typename V>
hipError_t launch_stencil(int mode, int tile, const GridArgs &g, const StencilVecs<V> &v, hipStream_t s,
                          hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);

// Workgroups of a stencil kernel that fit on one compute unit at once (0 if unknown).
template <typename V>
int stencil_blocks_per_cu(int mode, int tile);

// One-sweep iteration kernel, `rows` rows of the tile box per wavefront (4, 6 or 8).
template <typename V>
hipError_t launch_sweep(int rows, const GridArgs &g, const SweepVecs<V> &v, hipStream_t s);
template <typename V>
int sweep_blocks_per_cu(int rows);
// Batched sweeps over a device slot table (every active slot runs `rows`).
template <typename V>
hipError_t launch_sweep_batch(int rows, const BatchSweep<V> *slots, int nslots, int total_blocks, int xmode,
                              hipStream_t s);
inline bool valid_sweep_rows(int rows) { return rows == 4 || rows == 6 || rows == 8; }

// Checked builds: the source line of the first out-of-range index seen since
// the last call (0 if none), after waiting for stream s.  Normal builds: 0.
unsigned take_oob_line(hipStream_t s);
bool checked_build();

// e0 (optional): an event stamped with the dispatch's start.
hipError_t launch_finish(int which, DevScalars *sc, const double *partial, int nb, hipStream_t s,
                         hipEvent_t e0 = nullptr);

// Batched passes over a device slot table: every active slot runs the given
// tile shape (the same for all slots of a launch).
template <typename V>
hipError_t launch_stencil_batch(int mode, int tile, const BatchSlot<V> *slots, int nslots, int total_blocks,
                                hipStream_t s);
hipError_t launch_finish_batch(int which, const BatchFin *fins, int nslots, hipStream_t s);

// b on the first layer from Br; mono: NULL, or (closed wall) the output of
// launch_monopole, whose monopole is subtracted.
hipError_t launch_rhs(const double *br, const double *bfac, const double *dphi, int nt, int np, int pitch,
                      const double *mono, double *bplane, hipStream_t s);
// Closed wall: out[0] = area-weighted mean of Br, out[1] = 0 if Br is that
// mean up to rounding, else 1 (device, 2 doubles).
hipError_t launch_monopole(const double *br, const double *bfac, const double *dphi, int nt, int np, double *out,
                           hipStream_t s);
// B = -grad Phi on the cell faces from x (padded) and the b plane (device).
hipError_t launch_field(const double *x, const double *bplane, const double *bfac, const double *dphi, const double *ih,
                        const double *fr, const double *ft, const double *rinv, const double *sinv, int nr, int nt,
                        int np, int pitch, double *bfr, double *bft, double *bfp, hipStream_t s);
// Closed wall: x -= its mean weighted by vr_i vt_j dphi_k (inv_volume = 1 / sum
// of the weights); partial holds nblocks doubles, *mean receives the mean.
hipError_t launch_gauge(double *x, const double *vr, const double *vt, const double *dphi, int nr, int nt, int np,
                        int pitch, double inv_volume, double *partial, int nblocks, double *mean, hipStream_t s);

// phi-line block preconditioner (uniform phi, np <= kMaxLineCells): z = M^-1 r
// row by row (r and z stored as V, the recurrences in FP64), partial sums
// [0][b] = r.z and [1][b] = r.r for b < nblocks.
constexpr int kMaxLineCells = 32 * 64;
template <typename V>
hipError_t launch_line(const GridArgs &g, const V *r, V *z, double *partial, int nblocks, const DevScalars *sc,
                       int ignore_done, hipStream_t s);
// Workgroups of the line pass resident per CU (0 if unknown).
template <typename V>
int line_blocks_per_cu(int np);

// Point Jacobi z = D^-1 r (padded layout).
hipError_t launch_jacobi(const GridArgs &g, const double *r, double *z, hipStream_t s);

template <typename V>
hipError_t launch_fill(V *p, long long n, V val, hipStream_t s);

// Padded <-> packed copy of nrows rows (pack: rows of pitch -> rows of np;
// otherwise the reverse, leaving the padding of dst untouched).  Device memory.
hipError_t launch_repack(const double *src, double *dst, long long nrows, int np, int pitch, bool pack, hipStream_t s);

// Refinement helpers.
// r32 = float(r64 * sc->scale); e32 = 0; p32 = 0 (all npad elements)
hipError_t launch_cast_residual(const double *r64, float *r32, float *e32, float *p32, long long npad,
                                const DevScalars *sc, hipStream_t s);
// r32 = float(r64 * sc->scale); e32 = 0; pdst = f * psrc (all npad elements; pdst may be psrc)
hipError_t launch_resume_residual(const double *r64, float *r32, float *e32, const float *psrc, float *pdst,
                                  long long npad, const DevScalars *sc, float f, hipStream_t s);
// x64 += double(e32) / sc->scale (all npad elements)
hipError_t launch_add_correction(double *x64, const float *e32, long long npad, const DevScalars *sc, hipStream_t s);
// x += x_lag p_lag (both from sc) on the grid cells, if the last sweep left x
// one increment behind (sweeps with xmode 1 and 2); nothing otherwise.
template <typename V>
hipError_t launch_x_catchup(V *x, const DevScalars *sc, int nr, int nt, int np, int pitch, hipStream_t s);
// per-workgroup partials of r.z and r.r (z = D^-1 r) for an FP32 vector; nblocks <= cap
hipError_t launch_dots_rz(const GridArgs &g, const float *r, double *partial, int nblocks, hipStream_t s);

hipError_t launch_poles(const double *x, const double *dphi, int nr, int nt, int np, int pitch, double period,
                        double *out, hipStream_t s);

}  // namespace pot3d
