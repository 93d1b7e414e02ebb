// kernels.hpp -- launchers of the gfx950 kernels (defined in kernels.hip).
#pragma once

#include "pot3d.h"
#include "solver.hpp"

namespace pot3d {

enum FinWhich : int {
    kFinInit = 0,   // after the initial residual pass: rho, ||b||, first test
    kFinSigma = 1,  // after update-p: alpha = rho / p.Ap
    kFinRho = 2,    // after update-r: convergence test, beta
    kFinTrue = 3    // after a residual pass without store: true relative residual
};

template <typename V>
hipError_t launch_stencil(int mode, int tj, const GridArgs &g, const StencilVecs<V> &v, hipStream_t s);

hipError_t launch_finish(int which, DevScalars *sc, const double *partial, int nb, hipStream_t s);

hipError_t launch_rhs(const double *br, const double *bfac, const double *dphi, int nt, int np, int pitch,
                      double *bplane, hipStream_t s);

template <typename V>
hipError_t launch_fill(V *p, long long n, V val, hipStream_t s);

hipError_t launch_poles(const double *x, const double *dphi, int nr, int nt, int np, int pitch, double period,
                        double *out, hipStream_t s);

}  // namespace pot3d
