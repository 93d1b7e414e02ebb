"""FP64 CPU oracle for the potential-field PCG solve (ctypes wrapper).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The GPU solver
library shares no code with it.  The arithmetic lives in ``pot3d_oracle.c``,
which documents the operator, right-hand side and PCG steps with their
sources in the paper (Sec. 2.1-2.3).

Every function here is pinned by the ``-m "not gpu"`` tests against:
* closed-form potentials;
* second-order grid convergence;
* exact symmetry and definiteness;
* dense solves on tiny grids;
* a library CG;
* conservation and symmetry identities.

Arrays use the phi-fastest C layout: ``x[i, j, k]`` with i radial, j polar and k azimuthal.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pot3d_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# Mutation testing only: a copy of the oracle compiled with a planted mistake
# (tests/test_oracle_mutations.py) is loaded from this path instead.
_LIB_OVERRIDE = os.environ.get("POT3D_ORACLE_LIB")

OK, EINVAL, ENOMEM, ENOCONV, EBREAKDOWN = 0, -1, -2, -4, -5
NCOEF = 8
DIAG, RM, RP, TM, TP, PM, PP, DTOP = range(NCOEF)

_lib = None


def build(force: bool = False) -> str:
    """Compile pot3d_oracle.c into liboracle.so with gcc (OpenMP, -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-Wall",
                        "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            lib = ctypes.CDLL(_LIB_OVERRIDE)
        else:
            build()
            lib = ctypes.CDLL(_LIB)
        d = ctypes.POINTER(ctypes.c_double)
        i = ctypes.c_int
        lib.orc_assemble.argtypes = [d, i, d, i, d, i, d]
        lib.orc_assemble.restype = i
        lib.orc_assemble_bc.argtypes = [d, i, d, i, d, i, i, d]
        lib.orc_assemble_bc.restype = i
        lib.orc_rhs_bc.argtypes = [d, i, d, i, d, i, i, d, d, d]
        lib.orc_rhs_bc.restype = None
        lib.orc_gauge.argtypes = [d, i, d, i, d, i, d]
        lib.orc_gauge.restype = None
        lib.orc_field.argtypes = [d, i, d, i, d, i, i, d, d, d, d, d]
        lib.orc_field.restype = None
        lib.orc_matvec.argtypes = [i, i, i, d, d, d]
        lib.orc_matvec.restype = None
        lib.orc_rhs.argtypes = [d, i, d, i, d, i, d, d]
        lib.orc_rhs.restype = None
        lib.orc_dot.argtypes = [d, d, ctypes.c_long]
        lib.orc_dot.restype = ctypes.c_double
        lib.orc_pcg.argtypes = [i, i, i, d, d, d, ctypes.c_double, i,
                                ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]
        lib.orc_pcg.restype = i
        lib.orc_pcg_pc.argtypes = [i, i, i, d, d, d, ctypes.c_double, i, i,
                                   ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]
        lib.orc_pcg_pc.restype = i
        lib.orc_line_solve.argtypes = [i, i, i, d, d, d]
        lib.orc_line_solve.restype = i
        lib.orc_set_threads.argtypes = [i]
        lib.orc_set_threads.restype = i
        lib.orc_true_relres.argtypes = [i, i, i, d, d, d]
        lib.orc_true_relres.restype = ctypes.c_double
        lib.orc_pole_values.argtypes = [i, i, i, d, d, d, d]
        lib.orc_pole_values.restype = None
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def assemble(rf, tf, pf, closed_wall: bool = False) -> np.ndarray:
    """Coefficient arrays (8, nr, nt, np): diag, W_r-, W_r+, W_t-, W_t+, W_p-, W_p+, D_top.
    closed_wall: Br = 0 on r = R1 (D_top = 0) instead of Phi = 0 there."""
    rf, tf, pf = _f64(rf), _f64(tf), _f64(pf)
    nr, nt, np_ = rf.size - 1, tf.size - 1, pf.size - 1
    coef = np.empty((NCOEF, nr, nt, np_))
    st = _load().orc_assemble_bc(_p(rf), nr, _p(tf), nt, _p(pf), np_, int(bool(closed_wall)), _p(coef))
    if st != OK:
        raise RuntimeError(f"orc_assemble failed: {st}")
    return coef


def matvec(coef: np.ndarray, x: np.ndarray) -> np.ndarray:
    _, nr, nt, np_ = coef.shape
    x = _f64(x).reshape(nr, nt, np_)
    y = np.empty_like(x)
    _load().orc_matvec(nr, nt, np_, _p(coef), _p(x), _p(y))
    return y


def rhs(rf, tf, pf, br, closed_wall: bool = False, return_monopole: bool = False):
    """b from Br on r = R0; with closed_wall the area-weighted mean of Br (the
    monopole, which a closed shell cannot carry) is removed first."""
    rf, tf, pf = _f64(rf), _f64(tf), _f64(pf)
    nr, nt, np_ = rf.size - 1, tf.size - 1, pf.size - 1
    br = _f64(br).reshape(nt, np_)
    b = np.empty((nr, nt, np_))
    mono = ctypes.c_double(0.0)
    if closed_wall:
        _load().orc_rhs_bc(_p(rf), nr, _p(tf), nt, _p(pf), np_, 1, _p(br), _p(b), ctypes.byref(mono))
    else:
        _load().orc_rhs(_p(rf), nr, _p(tf), nt, _p(pf), np_, _p(br), _p(b))
    return (b, mono.value) if return_monopole else b


def field(rf, tf, pf, x, br, closed_wall: bool = False):
    """B = -grad Phi on the cell faces: (Br (nr+1, nt, np), Bt (nr, nt+1, np),
    Bp (nr, nt, np) on the faces k+1/2).  br: the surface data, of which the
    part that enters b is used on r = R0."""
    rf, tf, pf = _f64(rf), _f64(tf), _f64(pf)
    nr, nt, np_ = rf.size - 1, tf.size - 1, pf.size - 1
    b = rhs(rf, tf, pf, br, closed_wall)
    tc = 0.5 * (tf[1:] + tf[:-1])
    w = (np.sin(tc) * np.diff(tf))[:, None] * np.diff(pf)[None, :] * rf[0] ** 2
    br0 = np.ascontiguousarray(b[0] / w)
    x = _f64(x).reshape(nr, nt, np_)
    bfr = np.empty((nr + 1, nt, np_))
    bft = np.empty((nr, nt + 1, np_))
    bfp = np.empty((nr, nt, np_))
    _load().orc_field(_p(rf), nr, _p(tf), nt, _p(pf), np_, int(bool(closed_wall)), _p(br0), _p(x), _p(bfr),
                      _p(bft), _p(bfp))
    return bfr, bft, bfp


def gauge(rf, tf, pf, x) -> np.ndarray:
    """Closed wall: x minus its cell-volume-weighted mean over the shell."""
    rf, tf, pf = _f64(rf), _f64(tf), _f64(pf)
    x = _f64(x).copy()
    _load().orc_gauge(_p(rf), rf.size - 1, _p(tf), tf.size - 1, _p(pf), pf.size - 1, _p(x))
    return x


def dot(a: np.ndarray, b: np.ndarray) -> float:
    a, b = _f64(a).ravel(), _f64(b).ravel()
    return float(_load().orc_dot(_p(a), _p(b), a.size))


PRECONDITIONERS = {"jacobi": 0, "phi_line": 1}


def pcg(coef: np.ndarray, b: np.ndarray, tol: float, maxit: int, x0=None, precond: str = "jacobi"):
    """PCG with the point-Jacobi ("jacobi", PC1 of Sec. 2.3) or the phi-line
    block preconditioner ("phi_line").  Returns (x, iters, relres_recursive, status)."""
    _, nr, nt, np_ = coef.shape
    b = _f64(b).reshape(nr, nt, np_)
    x = np.zeros_like(b) if x0 is None else _f64(x0).reshape(nr, nt, np_).copy()
    it = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    st = _load().orc_pcg_pc(nr, nt, np_, _p(coef), _p(b), _p(x), float(tol), int(maxit), PRECONDITIONERS[precond],
                            ctypes.byref(it), ctypes.byref(rr))
    return x, it.value, rr.value, st


def line_solve(coef: np.ndarray, r: np.ndarray) -> np.ndarray:
    """z = M^-1 r for the phi-line block preconditioner (one periodic
    tridiagonal solve per (i, j) row)."""
    _, nr, nt, np_ = coef.shape
    r = _f64(r).reshape(nr, nt, np_)
    z = np.empty_like(r)
    st = _load().orc_line_solve(nr, nt, np_, _p(coef), _p(r), _p(z))
    if st != OK:
        raise RuntimeError(f"orc_line_solve failed: {st}")
    return z


def set_threads(n: int = 0) -> int:
    """OpenMP threads for the following oracle calls (n <= 0: unchanged);
    returns the count in force."""
    return int(_load().orc_set_threads(int(n)))


def true_relres(coef: np.ndarray, b: np.ndarray, x: np.ndarray) -> float:
    _, nr, nt, np_ = coef.shape
    return float(_load().orc_true_relres(nr, nt, np_, _p(coef), _p(_f64(b)), _p(_f64(x))))


def pole_values(pf, x: np.ndarray):
    """(north, south), each of length nr: eq. (3) phi-averages on the rings next to the poles."""
    pf = _f64(pf)
    x = _f64(x)
    nr, nt, np_ = x.shape
    n = np.empty(nr)
    s = np.empty(nr)
    _load().orc_pole_values(nr, nt, np_, _p(pf), _p(x), _p(n), _p(s))
    return n, s


def solve(rf, tf, pf, br, tol: float, maxit: int, x0=None, closed_wall: bool = False, precond: str = "jacobi"):
    """Assemble, form b and run PCG.  Returns dict with phi, iters, relres, true_relres, status.
    closed_wall: Br = 0 on r = R1; the monopole of Br is removed from b and
    the solution is returned with zero cell-volume-weighted mean."""
    coef = assemble(rf, tf, pf, closed_wall)
    b = rhs(rf, tf, pf, br, closed_wall)
    x, iters, relres, st = pcg(coef, b, tol, maxit, x0, precond)
    if closed_wall:
        x = gauge(rf, tf, pf, x)
    return {"phi": x, "iters": iters, "relres": relres, "status": st,
            "true_relres": true_relres(coef, b, x) if np.any(b) else 0.0, "coef": coef, "b": b}


def to_sparse(coef: np.ndarray):
    """The same operator as a scipy CSR matrix, built from the coefficient
    arrays and the neighbour offsets (phi wraps; r and theta do not)."""
    import scipy.sparse as sp

    _, nr, nt, np_ = coef.shape
    n = nr * nt * np_
    idx = np.arange(n).reshape(nr, nt, np_)
    rows = [idx.ravel()]
    cols = [idx.ravel()]
    vals = [coef[DIAG].ravel()]

    def add(mask_rows, nb, w):
        rows.append(idx[mask_rows].ravel())
        cols.append(nb.ravel())
        vals.append(-w[mask_rows].ravel())

    if nr > 1:
        add(np.s_[1:, :, :], idx[:-1, :, :], coef[RM])
        add(np.s_[:-1, :, :], idx[1:, :, :], coef[RP])
    if nt > 1:
        add(np.s_[:, 1:, :], idx[:, :-1, :], coef[TM])
        add(np.s_[:, :-1, :], idx[:, 1:, :], coef[TP])
    if np_ > 1:
        add(np.s_[:, :, :], np.roll(idx, 1, axis=2), coef[PM])
        add(np.s_[:, :, :], np.roll(idx, -1, axis=2), coef[PP])
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    A.sum_duplicates()
    return A
