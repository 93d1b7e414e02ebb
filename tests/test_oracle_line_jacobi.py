"""Pins of the oracle's phi-line block preconditioner (CPU only).

M is the block diagonal of A whose blocks are whole azimuthal rows: for each
(i, j), the principal submatrix of A on the cells k = 0 .. np-1 of that row
(the diagonal and the two periodic azimuthal weights).  Sec. 2.3 uses only the
diagonal (PC1); Sec. 6 asks for stronger preconditioners that still map well
onto vector hardware.  The oracle solves each block by the Thomas algorithm
with a Sherman-Morrison correction for the periodic corners.  Pinned here by:
* the definition: each block of M cut out of the dense A and solved by LAPACK;
* a closed form: on a uniform phi grid each block is circulant, so a Fourier
  mode cos(m phi_k) is an eigenvector with eigenvalue d - 2 w cos(m dphi);
* symmetry and definiteness of M^-1;
* PCG with M: the dense solution on tiny grids, and scipy's CG with the same M.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from workloads import SMALL, grids

from test_oracle_operator import TINY, faces

LINE_CASES = TINY + [(3, 5, 1, "uniform", "uniform", "uniform"), (3, 5, 2, "stretched", "ratio3", "uniform"),
                     (4, 7, 31, "stretched", "ratio3", "jittered")]


def row_blocks(coef):
    """The blocks of M, cut from the dense operator A itself."""
    _, nr, nt, np_ = coef.shape
    A = oracle.to_sparse(coef).toarray()
    for row in range(nr * nt):
        ix = np.arange(row * np_, (row + 1) * np_)
        yield ix, A[np.ix_(ix, ix)]


@pytest.mark.parametrize("case", LINE_CASES)
def test_line_solve_is_the_block_solve(case):
    coef = oracle.assemble(*faces(*case))
    r = np.random.default_rng(11).standard_normal(coef.shape[1:])
    z = oracle.line_solve(coef, r).ravel()
    for ix, blk in row_blocks(coef):
        want = np.linalg.solve(blk, r.ravel()[ix])
        assert np.abs(z[ix] - want).max() <= 1e-12 * np.abs(want).max(), ix[0]


def test_line_solve_fourier_modes_on_a_circulant_row():
    """Uniform phi: block (i, j) is d I - w (shift + shift^-1) with one d and
    one w per row, so cos(m phi_k) maps to cos(m phi_k) / (d - 2 w cos(m dphi))."""
    nr, nt, np_ = 3, 6, 16
    rf, tf = grids.r_faces_stretched(nr, beta=2.99), grids.theta_faces_ratio3(nt)
    pf = grids.phi_faces_uniform(np_)
    coef = oracle.assemble(rf, tf, pf)
    phic = 0.5 * (pf[1:] + pf[:-1])
    dphi = 2 * np.pi / np_
    for m in (0, 1, 3, 7):
        r = np.broadcast_to(np.cos(m * phic), (nr, nt, np_)).copy()
        z = oracle.line_solve(coef, r)
        d = coef[oracle.DIAG][:, :, 0]
        w = coef[oracle.PP][:, :, 0]
        assert np.allclose(coef[oracle.PM], w[:, :, None], rtol=1e-14, atol=0)
        lam = d - 2.0 * w * np.cos(m * dphi)
        want = r / lam[:, :, None]
        assert np.abs(z - want).max() <= 1e-13 * np.abs(want).max(), m


@pytest.mark.parametrize("case", TINY[:3])
def test_line_inverse_is_symmetric_positive_definite(case):
    coef = oracle.assemble(*faces(*case))
    rng = np.random.default_rng(2)
    x, y = rng.standard_normal((2,) + coef.shape[1:])
    mx, my = oracle.line_solve(coef, x), oracle.line_solve(coef, y)
    assert abs(np.vdot(y, mx) - np.vdot(x, my)) <= 1e-13 * np.linalg.norm(mx) * np.linalg.norm(y)
    assert np.vdot(x, mx) > 0


@pytest.mark.parametrize("case", TINY)
def test_pcg_phi_line_matches_dense_solve(case):
    rf, tf, pf = faces(*case)
    br = np.random.default_rng(0).standard_normal((tf.size - 1, pf.size - 1))
    coef = oracle.assemble(rf, tf, pf)
    b = oracle.rhs(rf, tf, pf, br)
    A = oracle.to_sparse(coef).toarray()
    xs = np.linalg.solve(A, b.ravel())
    x, iters, relres, st = oracle.pcg(coef, b, 1e-14, 10_000, precond="phi_line")
    assert st == oracle.OK and relres <= 1e-14
    assert np.linalg.norm(x.ravel() - xs) <= 1e-10 * np.linalg.norm(xs)
    assert iters <= b.size + 5


def line_operator(coef):
    """M as a sparse matrix (the within-row entries of A) and its LU."""
    _, nr, nt, np_ = coef.shape
    A = oracle.to_sparse(coef).tocoo()
    keep = (A.row // np_) == (A.col // np_)
    M = sp.csc_matrix((A.data[keep], (A.row[keep], A.col[keep])), shape=A.shape)
    return M, spla.splu(M)


def test_pcg_phi_line_matches_scipy_cg():
    """The 32 x 64 x 128 workload: the oracle's line-preconditioned PCG and
    scipy's CG with the same M (applied through a sparse LU) agree."""
    rf, tf, pf = SMALL.faces()
    br = SMALL.br((rf, tf, pf))
    coef = oracle.assemble(rf, tf, pf)
    b = oracle.rhs(rf, tf, pf, br).ravel()
    A = oracle.to_sparse(coef).tocsr()
    _, lu = line_operator(coef)
    n_cb = [0]
    xs, info = spla.cg(A, b, rtol=SMALL.tol, atol=0.0, maxiter=100_000,
                       M=spla.LinearOperator(A.shape, matvec=lu.solve),
                       callback=lambda xk: n_cb.__setitem__(0, n_cb[0] + 1))
    assert info == 0
    x, iters, relres, st = oracle.pcg(coef, b, SMALL.tol, 100_000, precond="phi_line")
    assert st == oracle.OK
    assert abs(iters - n_cb[0]) <= 2, (iters, n_cb[0])
    assert np.linalg.norm(x.ravel() - xs) <= 1e-9 * np.linalg.norm(xs)
    # the point of the block preconditioner: fewer iterations than PC1 here
    _, iters_j, _, st_j = oracle.pcg(coef, b, SMALL.tol, 100_000)
    assert st_j == oracle.OK and iters < 0.8 * iters_j, (iters, iters_j)
