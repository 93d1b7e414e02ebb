"""CPU: the one-sweep rearrangement of the Jacobi-PCG (Sec. 2.3) gives the
same iterates as the oracle's PCG.

The GPU's one-sweep kernel computes, in sweep j, r_j = r_{j-1} - alpha A p_{j-1},
x_j = x_{j-1} + alpha p_{j-1}, z_j = D^-1 r_j, p_j = z_j + beta_j p_{j-1} and
w_j = A p_j, with the dot products r.z, r.r, p.w, z.w and w.D^-1 w; its
finisher takes alpha_j = r.z / p.w and predicts the next r.z as
r.z - 2 alpha z.w + alpha^2 w.D^-1 w for beta_{j+1}.  This test runs that
recurrence in numpy on the oracle's own operator (scipy CSR from the
oracle's coefficient arrays) and compares it with oracle.pcg: the iterates
at fixed iteration counts, and the iteration count and solution at a
tolerance.  The algebra is then the paper's PCG, and the GPU parity tests
check the kernel against the oracle directly.
"""
import numpy as np
import pytest

import oracle
from workloads import grids, magnetograms


def faces(nr, nt, np_):
    return grids.r_faces_stretched(nr), grids.theta_faces_ratio3(nt), grids.phi_faces_uniform(np_)


def one_sweep(A, d, b, tol, maxit):
    """Returns (x, iterations, status) as the library's one-sweep loop does."""
    x = np.zeros_like(b)
    r = b.copy()
    p = np.zeros_like(b)
    bnorm = np.linalg.norm(b)
    if np.linalg.norm(r) <= tol * bnorm:
        return x, 0, oracle.OK
    if maxit <= 0:
        return x, 0, oracle.ENOCONV
    alpha = beta = 0.0
    j = 0
    while True:
        r = r - alpha * (A @ p)
        x = x + alpha * p
        z = r / d
        p = z + beta * p
        w = A @ p
        rz, rr, pw, zw, wdw = r @ z, r @ r, p @ w, z @ w, w @ (w / d)
        if j > 0:
            if np.sqrt(rr) <= tol * bnorm:
                return x, j, oracle.OK
            if j >= maxit:
                return x, j, oracle.ENOCONV
        alpha = rz / pw
        rz_next = rz - 2.0 * alpha * zw + alpha * alpha * wdw
        beta = rz_next / rz if rz_next > 0.0 else 0.0
        j += 1


@pytest.mark.parametrize("shape", [(6, 10, 16), (12, 20, 40), (20, 37, 101)])
def test_fixed_count_iterates_match_oracle(shape):
    rf, tf, pf = faces(*shape)
    br = magnetograms.br_bipoles(tf, pf, 20, seed=4)
    coef = oracle.assemble(rf, tf, pf)
    b = oracle.rhs(rf, tf, pf, br).ravel()
    A = oracle.to_sparse(coef)
    d = A.diagonal()
    for K in (1, 2, 3, 10, 40):
        xo, io, _, so = oracle.pcg(coef, b, 0.0, K)
        xs, js, ss = one_sweep(A, d, b, 0.0, K)
        assert io == js == K and so == ss == oracle.ENOCONV
        err = np.linalg.norm(xs - xo.ravel()) / np.linalg.norm(xo)
        assert err <= 1e-12, (shape, K, err)


@pytest.mark.parametrize("shape", [(12, 20, 40), (20, 37, 101)])
def test_converged_solution_and_count_match_oracle(shape):
    rf, tf, pf = faces(*shape)
    br = magnetograms.br_bipoles(tf, pf, 20, seed=9)
    coef = oracle.assemble(rf, tf, pf)
    b = oracle.rhs(rf, tf, pf, br).ravel()
    A = oracle.to_sparse(coef)
    xo, io, _, so = oracle.pcg(coef, b, 1e-10, 100_000)
    xs, js, ss = one_sweep(A, A.diagonal(), b, 1e-10, 100_000)
    assert so == ss == oracle.OK
    assert abs(js - io) <= 1, (js, io)
    assert np.linalg.norm(xs - xo.ravel()) <= 1e-9 * np.linalg.norm(xo)


def test_prediction_is_the_next_residual_product():
    """The predicted r.z equals the r.z of the residual the next sweep forms
    (to rounding), and a non-positive prediction restarts with beta = 0: the
    step is then a steepest-descent step, which still converges."""
    rf, tf, pf = faces(8, 12, 24)
    br = magnetograms.br_bipoles(tf, pf, 10, seed=1)
    coef = oracle.assemble(rf, tf, pf)
    b = oracle.rhs(rf, tf, pf, br).ravel()
    A = oracle.to_sparse(coef)
    d = A.diagonal()
    rng = np.random.default_rng(3)
    r = rng.standard_normal(b.size)
    p = rng.standard_normal(b.size)
    w = A @ p
    alpha = 0.37
    pred = r @ (r / d) - 2 * alpha * (r / d) @ w + alpha * alpha * w @ (w / d)
    rn = r - alpha * w
    assert abs(pred - rn @ (rn / d)) <= 1e-12 * abs(pred)
    # restart guard: with beta forced to 0 every sweep the loop is Jacobi-preconditioned steepest descent
    x = np.zeros_like(b)
    r = b.copy()
    for _ in range(200):
        z = r / d
        w = A @ z
        a = (r @ z) / (z @ w)
        x += a * z
        r -= a * w
    assert np.linalg.norm(b - A @ x) < np.linalg.norm(b)
