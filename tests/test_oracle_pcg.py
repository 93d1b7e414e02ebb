"""Pin the oracle's Jacobi-PCG (Sec. 2.3, PC1) against definitions (CPU only).

* Dense solves on tiny grids: the PCG result against A^-1 b computed by LAPACK.
* A library CG: scipy's preconditioned CG with M = diag(A)^-1 on the same system.
* CG invariants: the A-norm error never grows; termination within n steps.
* Linear and symmetry identities: superposition, equatorial antisymmetry,
  global flux balance.
* Edge cases: zero data, warm start at the solution, iteration cap, NaN data,
  fixed-count mode, restart from a partial iterate.
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
from workloads import SMALL, grids, magnetograms

from test_oracle_operator import TINY, faces


def tiny_problem(case, seed=0):
    rf, tf, pf = faces(*case)
    rng = np.random.default_rng(seed)
    br = rng.standard_normal((tf.size - 1, pf.size - 1))
    coef = oracle.assemble(rf, tf, pf)
    b = oracle.rhs(rf, tf, pf, br)
    return rf, tf, pf, br, coef, b


@pytest.mark.parametrize("case", TINY)
def test_pcg_matches_dense_solve(case):
    _, _, _, _, coef, b = tiny_problem(case)
    A = oracle.to_sparse(coef).toarray()
    xs = np.linalg.solve(A, b.ravel())
    x, iters, relres, st = oracle.pcg(coef, b, 1e-14, 10_000)
    assert st == oracle.OK and relres <= 1e-14
    assert np.linalg.norm(x.ravel() - xs) <= 1e-10 * np.linalg.norm(xs)
    # CG terminates in at most n steps in exact arithmetic; allow a few for rounding
    assert iters <= b.size + 5


def test_pcg_matches_scipy_cg_on_small_workload():
    rf, tf, pf = SMALL.faces()
    br = SMALL.br((rf, tf, pf))
    coef = oracle.assemble(rf, tf, pf)
    b = oracle.rhs(rf, tf, pf, br)
    x, iters, relres, st = oracle.pcg(coef, b, SMALL.tol, 100_000)
    assert st == oracle.OK and relres <= SMALL.tol
    A = oracle.to_sparse(coef)
    dinv = 1.0 / coef[oracle.DIAG].ravel()
    M = spla.LinearOperator(A.shape, matvec=lambda v: dinv * v)
    count = [0]

    def cb(_):
        count[0] += 1

    xs, info = spla.cg(A, b.ravel(), rtol=SMALL.tol, atol=0.0, maxiter=100_000, M=M, callback=cb)
    assert info == 0
    assert abs(count[0] - iters) <= 2, (count[0], iters)
    assert np.linalg.norm(x.ravel() - xs) <= 1e-9 * np.linalg.norm(xs)


def test_a_norm_error_monotone():
    case = (4, 6, 8, "stretched", "ratio3", "jittered")
    _, _, _, _, coef, b = tiny_problem(case, seed=4)
    A = oracle.to_sparse(coef).toarray()
    xs = np.linalg.solve(A, b.ravel())
    prev = math.inf
    for k in range(0, 60):
        x, iters, _, st = oracle.pcg(coef, b, 0.0, k)
        assert iters == k
        e = x.ravel() - xs
        ea = math.sqrt(max(e @ A @ e, 0.0))
        assert ea <= prev * (1 + 1e-12) + 1e-14
        prev = ea


def test_zero_data_gives_zero():
    case = TINY[1]
    rf, tf, pf, br, coef, _ = tiny_problem(case)
    b = oracle.rhs(rf, tf, pf, np.zeros_like(br))
    x0 = np.ones(coef.shape[1:])
    x, iters, relres, st = oracle.pcg(coef, b, 1e-10, 100, x0=x0)
    assert st == oracle.OK and iters == 0 and np.all(x == 0)


def test_warm_start_at_solution_and_restart():
    case = (5, 8, 12, "stretched", "ratio3", "uniform")
    _, _, _, _, coef, b = tiny_problem(case, seed=9)
    x, iters, relres, st = oracle.pcg(coef, b, 1e-12, 1000)
    assert st == oracle.OK and iters > 5
    x2, iters2, _, st2 = oracle.pcg(coef, b, 1e-12, 1000, x0=x)
    assert st2 == oracle.OK and iters2 == 0 and np.array_equal(x, x2)
    # stop part-way, restart from the partial iterate, reach the same solution
    xp, ip, _, stp = oracle.pcg(coef, b, 1e-12, 7)
    assert stp == oracle.ENOCONV and ip == 7
    xr, ir, _, str_ = oracle.pcg(coef, b, 1e-12, 1000, x0=xp)
    assert str_ == oracle.OK
    assert np.linalg.norm(xr - x) <= 1e-9 * np.linalg.norm(x)


def test_iteration_cap_and_fixed_count():
    _, _, _, _, coef, b = tiny_problem(TINY[2])
    x, iters, relres, st = oracle.pcg(coef, b, 1e-14, 3)
    assert st == oracle.ENOCONV and iters == 3 and relres > 1e-14
    x, iters, relres, st = oracle.pcg(coef, b, 0.0, 11)
    assert st == oracle.ENOCONV and iters == 11


def test_nan_data_breaks_down():
    rf, tf, pf, br, coef, _ = tiny_problem(TINY[0])
    br = br.copy()
    br[1, 2] = np.nan
    b = oracle.rhs(rf, tf, pf, br)
    x, iters, relres, st = oracle.pcg(coef, b, 1e-10, 100)
    assert st == oracle.EBREAKDOWN and iters == 0


def test_superposition_and_flux_balance():
    rf = grids.r_faces_stretched(10, beta=2.99)
    tf = grids.theta_faces_ratio3(20)
    pf = grids.phi_faces_uniform(24)
    coef = oracle.assemble(rf, tf, pf)
    rng = np.random.default_rng(12)
    b1 = oracle.rhs(rf, tf, pf, rng.standard_normal((20, 24)))
    b2 = oracle.rhs(rf, tf, pf, rng.standard_normal((20, 24)))
    x1 = oracle.pcg(coef, b1, 1e-13, 10_000)[0]
    x2 = oracle.pcg(coef, b2, 1e-13, 10_000)[0]
    x12, _, relres, _ = oracle.pcg(coef, b1 + b2, 1e-13, 10_000)
    assert np.linalg.norm(x12 - x1 - x2) <= 1e-10 * np.linalg.norm(x12)
    # all flux entering through r = 1 leaves through the source surface:
    # sum(b) = sum(Dtop * Phi_top) + sum(residual)
    r = b1 - oracle.matvec(coef, x1)
    lhs = b1.sum()
    rhs = float(np.sum(coef[oracle.DTOP][-1] * x1[-1])) + r.sum()
    assert abs(lhs - rhs) <= 1e-12 * np.abs(b1).sum()


def test_equatorial_antisymmetry_of_solution():
    rf = grids.r_faces_stretched(8, beta=2.99)
    tf = grids.theta_faces_ratio3(16)
    pf = grids.phi_faces_uniform(32)
    tc, pc = grids.sample_points(tf, pf)
    # odd in cos(theta): l + m odd modes
    br = magnetograms.real_sph_harm(1, 0, tc[:, None], pc[None, :]) \
        + 0.3 * magnetograms.real_sph_harm(3, 2, tc[:, None], pc[None, :])
    res = oracle.solve(rf, tf, pf, br, 1e-13, 10_000)
    phi = res["phi"]
    np.testing.assert_allclose(phi[:, ::-1, :], -phi, atol=1e-11 * np.abs(phi).max())


@pytest.mark.parametrize("case", TINY)
def test_true_relres_fixed_values(case):
    """The true relative residual ||b - A x||_2 / ||b||_2 (Sec. 4.1's relative
    tolerance, recomputed from x) at points where its value is fixed by the
    algebra alone, with x* = A^-1 b from a dense LAPACK solve:
      x = 0        -> exactly 1 (the residual is b);
      x = 2 x*     -> 1 (the residual is -b);
      x = -x*      -> 2 (the residual is 2 b);
      x = (1+e) x* -> e (the residual is -e b);
      x = x*       -> rounding only.
    A dropped square root, a ||b||^2 denominator or a sign error in b - A x
    each fails one of these."""
    _, _, _, _, coef, b = tiny_problem(case, seed=3)
    A = oracle.to_sparse(coef).toarray()
    xs = np.linalg.solve(A, b.ravel()).reshape(b.shape)
    assert oracle.true_relres(coef, b, np.zeros_like(b)) == 1.0
    assert abs(oracle.true_relres(coef, b, 2.0 * xs) - 1.0) <= 1e-12
    assert abs(oracle.true_relres(coef, b, -xs) - 2.0) <= 1e-12
    for eps in (1e-3, 0.25, 3.0):
        assert abs(oracle.true_relres(coef, b, (1.0 + eps) * xs) - eps) <= 1e-9 * eps + 1e-13
    assert oracle.true_relres(coef, b, xs) <= 1e-13
    # a scaled problem: the ratio does not depend on the units of b
    assert abs(oracle.true_relres(coef, 1e6 * b, 1e6 * 1.5 * xs) - 0.5) <= 1e-12


def test_true_relres_random_against_numpy():
    """On a random x the value equals the definition computed with numpy from
    the dense operator (a plain sum of squares, no compensation)."""
    _, _, _, _, coef, b = tiny_problem(TINY[-1], seed=4)
    A = oracle.to_sparse(coef).toarray()
    x = np.random.default_rng(5).standard_normal(b.shape)
    res = b.ravel() - A @ x.ravel()
    want = math.sqrt(float(res @ res)) / math.sqrt(float(b.ravel() @ b.ravel()))
    assert abs(oracle.true_relres(coef, b, x) - want) <= 1e-13 * want
