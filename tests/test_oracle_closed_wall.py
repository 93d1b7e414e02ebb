"""Oracle pins for the closed-wall upper boundary (Sec. 2.1: Br = 0 on r = R1).

With no flux through the top face the system is singular: its null space is
the constants.  The oracle removes the monopole of Br (a closed shell carries
no net flux) and returns the solution with zero cell-volume-weighted mean.
Pinned here against what the mathematics fixes:
* the operator annihilates constants, is symmetric, and has exactly one zero
  eigenvalue (dense, on tiny grids);
* the monopole-free b sums to zero, and Br = const gives Phi = 0;
* PCG reaches the dense minimum-norm solution (pseudo-inverse), up to the
  gauge;
* the discrete solutions converge at second order to the closed forms
  Phi = (A r^l + B r^-(l+1)) Y_lm with dPhi/dr = -Y_lm at r = 1 and
  dPhi/dr = 0 at r = R1.
"""
import math

import numpy as np
import pytest

import oracle
from workloads import grids, magnetograms


def faces(nr, nt, np_, tmap="ratio3"):
    rf = grids.r_faces_stretched(nr, beta=2.99)
    tf = grids.theta_faces_ratio3(nt) if tmap == "ratio3" else grids.theta_faces_uniform(nt)
    return rf, tf, grids.phi_faces_uniform(np_)


def volumes(rf, tf, pf):
    rc = 0.5 * (rf[1:] + rf[:-1])
    tc = 0.5 * (tf[1:] + tf[:-1])
    return (rc ** 2 * np.diff(rf))[:, None, None] * (np.sin(tc) * np.diff(tf))[None, :, None] \
        * np.diff(pf)[None, None, :]


@pytest.mark.parametrize("shape", [(3, 4, 6), (4, 6, 8)])
def test_closed_wall_operator_null_space(shape):
    rf, tf, pf = faces(*shape)
    A = oracle.to_sparse(oracle.assemble(rf, tf, pf, closed_wall=True)).toarray()
    n = A.shape[0]
    scale = np.abs(A).max()
    assert np.abs(A @ np.ones(n)).max() <= 1e-13 * scale
    assert np.array_equal(A, A.T)
    ev = np.linalg.eigvalsh(A)
    assert abs(ev[0]) <= 1e-12 * scale and ev[1] > 1e-6 * scale
    # the source-surface operator differs only by D_top on the top layer, and is definite
    A0 = oracle.to_sparse(oracle.assemble(rf, tf, pf)).toarray()
    d = np.diag(A0 - A).reshape(shape)
    assert np.all(d[:-1] == 0.0) and np.all(d[-1] > 0.0)
    assert np.count_nonzero(A0 - A - np.diag(np.diag(A0 - A))) == 0
    assert np.linalg.eigvalsh(A0)[0] > 0.0


def test_monopole_removed_and_constant_data_give_zero():
    rf, tf, pf = faces(5, 8, 12)
    rng = np.random.default_rng(4)
    br = rng.standard_normal((8, 12)) + 3.0
    b, mono = oracle.rhs(rf, tf, pf, br, closed_wall=True, return_monopole=True)
    tc = 0.5 * (tf[1:] + tf[:-1])
    w = (np.sin(tc) * np.diff(tf))[:, None] * np.diff(pf)[None, :]
    assert mono == pytest.approx(np.sum(w * br) / np.sum(w), rel=1e-14)
    assert abs(b.sum()) <= 1e-13 * np.abs(b).sum()
    res = oracle.solve(rf, tf, pf, np.full((8, 12), 2.5), 1e-12, 1000, closed_wall=True)
    assert res["status"] == oracle.OK and res["iters"] == 0 and np.all(res["phi"] == 0.0)


@pytest.mark.parametrize("shape", [(3, 4, 6), (4, 6, 8), (5, 7, 9)])
def test_pcg_matches_dense_pseudo_inverse(shape):
    rf, tf, pf = faces(*shape)
    br = np.random.default_rng(sum(shape)).standard_normal(shape[1:])
    coef = oracle.assemble(rf, tf, pf, closed_wall=True)
    b = oracle.rhs(rf, tf, pf, br, closed_wall=True)
    A = oracle.to_sparse(coef).toarray()
    x_pinv = np.linalg.pinv(A, rcond=1e-12) @ b.ravel()
    ref = oracle.gauge(rf, tf, pf, x_pinv.reshape(shape))
    res = oracle.solve(rf, tf, pf, br, 1e-13, 10_000, closed_wall=True)
    assert res["status"] == oracle.OK
    assert np.abs(res["phi"] - ref).max() <= 1e-9 * np.abs(ref).max()
    # the gauge: zero volume-weighted mean
    v = volumes(rf, tf, pf)
    assert abs(np.sum(v * res["phi"])) <= 1e-12 * np.sum(v * np.abs(res["phi"]))


def closed_wall_mode(l, m, nr, nt, np_):
    rf, tf, pf = faces(nr, nt, np_)
    tc, pc = grids.sample_points(tf, pf)
    br = magnetograms.real_sph_harm(l, m, tc[:, None], pc[None, :])
    res = oracle.solve(rf, tf, pf, br, 1e-13, 100_000, closed_wall=True)
    assert res["status"] == oracle.OK
    R1 = rf[-1]
    # dPhi/dr = -Y at r = 1 and 0 at r = R1 for Phi = (A r^l + B r^-(l+1)) Y
    B = 1.0 / ((l + 1) * (1.0 - R1 ** (-(2 * l + 1))))
    A = B * (l + 1) * R1 ** (-(2 * l + 1)) / l
    rc = 0.5 * (rf[1:] + rf[:-1])
    ex = (A * rc ** l + B * rc ** (-(l + 1)))[:, None, None] * br[None, :, :]
    ex = oracle.gauge(rf, tf, pf, ex)
    return np.abs(res["phi"] - ex).max() / np.abs(ex).max()


@pytest.mark.parametrize("lm", [(1, 0), (2, 1), (3, -2)])
def test_closed_wall_second_order_convergence(lm):
    errs = [closed_wall_mode(*lm, 8 * s, 16 * s, 32 * s) for s in (1, 2, 4)]
    order = math.log2(errs[1] / errs[2])
    assert 1.8 <= order <= 2.2, (lm, errs)
    assert errs[-1] < 5e-3
