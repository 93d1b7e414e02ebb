"""Oracle pins for the field output B = -grad Phi (Sec. 2.1) on the cell faces.

* Discrete Gauss law: for ANY Phi, the net outward flux of B from each cell,
  with the face areas of the scheme, equals (A Phi - b) in that cell, for both
  upper boundaries (the operator is the flux divergence of these differences);
* the surface data come back on r = R0 and the pole faces carry zero;
* on the dipole solution the face values converge at second order to the
  exact B = -grad((a r + b / r^2) cos(theta)).
"""
import math

import numpy as np
import pytest

import oracle
from workloads import grids, magnetograms


def faces(nr, nt, np_):
    return grids.r_faces_stretched(nr, beta=2.99), grids.theta_faces_ratio3(nt), grids.phi_faces_jittered(np_, seed=2)


def net_outward_flux(rf, tf, pf, bfr, bft, bfp):
    rc = 0.5 * (rf[1:] + rf[:-1])
    tc = 0.5 * (tf[1:] + tf[:-1])
    dr, dt, dp = np.diff(rf), np.diff(tf), np.diff(pf)
    ar = (rf ** 2)[:, None, None] * (np.sin(tc) * dt)[None, :, None] * dp[None, None, :]      # (nr+1, nt, np)
    at = (rc * dr)[:, None, None] * np.sin(tf)[None, :, None] * dp[None, None, :]            # (nr, nt+1, np)
    ap = (rc * dr)[:, None, None] * dt[None, :, None] * np.ones_like(dp)[None, None, :]      # (nr, nt, np)
    fr, ft, fp = bfr * ar, bft * at, bfp * ap
    net = (fr[1:] - fr[:-1]) + (ft[:, 1:] - ft[:, :-1]) + (fp - np.roll(fp, 1, axis=2))
    scale = np.abs(fr[1:]) + np.abs(fr[:-1]) + np.abs(ft[:, 1:]) + np.abs(ft[:, :-1]) + np.abs(fp) \
        + np.abs(np.roll(fp, 1, axis=2))
    return net, scale


@pytest.mark.parametrize("closed_wall", [False, True], ids=["source_surface", "closed_wall"])
@pytest.mark.parametrize("shape", [(3, 4, 5), (6, 9, 14)])
def test_discrete_gauss_law_for_any_phi(shape, closed_wall):
    rf, tf, pf = faces(*shape)
    rng = np.random.default_rng(7)
    x = rng.standard_normal(shape)
    br = rng.standard_normal(shape[1:]) + 0.5
    bfr, bft, bfp = oracle.field(rf, tf, pf, x, br, closed_wall)
    coef = oracle.assemble(rf, tf, pf, closed_wall)
    b = oracle.rhs(rf, tf, pf, br, closed_wall)
    net, scale = net_outward_flux(rf, tf, pf, bfr, bft, bfp)
    assert np.all(np.abs(net - (oracle.matvec(coef, x) - b)) <= 1e-13 * scale.max())
    # the boundary faces
    tc = 0.5 * (tf[1:] + tf[:-1])
    w = (np.sin(tc) * np.diff(tf))[:, None] * np.diff(pf)[None, :] * rf[0] ** 2
    np.testing.assert_allclose(bfr[0], b[0] / w, rtol=1e-14, atol=0)
    assert np.all(bft[:, 0] == 0.0) and np.all(bft[:, -1] == 0.0)
    if closed_wall:
        assert np.all(bfr[-1] == 0.0)


def dipole_field_error(s):
    nr, nt, np_ = 8 * s, 16 * s, 16 * s
    rf = grids.r_faces_stretched(nr, beta=2.99)
    tf = grids.theta_faces_ratio3(nt)
    pf = grids.phi_faces_uniform(np_)
    br = magnetograms.br_dipole(tf, pf)
    res = oracle.solve(rf, tf, pf, br, 1e-13, 100_000)
    bfr, bft, _ = oracle.field(rf, tf, pf, res["phi"], br)
    R1 = rf[-1]
    a = -1.0 / (1.0 + 2.0 * R1 ** 3)
    b = -a * R1 ** 3
    tc = 0.5 * (tf[1:] + tf[:-1])
    rc = 0.5 * (rf[1:] + rf[:-1])
    ex_r = -(a - 2.0 * b / rf ** 3)[:, None] * np.cos(tc)[None, :]                 # on r-faces
    ex_t = ((a * rc + b / rc ** 2) / rc)[:, None] * np.sin(tf)[None, :]            # on theta-faces
    er = np.abs(bfr[:, :, 0] - ex_r).max() / np.abs(ex_r).max()
    et = np.abs(bft[:, :, 0] - ex_t).max() / np.abs(ex_t).max()
    return er, et


def test_dipole_field_second_order():
    errs = [dipole_field_error(s) for s in (1, 2, 4)]
    for c in (0, 1):
        order = math.log2(errs[1][c] / errs[2][c])
        assert 1.7 <= order <= 2.3, errs
