"""Pin the oracle's discrete solution to closed-form potentials (CPU only).

For a surface map Br = c Y_lm, the boundary-value problem of Sec. 2.1 has the
exact solution Phi = (a r^l + b r^-(l+1)) Y_lm.  The paper calls its scheme
globally second order (Sec. 2.2).  The oracle's solution must converge to
these potentials at rate two under grid refinement.  A dropped metric factor,
a wrong sign or index, or a bad pole or seam treatment breaks that rate.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from workloads import SMALL, grids, magnetograms

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))
R1 = GOLDEN["R1"]


def radial_coeffs(l, c=1.0, r1=R1):
    """(a, b) with l a - (l+1) b = -c and a r1^l + b r1^-(l+1) = 0."""
    if l == 0:
        return 0.0, c
    a = -c / (l + (l + 1) * r1 ** (2 * l + 1))
    return a, -a * r1 ** (2 * l + 1)


def exact_phi(l, m, c, rc, tc, pc, r1=R1):
    a, b = radial_coeffs(l, c, r1)
    radial = a * rc ** l + b * rc ** (-l - 1)
    if l == 0:
        radial = radial - c / r1
        return radial[:, None, None] * np.ones((1, tc.size, pc.size)) / math.sqrt(4 * math.pi)
    Y = magnetograms.real_sph_harm(l, m, tc[:, None], pc[None, :])
    return radial[:, None, None] * Y[None, :, :]


def test_golden_coefficients():
    """The hand-worked fractions match the coefficient helper used below."""
    for key, l in (("l1_dipole", 1), ("l2", 2)):
        a, b = radial_coeffs(l)
        assert float(Fraction(GOLDEN[key]["a_fraction"])) == pytest.approx(a, rel=1e-15)
        assert float(Fraction(GOLDEN[key]["b_fraction"])) == pytest.approx(b, rel=1e-15)
        assert a + b == pytest.approx(GOLDEN[key]["phi_at_r1"], rel=1e-14)
    # monopole: Phi = 1/r - 1/R1
    assert 1.0 - 1.0 / R1 == pytest.approx(GOLDEN["l0_monopole"]["phi_at_r1"], rel=1e-15)


def centres(f):
    return 0.5 * (f[:-1] + f[1:])


def solve_mode(l, m, nr, nt, np_, tmap="ratio3"):
    rf = grids.r_faces_stretched(nr, beta=2.99)
    tf = grids.theta_faces_ratio3(nt) if tmap == "ratio3" else grids.theta_faces_uniform(nt)
    pf = grids.phi_faces_uniform(np_)
    tc, pc = grids.sample_points(tf, pf)
    if l == 0:
        br = np.full((nt, np_), 1.0 / math.sqrt(4 * math.pi))
    else:
        br = magnetograms.real_sph_harm(l, m, tc[:, None], pc[None, :])
    res = oracle.solve(rf, tf, pf, br, 1e-13, 100000)
    assert res["status"] == oracle.OK
    ex = exact_phi(l, m, 1.0, centres(rf), tc, pc)
    vol = ((rf[1:] ** 3 - rf[:-1] ** 3) / 3)[:, None, None] * (np.sin(tc) * np.diff(tf))[None, :, None] \
        * np.diff(pf)[None, None, :]
    err = res["phi"] - ex
    emax = np.abs(err).max() / np.abs(ex).max()
    el2 = math.sqrt(np.sum(vol * err ** 2) / np.sum(vol * ex ** 2))
    return emax, el2, res, rf, tf, pf


@pytest.mark.parametrize("lm", [(0, 0), (1, 0), (2, 1), (3, -2)])
def test_second_order_convergence(lm):
    l, m = lm
    errs = [solve_mode(l, m, 8 * s, 16 * s, 32 * s)[:2] for s in (1, 2, 4)]
    for norm in (0, 1):
        e = [x[norm] for x in errs]
        orders = [math.log2(e[i] / e[i + 1]) for i in range(2)]
        assert 1.8 <= orders[-1] <= 2.2, (lm, norm, e, orders)
        assert orders[0] > 1.7, (lm, norm, e, orders)
    assert errs[-1][0] < 3e-3


def test_uniform_theta_also_second_order():
    e = [solve_mode(1, 1, 8 * s, 16 * s, 32 * s, tmap="uniform")[0] for s in (1, 2, 4)]
    assert 1.8 <= math.log2(e[1] / e[2]) <= 2.2


def test_small_workload_matches_harmonic_sum():
    """The 32 x 64 x 128 harmonic workload (l = 1..8) against its closed form."""
    rf, tf, pf = SMALL.faces()
    br, coeffs = magnetograms.br_harmonics(tf, pf, SMALL.lmax, SMALL.seed)
    res = oracle.solve(rf, tf, pf, br, SMALL.tol, 100000)
    assert res["status"] == oracle.OK
    tc, pc = grids.sample_points(tf, pf)
    ex = sum(exact_phi(l, m, c, centres(rf), tc, pc) for l, m, c in coeffs)
    rel = np.abs(res["phi"] - ex).max() / np.abs(ex).max()
    # l = 8 on 64 polar cells is coarse; the bound is a few percent, not 1e-3
    assert rel < 0.05
    assert res["true_relres"] < 1e-9


def test_pole_values_converge_to_ring_value():
    """Eq. (3): the pole value is the phi-average on the ring half a pole cell
    away.  For the dipole it tends to Phi_exact(r, theta = eps) at second order,
    and for an axisymmetric field it equals the ring value exactly."""
    errs = []
    for s in (1, 2, 4):
        _, _, res, rf, tf, pf = solve_mode(1, 0, 8 * s, 16 * s, 32 * s)
        north, south = oracle.pole_values(pf, res["phi"])
        np.testing.assert_allclose(north, res["phi"][:, 0, :].mean(axis=1), rtol=1e-12)
        tc, pc = grids.sample_points(tf, pf)
        a, b = radial_coeffs(1)
        rc = centres(rf)
        exn = (a * rc + b / rc ** 2) * math.sqrt(3 / (4 * math.pi)) * math.cos(tc[0])
        exs = (a * rc + b / rc ** 2) * math.sqrt(3 / (4 * math.pi)) * math.cos(tc[-1])
        errs.append(max(np.abs(north - exn).max(), np.abs(south - exs).max()) / np.abs(exn).max())
        # odd dipole: south = -north on the symmetric grid
        np.testing.assert_allclose(south, -north, rtol=1e-7, atol=1e-12)
    assert math.log2(errs[1] / errs[2]) > 1.8
