"""Pins of the oracle's operator A and right-hand side b (CPU only).

A is the Sec. 2.2 finite-difference Laplacian with the spherical metric restored,
scaled by the cell volume and negated.  These tests pin it with properties
that follow from the mathematics, not by retyping the weights:
* exact symmetry and definiteness (Sec. 2.3 calls A symmetric);
* A . 1 vanishing away from the Dirichlet top;
* invariance under a phi rotation and an equatorial reflection;
* agreement between the stencil matvec and an assembled sparse matrix.
Grid convergence to closed forms is in test_oracle_closed_form.py.
"""
import math

import numpy as np
import pytest

import oracle
from workloads import SMALL, grids

TINY = [
    # (nr, nt, np, r-map, theta-map, phi-map)
    (3, 4, 6, "uniform", "uniform", "uniform"),
    (4, 6, 8, "stretched", "ratio3", "jittered"),
    (5, 8, 12, "stretched", "ratio3", "uniform"),
    (2, 3, 3, "stretched", "uniform", "jittered"),
]


def faces(nr, nt, np_, rmap, tmap, pmap, seed=0):
    rf = grids.r_faces_stretched(nr, beta=2.99) if rmap == "stretched" else grids.r_faces_uniform(nr)
    tf = grids.theta_faces_ratio3(nt) if tmap == "ratio3" else grids.theta_faces_uniform(nt)
    pf = grids.phi_faces_jittered(np_, seed=seed + 3) if pmap == "jittered" else grids.phi_faces_uniform(np_)
    return rf, tf, pf


@pytest.mark.parametrize("case", TINY)
def test_exactly_symmetric_and_spd(case):
    coef = oracle.assemble(*faces(*case))
    A = oracle.to_sparse(coef).toarray()
    assert np.max(np.abs(A - A.T)) <= 1e-15 * np.max(np.abs(A))
    np.linalg.cholesky(A)  # raises if not positive definite
    ev = np.linalg.eigvalsh(A)
    assert ev.min() > 0
    # off-diagonals are non-positive and the diagonal dominates (an M-matrix)
    off = A - np.diag(np.diag(A))
    assert np.all(off <= 0)
    assert np.all(np.diag(A) >= -off.sum(axis=1) - 1e-15 * np.abs(A).max())


@pytest.mark.parametrize("case", TINY)
def test_stencil_matches_assembled_matrix(case):
    coef = oracle.assemble(*faces(*case))
    A = oracle.to_sparse(coef)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(coef.shape[1:])
    np.testing.assert_allclose(oracle.matvec(coef, x).ravel(), A @ x.ravel(), rtol=1e-13, atol=1e-13)


def test_symmetry_on_random_vectors_small():
    rf, tf, pf = SMALL.faces()
    coef = oracle.assemble(rf, tf, pf)
    rng = np.random.default_rng(1)
    x = rng.standard_normal(coef.shape[1:])
    y = rng.standard_normal(coef.shape[1:])
    a = oracle.dot(x, oracle.matvec(coef, y))
    b = oracle.dot(y, oracle.matvec(coef, x))
    assert abs(a - b) <= 1e-12 * abs(a)


@pytest.mark.parametrize("case", TINY + [(8, 16, 32, "stretched", "ratio3", "uniform")])
def test_constant_in_nullspace_except_top(case):
    """The Laplacian of a constant vanishes; only the Phi = 0 top face leaks:
    A . 1 = D_top on the outer layer and 0 elsewhere (Neumann bottom, closed
    poles, periodic phi)."""
    coef = oracle.assemble(*faces(*case))
    y = oracle.matvec(coef, np.ones(coef.shape[1:]))
    scale = coef[oracle.DIAG].max()
    np.testing.assert_allclose(y[:-1], 0.0, atol=1e-14 * scale)
    np.testing.assert_allclose(y[-1], coef[oracle.DTOP][-1], rtol=1e-12, atol=1e-14 * scale)
    assert np.all(coef[oracle.DTOP][:-1] == 0) and np.all(coef[oracle.DTOP][-1] > 0)


def test_pole_faces_carry_no_weight():
    coef = oracle.assemble(*faces(6, 10, 16, "stretched", "ratio3", "uniform"))
    assert np.all(coef[oracle.TM][:, 0, :] == 0.0)
    assert np.all(coef[oracle.TP][:, -1, :] == 0.0)
    assert np.all(coef[oracle.RM][0] == 0.0)      # Neumann bottom: no inward radial coupling
    assert np.all(coef[oracle.RP][-1] == 0.0)     # top coupling lives on the diagonal


def test_phi_rotation_equivariance():
    rf, tf, pf = faces(6, 10, 16, "stretched", "ratio3", "uniform")
    coef = oracle.assemble(rf, tf, pf)
    x = np.random.default_rng(2).standard_normal(coef.shape[1:])
    for s in (1, 5, 15):
        np.testing.assert_allclose(oracle.matvec(coef, np.roll(x, s, axis=2)),
                                   np.roll(oracle.matvec(coef, x), s, axis=2), rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("tmap", ["uniform", "ratio3"])
def test_equatorial_reflection(tmap):
    rf, tf, pf = faces(5, 9, 12, "stretched", tmap, "uniform")
    coef = oracle.assemble(rf, tf, pf)
    x = np.random.default_rng(3).standard_normal(coef.shape[1:])
    np.testing.assert_allclose(oracle.matvec(coef, x[:, ::-1, :]),
                               oracle.matvec(coef, x)[:, ::-1, :], rtol=1e-11, atol=1e-13)


def test_rhs_is_surface_flux():
    """b carries Br times the r = 1 face area only; summed over the sphere it
    is the net surface flux, which vanishes for a dipole map (the integral of
    cos(theta) over the sphere is zero and the polar grid is symmetric)."""
    rf, tf, pf = faces(4, 32, 16, "stretched", "ratio3", "uniform")
    tc, pc = grids.sample_points(tf, pf)
    br = np.cos(tc)[:, None] * np.ones((1, 16))
    b = oracle.rhs(rf, tf, pf, br)
    assert np.all(b[1:] == 0)
    assert abs(b.sum()) < 1e-14
    ones = oracle.rhs(rf, tf, pf, np.ones((32, 16)))
    # face areas sum to the surface of the unit sphere to second order
    assert abs(ones.sum() - 4 * math.pi) < 4 * math.pi * 5e-3
