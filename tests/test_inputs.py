"""Seeded synthetic inputs: grid faces and surface maps (CPU only)."""
import math

import numpy as np
import pytest

from workloads import C151, C301, SMALL, configs, grids, magnetograms


def test_workload_sizes():
    # unknowns = cells (cell-centred unknowns), matching the stated problem sizes
    assert SMALL.n == 262_144
    assert C151.n == 27_316_051
    assert C301.n == 247_157_421


@pytest.mark.parametrize("nr", [1, 8, 32, 151, 301])
def test_r_faces(nr):
    rf = grids.r_faces_stretched(nr)
    assert rf.size == nr + 1
    assert rf[0] == 1.0 and rf[-1] == 2.5
    assert np.all(np.diff(rf) > 0)


def test_r_stretch_ratio_151():
    dr = np.diff(grids.r_faces_stretched(151))
    np.testing.assert_allclose(dr[1:] / dr[:-1], 1.02, rtol=1e-10)


def test_theta_ratio3():
    for nt in (64, 301, 641):
        tf = grids.theta_faces_ratio3(nt)
        assert tf[0] == 0.0 and tf[-1] == math.pi
        dt = np.diff(tf)
        assert np.all(dt > 0)
        # symmetric about the equator
        np.testing.assert_allclose(dt, dt[::-1], rtol=1e-12)
        ratio = dt[0] / dt[nt // 2]
        assert 2.9 < ratio <= 3.0


def test_phi_faces():
    pf = grids.phi_faces_uniform(601)
    assert pf[0] == 0.0 and pf[-1] == 2 * math.pi
    np.testing.assert_allclose(np.diff(pf), 2 * math.pi / 601, rtol=1e-12)
    pj = grids.phi_faces_jittered(12, seed=4)
    assert pj[0] == 0.0 and pj[-1] == 2 * math.pi and np.all(np.diff(pj) > 0)


def test_spherical_harmonics_orthonormal():
    # midpoint quadrature on a fine sphere grid
    tf = grids.theta_faces_uniform(400)
    pf = grids.phi_faces_uniform(800)
    tc, pc = grids.sample_points(tf, pf)
    w = (np.sin(tc) * np.diff(tf))[:, None] * np.diff(pf)[None, :]
    modes = [(1, 0), (1, 1), (1, -1), (2, -2), (3, 2), (5, -3), (8, 8)]
    Y = {lm: magnetograms.real_sph_harm(lm[0], lm[1], tc[:, None], pc[None, :]) for lm in modes}
    for a in modes:
        for b in modes:
            g = float(np.sum(w * Y[a] * Y[b]))
            assert abs(g - (1.0 if a == b else 0.0)) < 2e-4, (a, b, g)


def test_harmonic_coefficients_seeded():
    c1 = magnetograms.harmonic_coefficients(8, 1)
    c2 = magnetograms.harmonic_coefficients(8, 1)
    assert c1 == c2
    assert len(c1) == sum(2 * l + 1 for l in range(1, 9))
    assert [lm[:2] for lm in c1[:4]] == [(1, -1), (1, 0), (1, 1), (2, -2)]


def test_bipoles_deterministic_and_seeded():
    rf, tf, pf = configs.Workload("t", 4, 64, 128, 1e-9, 7, "ratio3", "bipoles", nbip=20).faces()
    a = magnetograms.br_bipoles(tf, pf, 20, seed=7)
    b = magnetograms.br_bipoles(tf, pf, 20, seed=7)
    c = magnetograms.br_bipoles(tf, pf, 20, seed=8)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)
    assert a.shape == (64, 128)


def test_bipole_zero_net_flux():
    # one bipole on a fine sphere grid: the two spots cancel
    tf = grids.theta_faces_uniform(720)
    pf = grids.phi_faces_uniform(1440)
    tc, _ = grids.sample_points(tf, pf)
    w = (np.sin(tc) * np.diff(tf))[:, None] * np.diff(pf)[None, :]
    for seed in (1, 2, 3):
        br = magnetograms.br_bipoles(tf, pf, 1, seed=seed, dipole=0.0)
        flux = magnetograms.draw_bipoles(1, seed)[0][4]
        pos = float(np.sum(w * np.maximum(br, 0)))
        net = float(np.sum(w * br))
        assert abs(net) < 1e-3 * flux
        # the spots overlap a little, so the positive part is somewhat below F
        assert 0.5 * flux < pos < 1.05 * flux


def test_bipole_flux_power_law():
    bp = magnetograms.draw_bipoles(20000, seed=11)
    f = np.array([b[4] for b in bp])
    assert f.min() >= 0.01 and f.max() <= 1.0
    # empirical CDF against the truncated power law with density ~ F^-1.8
    e = 0.8
    for q in (0.02, 0.05, 0.1, 0.3):
        cdf = (0.01 ** -e - q ** -e) / (0.01 ** -e - 1.0)
        assert abs(np.mean(f <= q) - cdf) < 0.015
    sig = np.degrees([b[3] for b in bp])
    assert sig.min() >= 2.0 and sig.max() <= 5.0


def test_serve_trace_seeded():
    a = [configs.serve_request(i) for i in range(8)]
    b = [configs.serve_request(i) for i in range(8)]
    assert a == b
    assert all((w.nr, w.nt, w.np) in configs.SERVE_SIZES for w in a)
    assert all(50 <= w.nbip <= 500 for w in a)
    t = configs.poisson_arrivals(2000, 20.0, seed=3)
    assert np.all(np.diff(t) > 0)
    assert abs(2000 / t[-1] - 20.0) < 2.0
