"""Seeded synthetic surface maps Br(theta, phi) at r = 1.

The paper's test case drives the solve with an observed surface field
(Sec. 4.1, "Test Case") that is not available here.  These generators stand in
for it with fields of the same character, sampled at the angular midpoints of
the faces (the positions of the unknowns next to the lower boundary):

* ``br_harmonics``: a sum of real, orthonormal spherical harmonics of degree
  1..lmax with N(0, 1/l^2) coefficients.  Every term has a closed-form
  potential, which the tests use to pin the solver.
* ``br_bipoles``: a global dipole B0 cos(theta) plus Gaussian bipoles (active
  regions) at random positions, tilts and widths, with fluxes drawn from a
  power law.  Each bipole carries zero net flux.

Nothing here touches the solver's discretization: values are point samples.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import gammaln, lpmv

from .grids import sample_points


def real_sph_harm(l: int, m: int, theta: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """Real spherical harmonic of degree l, order m, orthonormal on the unit sphere.

    m > 0 -> sqrt(2) N_lm P_l^m(cos t) cos(m p); m < 0 -> sqrt(2) N_l|m| P_l^|m|(cos t) sin(|m| p);
    m = 0 -> N_l0 P_l(cos t), with N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!).
    ``theta`` and ``phi`` broadcast against each other.
    """
    am = abs(m)
    if am > l:
        raise ValueError("|m| must be <= l")
    lognorm = 0.5 * (math.log((2 * l + 1) / (4.0 * math.pi)) + gammaln(l - am + 1) - gammaln(l + am + 1))
    plm = lpmv(am, l, np.cos(theta))
    if m == 0:
        return math.exp(lognorm) * plm * np.ones_like(phi)
    ang = np.cos(am * phi) if m > 0 else np.sin(am * phi)
    return math.sqrt(2.0) * math.exp(lognorm) * plm * ang


def harmonic_coefficients(lmax: int, seed: int) -> list[tuple[int, int, float]]:
    """(l, m, c_lm) with c_lm ~ N(0, 1/l^2), drawn in (l = 1..lmax, m = -l..l) order."""
    rng = np.random.default_rng(seed)
    out = []
    for l in range(1, lmax + 1):
        for m in range(-l, l + 1):
            out.append((l, m, float(rng.normal(0.0, 1.0 / l))))
    return out


def br_from_coefficients(t_faces, p_faces, coeffs) -> np.ndarray:
    tc, pc = sample_points(t_faces, p_faces)
    th = tc[:, None]
    ph = pc[None, :]
    br = np.zeros((tc.size, pc.size))
    for l, m, c in coeffs:
        br += c * real_sph_harm(l, m, th, ph)
    return br


def br_harmonics(t_faces, p_faces, lmax: int, seed: int):
    """Br (nt x np, phi fastest) and its coefficient list."""
    coeffs = harmonic_coefficients(lmax, seed)
    return br_from_coefficients(t_faces, p_faces, coeffs), coeffs


def br_dipole(t_faces, p_faces, b0: float = 1.0) -> np.ndarray:
    """Br = b0 cos(theta) sampled at the angular midpoints."""
    tc, pc = sample_points(t_faces, p_faces)
    return b0 * np.cos(tc)[:, None] * np.ones((1, pc.size))


def _unit(theta, phi):
    theta, phi = np.broadcast_arrays(np.asarray(theta, dtype=np.float64), np.asarray(phi, dtype=np.float64))
    st = np.sin(theta)
    return np.stack([st * np.cos(phi), st * np.sin(phi), np.cos(theta)], axis=-1)


def draw_bipoles(n: int, seed: int, fmin: float = 0.01, fmax: float = 1.0, index: float = 1.8,
                 sigma_deg=(2.0, 5.0)):
    """Bipole parameters, drawn per bipole in the order: centre (sin lat, lon),
    tilt, width, flux.  Flux has density ~ F^-index on [fmin, fmax] (inverse CDF)."""
    rng = np.random.default_rng(seed)
    out = []
    e = index - 1.0
    for _ in range(n):
        sinlat = rng.uniform(-1.0, 1.0)
        lon = rng.uniform(0.0, 2.0 * math.pi)
        tilt = rng.uniform(0.0, 2.0 * math.pi)
        sigma = math.radians(rng.uniform(*sigma_deg))
        u = rng.uniform(0.0, 1.0)
        flux = (fmin ** (-e) - u * (fmin ** (-e) - fmax ** (-e))) ** (-1.0 / e)
        out.append((math.asin(sinlat), lon, tilt, sigma, flux))
    return out


def br_bipoles(t_faces, p_faces, nbip: int, seed: int, dipole: float = 5.0) -> np.ndarray:
    """dipole*cos(theta) + sum of Gaussian bipoles; nt x np, phi fastest.

    Each bipole places two spots of opposite sign at great-circle distance
    +-2 sigma from its centre along the tilt bearing; a spot contributes
    +-F/(2 pi sigma^2) exp(-d^2 / (2 sigma^2)) at angular distance d.  Terms are
    evaluated only where d < 12 sigma (exp(-72) ~ 5e-32, below FP64 resolution
    of the sum), and only on the rows and columns that can lie that close, so
    large maps stay cheap.
    """
    tc, pc = sample_points(t_faces, p_faces)
    nt, nph = tc.size, pc.size
    br = dipole * np.cos(tc)[:, None] * np.ones((1, nph))
    if nbip == 0:
        return br
    pts = _unit(tc[:, None], pc[None, :])            # nt x np x 3
    for lat, lon, tilt, sigma, flux in draw_bipoles(nbip, seed):
        c = _unit(np.array(math.pi / 2 - lat), np.array(lon))
        north = np.array([-math.sin(lat) * math.cos(lon), -math.sin(lat) * math.sin(lon), math.cos(lat)])
        east = np.array([-math.sin(lon), math.cos(lon), 0.0])
        t = math.cos(tilt) * north + math.sin(tilt) * east
        delta = 2.0 * sigma
        amp = flux / (2.0 * math.pi * sigma * sigma)
        reach = 12.0 * sigma
        for sgn in (1.0, -1.0):
            s = math.cos(delta) * c + sgn * math.sin(delta) * t
            s /= np.linalg.norm(s)
            scol = math.acos(max(-1.0, min(1.0, s[2])))
            # rows that can be within reach of the spot centre
            jlo = np.searchsorted(tc, scol - reach, side="left")
            jhi = np.searchsorted(tc, scol + reach, side="right")
            if jhi <= jlo:
                continue
            # columns that can be within reach: a point within angular
            # distance R of a centre at colatitude c differs from it in
            # longitude by at most asin(sin R / sin c) when the cap misses the
            # poles (otherwise every column); 0.01 rad of margin covers rounding
            slon = math.atan2(s[1], s[0])
            if scol - reach > 0.0 and scol + reach < math.pi:
                half = math.asin(min(1.0, math.sin(reach) / math.sin(scol))) + 0.01
                dl = np.abs(np.remainder(pc - slon + math.pi, 2.0 * math.pi) - math.pi)
                cols = np.nonzero(dl <= half)[0]
            else:
                cols = np.arange(nph)
            if cols.size == 0:
                continue
            sub = pts[jlo:jhi][:, cols]
            chord = np.linalg.norm(sub - s, axis=-1)
            d = 2.0 * np.arcsin(np.minimum(1.0, 0.5 * chord))
            m = d < reach
            contrib = np.zeros_like(d)
            contrib[m] = sgn * amp * np.exp(-0.5 * (d[m] / sigma) ** 2)
            br[jlo:jhi, cols] += contrib
    return br
