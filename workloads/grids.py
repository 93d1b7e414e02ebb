"""Seeded synthetic grids: face coordinates of the (r, theta, phi) shell mesh.

This module only lays out face positions.  It holds none of the solver's
arithmetic (no cell centres, metric factors or operator weights); the solver
library and the oracle each derive those from the faces on their own.

The paper solves on a nonuniform, logically rectangular spherical grid
(Sec. 2.2 "Finite-Difference") between the solar surface r = 1 and an outer
radius R1 (Sec. 2.1, upper boundary condition).  It does not print its mesh
mappings, so the families below are the stated stand-ins:

* r: geometric-like stretching r_f(s) = r0 + (r1 - r0) (e^{b s} - 1)/(e^b - 1),
  s = c / nr.  With b = 151 ln 1.02 every cell is 1.02x wider than the one
  below at nr = 151; other nr keep the same b (same mapping, refined).
* theta: theta_f(s) = pi s + sin(2 pi s)/4, whose derivative is three times
  larger at the poles than at the equator ("cell ratio up to 3").
* theta uniform: theta_f(s) = pi s.
* phi: uniform on [0, 2 pi].
"""
from __future__ import annotations

import math

import numpy as np

R0 = 1.0
R1 = 2.5
# Stretching exponent: 1.02 growth per cell at nr = 151.
BETA_151 = 151.0 * math.log(1.02)


def r_faces_stretched(nr: int, beta: float = BETA_151, r0: float = R0, r1: float = R1) -> np.ndarray:
    """nr+1 radial faces, exponentially stretched away from r0."""
    if nr < 1:
        raise ValueError("nr must be >= 1")
    s = np.arange(nr + 1, dtype=np.float64) / nr
    if beta == 0.0:
        f = s
    else:
        f = np.expm1(beta * s) / math.expm1(beta)
    r = r0 + (r1 - r0) * f
    r[0] = r0
    r[-1] = r1
    return r


def r_faces_uniform(nr: int, r0: float = R0, r1: float = R1) -> np.ndarray:
    return r_faces_stretched(nr, beta=0.0, r0=r0, r1=r1)


def theta_faces_ratio3(nt: int) -> np.ndarray:
    """nt+1 polar faces from 0 to pi; pole cells are 3x the equator cells."""
    if nt < 1:
        raise ValueError("nt must be >= 1")
    s = np.arange(nt + 1, dtype=np.float64) / nt
    t = math.pi * s + 0.25 * np.sin(2.0 * math.pi * s)
    t[0] = 0.0
    t[-1] = math.pi
    return t


def theta_faces_uniform(nt: int) -> np.ndarray:
    if nt < 1:
        raise ValueError("nt must be >= 1")
    t = math.pi * np.arange(nt + 1, dtype=np.float64) / nt
    t[-1] = math.pi
    return t


def phi_faces_uniform(np_: int) -> np.ndarray:
    if np_ < 1:
        raise ValueError("np must be >= 1")
    p = 2.0 * math.pi * np.arange(np_ + 1, dtype=np.float64) / np_
    p[-1] = 2.0 * math.pi
    return p


def phi_faces_jittered(np_: int, seed: int, amp: float = 0.3) -> np.ndarray:
    """Nonuniform periodic phi faces (for tests of the general case)."""
    rng = np.random.default_rng(seed)
    h = 1.0 + amp * (2.0 * rng.random(np_) - 1.0)
    p = np.concatenate([[0.0], np.cumsum(h)])
    p *= 2.0 * math.pi / p[-1]
    p[0] = 0.0
    p[-1] = 2.0 * math.pi
    return p


def sample_points(t_faces: np.ndarray, p_faces: np.ndarray):
    """Angular positions at which a surface map is sampled: the midpoints of
    the theta and phi faces (the locations of the unknowns next to r = 1)."""
    tc = 0.5 * (t_faces[:-1] + t_faces[1:])
    pc = 0.5 * (p_faces[:-1] + p_faces[1:])
    return tc, pc
