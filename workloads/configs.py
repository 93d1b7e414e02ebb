"""The named synthetic workloads (grid + surface map + tolerance), seeded.

| name  | grid (nr x nt x np) | r / theta mapping      | Br                                  | tol   |
|-------|---------------------|------------------------|-------------------------------------|-------|
| small | 32 x 64 x 128       | stretched / uniform    | harmonics l = 1..8, N(0, 1/l^2)     | 1e-10 |
| c151  | 151 x 301 x 601     | 1.02 per cell / ratio 3| dipole 5 + 200 power-law bipoles    | 1e-10 |
| c301  | 301 x 641 x 1281    | same mapping / ratio 3 | dipole 5 + 2000 power-law bipoles   | 1e-9  |
| mixed | = c151 (FP32 inner PCG, FP64 outer correction)                              | 1e-10 |
| serve | sizes from {64x128x256, 101x201x401, 151x301x601}, 50..500 bipoles          | 1e-9  |

The paper's own case (Sec. 4.1) is 200 x 720 x 1440 with an observed surface
map at relative tolerance 1e-9; these stand in for it with seeded data.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import grids, magnetograms


_BR_CACHE: dict = {}


@dataclass(frozen=True)
class Workload:
    name: str
    nr: int
    nt: int
    np: int
    tol: float
    seed: int
    theta_map: str      # "uniform" | "ratio3"
    br_kind: str        # "harmonics" | "bipoles" | "dipole"
    nbip: int = 0
    lmax: int = 8

    @property
    def n(self) -> int:
        return self.nr * self.nt * self.np

    def faces(self):
        rf = grids.r_faces_stretched(self.nr)
        tf = grids.theta_faces_uniform(self.nt) if self.theta_map == "uniform" else grids.theta_faces_ratio3(self.nt)
        pf = grids.phi_faces_uniform(self.np)
        return rf, tf, pf

    def br(self, faces=None) -> np.ndarray:
        rf, tf, pf = faces if faces is not None else self.faces()
        if self.br_kind == "harmonics":
            return magnetograms.br_harmonics(tf, pf, self.lmax, self.seed)[0]
        if self.br_kind == "bipoles":
            # large maps take tens of seconds to sample: keep one copy per
            # workload for the process (a copy is returned)
            key = (self.name, self.nbip, self.seed, tf.tobytes(), pf.tobytes())
            if key not in _BR_CACHE:
                if len(_BR_CACHE) >= 4:
                    _BR_CACHE.clear()
                _BR_CACHE[key] = magnetograms.br_bipoles(tf, pf, self.nbip, self.seed)
            return _BR_CACHE[key].copy()
        if self.br_kind == "dipole":
            return magnetograms.br_dipole(tf, pf)
        raise ValueError(self.br_kind)

    def describe(self) -> str:
        return f"{self.name}:{self.nr}x{self.nt}x{self.np}"


SMALL = Workload("small_32x64x128", 32, 64, 128, 1e-10, 1, "uniform", "harmonics")
C151 = Workload("bipole_151x301x601", 151, 301, 601, 1e-10, 2, "ratio3", "bipoles", nbip=200)
C301 = Workload("bipole_301x641x1281", 301, 641, 1281, 1e-9, 3, "ratio3", "bipoles", nbip=2000)

WORKLOADS = {w.name: w for w in (SMALL, C151, C301)}

SERVE_SIZES = ((64, 128, 256), (101, 201, 401), (151, 301, 601))


def serve_request(req_id: int, base_seed: int = 5) -> Workload:
    """One request of the serving trace: a seeded size and bipole count."""
    rng = np.random.default_rng(base_seed * 1_000_003 + req_id)
    nr, nt, np_ = SERVE_SIZES[int(rng.integers(0, len(SERVE_SIZES)))]
    nbip = int(rng.integers(50, 501))
    return Workload(f"serve_{req_id}", nr, nt, np_, 1e-9, base_seed + req_id, "ratio3", "bipoles", nbip=nbip)


def poisson_arrivals(count: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson stream with the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))
