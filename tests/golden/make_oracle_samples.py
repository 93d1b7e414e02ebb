"""Write sampled oracle results for a full-size workload to a small JSON fixture
(point-Jacobi PCG, or with --precond phi_line the phi-line block preconditioner).

Calls only ``oracle`` and ``workloads``.  The GPU parity tests at full size
compare the solver's Phi at these seeded indices, its iteration count and its
pole values against the oracle's.  A full oracle solve at that size takes
minutes, too long to repeat inside a test.

    python tests/golden/make_oracle_samples.py bipole_151x301x601
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import WORKLOADS  # noqa: E402

# Fixed-count iterates for parity without stopping.  On this grid two correct
# FP64 CG implementations (this oracle and scipy's) agree to 3e-14 after 20
# iterations but drift apart to ~1e-8 by 50: rounding differences grow fast on
# an ill-conditioned system, so only short fixed counts are compared tightly.
FIXED_KS = (5, 20)


def sample_indices(nr, nt, np_, count=1024, seed=2024):
    rng = np.random.default_rng(seed)
    n = nr * nt * np_
    idx = set(int(v) for v in rng.choice(n, size=count, replace=False))
    # structured points: bottom/top layers, pole rows, the periodic seam
    for i in (0, 1, nr // 2, nr - 2, nr - 1):
        for j in (0, 1, nt // 2, nt - 2, nt - 1):
            for k in (0, 1, np_ // 2, np_ - 2, np_ - 1):
                idx.add((i * nt + j) * np_ + k)
    return np.array(sorted(idx), dtype=np.int64)


def layer_functionals(x, seed=7):
    """Per radial layer: the 2-norm, the plain sum and the dot product with a
    seeded N(0, 1) vector of Phi.  An error confined to a region the sampled
    indices miss still moves these to first order."""
    nr = x.shape[0]
    rng = np.random.default_rng(seed)
    l2, s1, sv = [], [], []
    for i in range(nr):
        xi = np.ascontiguousarray(x[i]).ravel()
        v = rng.standard_normal(xi.size)
        l2.append(float(np.sqrt(oracle.dot(xi, xi))))
        s1.append(float(xi.sum()))
        sv.append(float(oracle.dot(xi, v)))
    return {"seed": seed, "l2": l2, "sum": s1, "dot_randn": sv}


def main(name, solve=True, save_phi=None, precond="jacobi"):
    w = WORKLOADS[name]
    rf, tf, pf = w.faces()
    br = w.br((rf, tf, pf))
    coef = oracle.assemble(rf, tf, pf)
    b = oracle.rhs(rf, tf, pf, br)
    idx = sample_indices(w.nr, w.nt, w.np)
    suffix = "" if precond == "jacobi" else f"_{precond}"
    t0 = time.time()
    fixed = {}
    for K in FIXED_KS:
        xk, itk, rrk, stk = oracle.pcg(coef, b, 0.0, K, precond=precond)
        fixed[str(K)] = {"relres": rrk, "phi": xk.ravel()[idx].tolist(), "phi_max_abs": float(np.abs(xk).max())}
    t1 = time.time()
    if not solve:
        # fixed-count samples only (a full oracle solve at this size takes hours)
        out = {"_source": "oracle/pot3d_oracle.c Jacobi-PCG on the named seeded workload, fixed-count iterates only; "
                          "written by tests/golden/make_oracle_samples.py (calls only oracle/ and workloads/)",
               "workload": name, "nr": w.nr, "nt": w.nt, "np": w.np, "tol": w.tol,
               "indices": idx.tolist(), "fixed": fixed, "oracle_seconds": {"fixed_k": t1 - t0}}
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"oracle_{name}{suffix}.json")
        with open(path, "w") as f:
            json.dump(out, f, indent=None, separators=(",", ":"))
        print(path, t1 - t0)
        return
    x, iters, relres, st = oracle.pcg(coef, b, w.tol, 200_000, precond=precond)
    t2 = time.time()
    if save_phi:
        np.save(save_phi, x)
    north, south = oracle.pole_values(pf, x)
    out = {
        "_source": "oracle/pot3d_oracle.c Jacobi-PCG on the named seeded workload; written by "
                   "tests/golden/make_oracle_samples.py (calls only oracle/ and workloads/)",
        "workload": name, "nr": w.nr, "nt": w.nt, "np": w.np, "tol": w.tol, "precond": precond,
        "status": st, "iters": iters, "relres": relres,
        "true_relres": oracle.true_relres(coef, b, x),
        "phi_max_abs": float(np.abs(x).max()), "phi_l2": float(np.sqrt(oracle.dot(x, x))),
        "indices": idx.tolist(), "phi": x.ravel()[idx].tolist(),
        "fixed": fixed,
        "north": north.tolist(), "south": south.tolist(),
        "layers": layer_functionals(x),
        "oracle_seconds": {"fixed_k": t1 - t0, "solve": t2 - t1},
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"oracle_{name}{suffix}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=None, separators=(",", ":"))
    print(path, iters, relres, out["true_relres"], t2 - t1)


if __name__ == "__main__":
    # python tests/golden/make_oracle_samples.py NAME [--fixed-only] [--save-phi PATH.npy]
    #                                             [--precond phi_line]
    sp = sys.argv[sys.argv.index("--save-phi") + 1] if "--save-phi" in sys.argv else None
    pc = sys.argv[sys.argv.index("--precond") + 1] if "--precond" in sys.argv else "jacobi"
    main(sys.argv[1] if len(sys.argv) > 1 else "bipole_151x301x601", solve="--fixed-only" not in sys.argv,
         save_phi=sp, precond=pc)
