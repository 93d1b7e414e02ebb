"""Mutation check of the oracle's pins (CPU only).

Each case plants one plausible mistake in a copy of oracle/pot3d_oracle.c
(a dropped factor, a wrong face or neighbour index, a swapped ratio, a missing
term), compiles the copy with gcc into a temporary library, and runs a group of
pin tests against it in a child process (the oracle wrapper loads the copy
through POT3D_ORACLE_LIB).  The case passes when at least one pin fails.  The
repository's own oracle is never modified.
"""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "pot3d_oracle.c")

OP = "tests/test_oracle_operator.py"
PCG = "tests/test_oracle_pcg.py"
CF = "tests/test_oracle_closed_form.py"
LINE = "tests/test_oracle_line_jacobi.py"

# (name, text in the oracle, replacement, pin tests that should catch it)
MUTATIONS = [
    ("dropped r^2 on the radial faces",
     "wrp = area_r * rf[i + 1] * rf[i + 1] / (rc[i + 1] - rc[i]);", "wrp = area_r / (rc[i + 1] - rc[i]);",
     [OP]),
    ("wrong radial face in the upper weight",
     "wrp = area_r * rf[i + 1] * rf[i + 1] / (rc[i + 1] - rc[i]);",
     "wrp = area_r * rf[i] * rf[i] / (rc[i + 1] - rc[i]);", [OP]),
    ("wrong theta face index",
     "wtp = dp[k] * dr[i] * sin(tf[j + 1]) / (tc[j + 1] - tc[j]);",
     "wtp = dp[k] * dr[i] * sin(tf[j]) / (tc[j + 1] - tc[j]);", [OP]),
    ("wrong half-cell spacing at the source surface",
     "dtop = area_r * rf[nr] * rf[nr] / (rf[nr] - rc[nr - 1]);",
     "dtop = area_r * rf[nr] * rf[nr] / (rf[nr] - rf[nr - 1]);", [CF + "::test_second_order_convergence"]),
    ("wrong spacing across the phi seam",
     "double sp_minus = (k > 0) ? pc[k] - pc[k - 1] : pc[0] + ORC_TWO_PI - pc[np - 1];",
     "double sp_minus = (k > 0) ? pc[k] - pc[k - 1] : ORC_TWO_PI - pc[np - 1];", [OP]),
    ("wrong radius in the surface flux",
     "rf[0] * rf[0] * br[(long)j * np + k];", "rf[1] * rf[1] * br[(long)j * np + k];", [OP, CF]),
    ("inverted beta",
     "const double beta = rho_new / rho;", "const double beta = rho / rho_new;", [PCG]),
    ("sin(theta) multiplied instead of divided in the phi weight",
     "const double area_p = dr[i] * dt[j] / sin(tc[j]);", "const double area_p = dr[i] * dt[j] * sin(tc[j]);",
     [CF + "::test_second_order_convergence"]),
    ("wrong theta neighbour in the matvec",
     "if (j > 0)      s -= WTM[P] * x[idx3(i, j - 1, k, nt, np)];",
     "if (j > 0)      s -= WTM[P] * x[idx3(i, j + 1 < nt ? j + 1 : j - 1, k, nt, np)];", [OP]),
    ("no preconditioner",
     "for (long P = 0; P < N; P++) z[P] = r[P] / D[P];", "for (long P = 0; P < N; P++) z[P] = r[P];", [PCG]),
    ("phi neighbour does not wrap",
     "const int kp = (k == np - 1) ? 0 : k + 1;\n                    s -= WPM",
     "const int kp = (k == np - 1) ? np - 1 : k + 1;\n                    s -= WPM", [OP]),
    ("D_top left out of the diagonal",
     "D[P] = wrm + wrp + wtm + wtp + wpm + wpp + dtop;", "D[P] = wrm + wrp + wtm + wtp + wpm + wpp;", [OP]),
    ("true residual without the square roots",
     "const double num = sqrt(orc_dot(q, q, N)), den = sqrt(orc_dot(b, b, N));",
     "const double num = orc_dot(q, q, N), den = orc_dot(b, b, N);", [PCG + "::test_true_relres_fixed_values"]),
    ("line solve without the Sherman-Morrison correction",
     "for (int k = 0; k < n; k++) zz[k] = y[k] - f * q[k];", "for (int k = 0; k < n; k++) zz[k] = y[k];", [LINE]),
    ("line solve with a wrong corner sign",
     "const double vy = y[0] - (a[0] / g) * y[n - 1];", "const double vy = y[0] + (a[0] / g) * y[n - 1];", [LINE]),
]


def run_case(case, tmp):
    name, old, new, tests = case
    src = open(SRC).read()
    if src.count(old) != 1:
        return name, "text not found once"
    tag = str(abs(hash(name)))
    csrc = os.path.join(tmp, f"m{tag}.c")
    lib = os.path.join(tmp, f"m{tag}.so")
    with open(csrc, "w") as f:
        f.write(src.replace(old, new))
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-o", lib, csrc, "-lm"], check=True)
    env = dict(os.environ, POT3D_ORACLE_LIB=lib, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu", *tests],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return name, "caught" if r.returncode == 1 else f"not caught (pytest exit {r.returncode})"


def test_every_planted_mistake_fails_a_pin():
    with tempfile.TemporaryDirectory() as tmp, ThreadPoolExecutor(max_workers=4) as ex:
        results = list(ex.map(lambda c: run_case(c, tmp), MUTATIONS))
    missed = [(n, why) for n, why in results if why != "caught"]
    assert not missed, missed
