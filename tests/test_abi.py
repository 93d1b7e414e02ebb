"""C-ABI library: loads, exports every declared entry point, rejects bad
arguments before touching a device (CPU only; no compute calls)."""
import ctypes
import math
import os
import re
import subprocess
import sys

import numpy as np
import pytest

from paper_1709_01126_amd import pot3d as P
from workloads import grids

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pot3d.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\**\s*(pot3d_[a-z_0-9]+)\s*\(", src, flags=re.M)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("pot3d_create", "pot3d_solve", "pot3d_solve_device", "pot3d_destroy", "pot3d_last_error"):
        assert n in names
    assert set(names) == set(P.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = P.load()
    for n in declared_functions():
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", P.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (pot3d_\w+)", out))
    assert set(declared_functions()) <= exported


def test_version():
    assert "gfx950" in P.pot3d_version()


def good_faces():
    return grids.r_faces_stretched(4), grids.theta_faces_ratio3(6), grids.phi_faces_uniform(8)


def create_status(rf, tf, pf, upper=0, prec=0):
    st, ctx = P.pot3d_create(rf, tf, pf, upper, prec, 0)
    assert ctx is None
    return st


@pytest.mark.parametrize("mutate", [
    "r_nonmonotone", "r_nan", "r_nonpositive", "t_not_zero", "t_not_pi", "t_nonmonotone",
    "p_span", "p_nonmonotone", "nr_small", "nt_small", "np_small", "bad_upper", "bad_precision",
])
def test_create_rejects_invalid_input(mutate):
    rf, tf, pf = good_faces()
    rf, tf, pf = rf.copy(), tf.copy(), pf.copy()
    upper, prec = 0, 0
    if mutate == "r_nonmonotone":
        rf[2] = rf[1]
    elif mutate == "r_nan":
        rf[3] = np.nan
    elif mutate == "r_nonpositive":
        rf = rf - 2.0
    elif mutate == "t_not_zero":
        tf[0] = 0.01
    elif mutate == "t_not_pi":
        tf[-1] = math.pi - 0.01
    elif mutate == "t_nonmonotone":
        tf[2], tf[3] = tf[3], tf[2]
    elif mutate == "p_span":
        pf = pf * 0.5
    elif mutate == "p_nonmonotone":
        pf[4] = pf[3]
    elif mutate == "nr_small":
        rf = rf[:2]
    elif mutate == "nt_small":
        tf = np.array([0.0, math.pi])
    elif mutate == "np_small":
        pf = np.array([0.0, math.pi, 2 * math.pi])
    elif mutate == "bad_upper":
        upper = 7
    elif mutate == "bad_precision":
        prec = 9
    assert create_status(rf, tf, pf, upper, prec) == P.EINVAL
    assert P.pot3d_last_error(None) != ""


def test_closed_wall_passes_validation():
    """The closed-wall upper boundary is a valid argument: without a GPU the
    call gets as far as the device check (EDEVICE), not EINVAL."""
    rf, tf, pf = good_faces()
    st, ctx = P.pot3d_create(rf, tf, pf, P.UPPER_CLOSED_WALL, P.FP64, 0)
    if ctx is not None:
        P.pot3d_destroy(ctx)
    assert st != P.EINVAL


def test_null_arguments():
    lib = P.load()
    out = ctypes.c_void_p(None)
    d = ctypes.POINTER(ctypes.c_double)()
    assert lib.pot3d_create(d, 4, d, 6, d, 8, 0, 0, 0, ctypes.byref(out)) == P.EINVAL
    rf, tf, pf = good_faces()
    assert lib.pot3d_create(P._dp(rf), 4, P._dp(tf), 6, P._dp(pf), 8, 0, 0, 0, None) == P.EINVAL
    phi = np.empty(4 * 6 * 8)
    br = np.zeros(6 * 8)
    assert lib.pot3d_solve(None, P._dp(br), 1e-10, 10, None, P._dp(phi), None, None) == P.EINVAL
    assert P.pot3d_solve_device(None, 1, None, 1, None, 1e-10, 10)[0] == P.EINVAL
    assert P.pot3d_apply_device(None, 1, 2) == P.EINVAL
    assert P.pot3d_precondition_device(None, 1, 2) == P.EINVAL
    assert P.pot3d_set_preconditioner(None, P.PC_PHI_LINE) == P.EINVAL
    assert P.pot3d_rhs_device(None, 1, 2) == P.EINVAL
    north, south = np.empty(4), np.empty(4)
    assert lib.pot3d_pole_values(None, P._dp(north), P._dp(south)) == P.EINVAL
    assert P.pot3d_get_stats(None)[0] == P.EINVAL
    assert P.pot3d_time_kernels(None, 3)[0] == P.EINVAL
    assert P.pot3d_set_refinement_mode(None, P.REFINE_RELIABLE) == P.EINVAL
    assert P.pot3d_set_iteration(None, P.ITER_ONE_SWEEP) == P.EINVAL
    assert P.pot3d_field_device(None, 1, 2, 3) == P.EINVAL
    P.pot3d_destroy(None)


def test_server_rejects_invalid_arguments():
    lib = P.load()
    out = ctypes.c_void_p(None)
    assert lib.pot3d_server_create(0, 0, 4, 0.0, None) == P.EINVAL
    for prec, slots, budget in [(9, 4, 0.0), (0, 0, 0.0), (0, 65, 0.0), (1, 4, -1.0), (0, 4, math.inf),
                                (0, 4, math.nan)]:
        assert lib.pot3d_server_create(0, prec, slots, budget, ctypes.byref(out)) == P.EINVAL, (prec, slots, budget)
        assert out.value is None
        assert P.pot3d_server_last_error(None) != ""
    rf, tf, pf = good_faces()
    br = np.zeros(6 * 8)
    assert P.pot3d_server_submit(None, rf, tf, pf, br, 1e-10, 10)[0] == P.EINVAL
    assert P.pot3d_server_step(None)[0] == P.EINVAL
    assert P.pot3d_server_result(None, 1)[0] == P.EINVAL
    assert P.pot3d_server_get_stats(None)[0] == P.EINVAL
    assert P.pot3d_server_set_cache_budget(None, 1e9) == P.EINVAL
    P.pot3d_server_destroy(None)


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU; asking for more exits with a message
    before touching a device."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    res = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr or "single device" in res.stderr


# ---------------------------------------------------------------------------
# The Python marshalling checks sizes, dtypes, layout and device before any C
# call: the library reads nt*np or N doubles through the pointers it is given,
# so a wrong array must never reach it.

FAKE_CTX = 0x7E57   # never dereferenced: every call below must raise first


@pytest.fixture
def fake_ctx():
    P._CTX_SHAPE[FAKE_CTX] = (4, 6, 8, 0)
    yield FAKE_CTX
    P._CTX_SHAPE.pop(FAKE_CTX, None)


def test_host_solve_rejects_wrong_sizes(fake_ctx):
    n = 4 * 6 * 8
    good_br, phi = np.zeros(6 * 8), np.empty(n)
    with pytest.raises(ValueError, match="br"):
        P.pot3d_solve(fake_ctx, np.zeros(6 * 8 - 1), 1e-10, 10, None, phi)
    with pytest.raises(ValueError, match="phi0"):
        P.pot3d_solve(fake_ctx, good_br, 1e-10, 10, np.zeros(n + 1), phi)
    with pytest.raises(ValueError, match="phi"):
        P.pot3d_solve(fake_ctx, good_br, 1e-10, 10, None, np.empty(n - 1))
    with pytest.raises(ValueError, match="phi"):
        P.pot3d_solve(fake_ctx, good_br, 1e-10, 10, None, np.empty(n, dtype=np.float32))
    with pytest.raises(ValueError, match="phi"):
        P.pot3d_solve(fake_ctx, good_br, 1e-10, 10, None, np.empty((2 * n,))[::2])
    with pytest.raises(ValueError, match="radial"):
        P.pot3d_pole_values(fake_ctx, 5)


def test_unknown_context_is_rejected():
    with pytest.raises(ValueError, match="context"):
        P.pot3d_solve(0x1234, np.zeros(48), 1e-10, 10, None, np.empty(192))


def test_solver_methods_reject_bad_tensors():
    torch = pytest.importorskip("torch")
    s = object.__new__(P.Solver)   # no context: the checks come first
    s.ctx, s.nr, s.nt, s.np, s.device = None, 4, 6, 8, 0
    cpu = torch.zeros(4 * 6 * 8, dtype=torch.float64)
    with pytest.raises(ValueError, match="cuda"):
        s.solve_device(torch.zeros(48, dtype=torch.float64), cpu, 1e-10, 10)
    with pytest.raises(ValueError, match="cuda"):
        s.apply(cpu, cpu)
    with pytest.raises(ValueError, match="cuda"):
        s.rhs(torch.zeros(48, dtype=torch.float64), cpu)
    with pytest.raises(ValueError, match="tensor"):
        s.apply(np.zeros(192), cpu)


def test_tensor_check_order_and_messages():
    """The tensor check itself, on CPU tensors pretending to be on a device:
    dtype, layout and element count are each rejected."""
    torch = pytest.importorskip("torch")

    class OnDevice:
        """A CPU tensor reported as cuda:0 (the check reads is_cuda/device)."""
        def __init__(self, t):
            self.t = t

    t = torch.zeros(10, dtype=torch.float64)
    with pytest.raises(ValueError, match="cuda"):
        P._dev_tensor(t, 10, 0, "x")
    with pytest.raises(ValueError, match="torch tensor"):
        P._dev_tensor(OnDevice(t), 10, 0, "x")


def test_server_submit_rejects_wrong_sizes():
    rf, tf, pf = good_faces()
    with pytest.raises(ValueError, match="br"):
        P.pot3d_server_submit(None, rf, tf, pf, np.zeros(5), 1e-9, 100)
    with pytest.raises(ValueError, match="phi_out"):
        P.pot3d_server_submit(None, rf, tf, pf, np.zeros(6 * 8), 1e-9, 100, np.empty(3))


def test_noalloc_rejects_invalid_arguments_before_device_work():
    rf, tf, pf = good_faces()
    st, _, _ = P.pot3d_solve_noalloc(rf, tf, pf, P.UPPER_SOURCE_SURFACE, None, None, 1, None, 1e-10, 10)
    assert st == P.EINVAL
    st, _, _ = P.pot3d_solve_noalloc(rf, tf, pf, P.UPPER_SOURCE_SURFACE, 1, None, 2, None, -1.0, 10)
    assert st == P.EINVAL
    st, _, _ = P.pot3d_solve_noalloc(rf, tf, pf, 7, 1, None, 2, None, 1e-10, 10)
    assert st == P.EINVAL
    bad = rf.copy()
    bad[2] = bad[1]
    st, _, _ = P.pot3d_solve_noalloc(bad, tf, pf, P.UPPER_SOURCE_SURFACE, 1, None, 2, None, 1e-10, 10)
    assert st == P.EINVAL
    big = grids.r_faces_stretched(5000)
    st, _, _ = P.pot3d_solve_noalloc(big, tf, pf, P.UPPER_SOURCE_SURFACE, 1, None, 2, None, 1e-10, 10)
    assert st == P.EINVAL and "no-allocation" in P.pot3d_last_error(None)
