"""The entry point that allocates nothing (pot3d_solve_noalloc) against the
context solve it mirrors (pot3d_create + pot3d_solve_device), through the C
ABI.  It is meant for callers that cannot allocate device memory; its scratch
is a fixed-size device array that every call on a GPU shares.

Bar (the FP64 solve bar of the parity tests): at tol 1e-10 the two answers
agree to 1e-8 of ||Phi|| in the 2-norm and the max norm, and the iteration
counts within max(2, 0.5 %).  Checked on two calls in a row, the second on a
smaller grid (so the array holds the first call's data when it starts), then
again on the first grid, then with the closed wall and with a warm start.
"""
import ctypes

import numpy as np
import pytest

from paper_1709_01126_amd import pot3d as P
from workloads import grids, magnetograms

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def faces(nr, nt, np_):
    return grids.r_faces_stretched(nr), grids.theta_faces_ratio3(nt), grids.phi_faces_uniform(np_)


def noalloc_solve(rf, tf, pf, br, tol, maxit, upper=P.UPPER_SOURCE_SURFACE, phi0=None):
    nr, nt, np_ = rf.size - 1, tf.size - 1, pf.size - 1
    d_br = torch.from_numpy(np.ascontiguousarray(br)).to("cuda:0")
    d_phi = torch.full((nr, nt, np_), np.nan, dtype=torch.float64, device="cuda:0")
    d_phi0 = None if phi0 is None else torch.from_numpy(np.ascontiguousarray(phi0)).to("cuda:0")
    stream = torch.cuda.current_stream()
    st, it, rr = P.pot3d_solve_noalloc(rf, tf, pf, upper, d_br.data_ptr(),
                                       None if d_phi0 is None else d_phi0.data_ptr(), d_phi.data_ptr(),
                                       stream.cuda_stream, tol, maxit)
    torch.cuda.synchronize()
    return d_phi.cpu().numpy(), st, it, rr


def context_solve(rf, tf, pf, br, tol, maxit, upper=P.UPPER_SOURCE_SURFACE, phi0=None):
    with P.Solver(rf, tf, pf, upper_bc=upper) as s:
        d_phi = torch.empty(s.shape, dtype=torch.float64, device="cuda:0")
        st, it, rr = s.solve_device(torch.from_numpy(np.ascontiguousarray(br)).to("cuda:0"), d_phi, tol, maxit,
                                    phi0=None if phi0 is None else torch.from_numpy(phi0).to("cuda:0"))
        torch.cuda.synchronize()
        return d_phi.cpu().numpy(), st, it, rr


def close(a, b):
    return abs(a - b) <= max(2, int(0.005 * max(a, b)))


def check(shape, seed, upper=P.UPPER_SOURCE_SURFACE, warm=False):
    rf, tf, pf = faces(*shape)
    br, _ = magnetograms.br_harmonics(tf, pf, 4, seed=seed)
    phi0 = None
    if warm:
        phi0 = np.random.default_rng(seed).standard_normal(shape) * 1e-3
    tol = 1e-10
    a, sta, ita, rra = noalloc_solve(rf, tf, pf, br, tol, 100_000, upper, phi0)
    b, stb, itb, rrb = context_solve(rf, tf, pf, br, tol, 100_000, upper, phi0)
    print(f"[no-alloc] {shape} upper={upper} warm={warm}: iters {ita} vs {itb}, true relres {rra:.2e} vs {rrb:.2e}",
          flush=True)
    assert sta == stb == P.OK
    assert close(ita, itb)
    assert np.all(np.isfinite(a))
    assert np.linalg.norm(a - b) <= 1e-8 * np.linalg.norm(b)
    assert np.abs(a - b).max() <= 1e-8 * np.abs(b).max()
    assert abs(rra - rrb) <= 0.05 * rrb + 1e-14


def test_two_calls_second_smaller_then_first_again():
    check((20, 37, 101), 1)
    check((6, 10, 40), 2)
    check((20, 37, 101), 3)


def test_closed_wall_and_warm_start():
    check((9, 33, 129), 4, upper=P.UPPER_CLOSED_WALL)
    check((9, 33, 129), 5, warm=True)


def test_largest_serving_grid_and_limit():
    check((64, 128, 256), 6)
    rf, tf, pf = faces(101, 201, 401)
    st = P.pot3d_solve_noalloc(rf, tf, pf, P.UPPER_SOURCE_SURFACE, 1, None, 2, None, 1e-9, 10)[0]
    assert st == P.EINVAL
    assert "no-allocation" in P.pot3d_last_error(None)
