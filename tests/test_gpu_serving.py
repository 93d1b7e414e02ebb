"""GPU: the continuous-batching server against single solves and the oracle.

Bars:
* every result of the server is bitwise the one pot3d_solve returns for the
  same request on its own (same Phi, iteration count, status and true
  residual), in FP64 and FP32-refined mode and in both iteration forms
  (POT3D_ITERATION, read when the server and the contexts are created),
  whatever else shares the GPU;
* every FP64 result meets the single-solve parity bar against the oracle:
  ||Phi - Phi_orc|| <= 1e-8 ||Phi_orc|| at tol 1e-10;
* admission honours the slot count and the device-memory budget, and the
  per-grid contexts are reused.
"""
import numpy as np
import pytest

import oracle
from paper_1709_01126_amd import pot3d as P
from workloads import magnetograms

from test_gpu_parity import GRIDS, label, make_faces

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# a mix of grids: ragged tiles, phi shorter than a wavefront, the 32x64x128 grid
MIX = [GRIDS[3], GRIDS[4], GRIDS[5], GRIDS[2], GRIDS[6], GRIDS[4], GRIDS[3]]


def requests(cases, tol=1e-10, maxit=100_000, seed0=11):
    out = []
    for q, case in enumerate(cases):
        rf, tf, pf = make_faces(*case)
        br = magnetograms.br_bipoles(tf, pf, 20 + 7 * q, seed=seed0 + q)
        out.append((case, rf, tf, pf, br, tol, maxit))
    return out


def alone(reqs, precision):
    res = []
    for case, rf, tf, pf, br, tol, maxit in reqs:
        with P.Solver(rf, tf, pf, precision=precision) as s:
            phi, st, it, rr = s.solve(br, tol, maxit)
        res.append((phi, st, it, rr))
    return res


def run_server(reqs, precision, max_slots, budget=0.0, max_steps=100_000):
    with P.Server(precision=precision, max_slots=max_slots, hbm_budget_bytes=budget) as sv:
        ids = [sv.submit(rf, tf, pf, br, tol, maxit) for _, rf, tf, pf, br, tol, maxit in reqs]
        peak_active = 0
        for _ in range(max_steps):
            active, queued, finished = sv.step()
            peak_active = max(peak_active, active)
            if finished == len(ids):
                break
        stats = sv.stats()
        out = [sv.take(rid) for rid in ids]
    return out, peak_active, stats


@pytest.mark.parametrize("form", ["1", "0"], ids=["one_sweep", "two_pass"])
@pytest.mark.parametrize("precision", [P.FP64, P.FP32_REFINED], ids=["fp64", "fp32_refined"])
def test_server_results_equal_single_solves(precision, form, monkeypatch):
    monkeypatch.setenv("POT3D_ITERATION", form)
    reqs = requests(MIX)
    ref = alone(reqs, precision)
    out, peak, stats = run_server(reqs, precision, max_slots=3)
    print(f"\n[serving] {'fp64' if precision == P.FP64 else 'refined'} form {form}: {len(reqs)} requests, 3 slots, "
          f"{stats['replays']} replays, peak active {peak}, cached contexts {stats['cached_contexts']}", flush=True)
    assert peak == 3
    # iterations per replay: 2 x 16 sweeps in the one-sweep form, 16 pairs of passes in two
    assert stats["graph_iters"] == (32 if form == "1" else 16)
    for (case, *_), (phi_a, st_a, it_a, rr_a), (phi_s, info) in zip(reqs, ref, out):
        assert info["done"] == 1 and info["status"] == st_a == P.OK, (label(case), info)
        assert info["iters"] == it_a, (label(case), info["iters"], it_a)
        assert np.array_equal(phi_s, phi_a), (label(case), np.abs(phi_s - phi_a).max())
        assert info["relres_true"] == rr_a
        assert 0.0 <= info["t_submit"] <= info["t_admit"] <= info["t_done"]
    # the grids repeat: contexts are reused, at least one per distinct grid
    assert len({c[:3] for c in MIX}) <= stats["cached_contexts"] < len(MIX)


def test_server_fp64_matches_oracle():
    reqs = requests([GRIDS[4], GRIDS[5], GRIDS[2]])
    out, _, _ = run_server(reqs, P.FP64, max_slots=4)
    for (case, rf, tf, pf, br, tol, _), (phi, info) in zip(reqs, out):
        ref = oracle.solve(rf, tf, pf, br, tol, 100_000)
        e2 = np.linalg.norm(phi - ref["phi"]) / np.linalg.norm(ref["phi"])
        emax = np.abs(phi - ref["phi"]).max() / np.abs(ref["phi"]).max()
        print(f"[serving vs oracle] {label(case)} iters={info['iters']} (oracle {ref['iters']}) "
              f"err2={e2:.2e} errmax={emax:.2e}", flush=True)
        assert info["status"] == P.OK
        assert e2 <= 1e-8 and emax <= 1e-8
        assert abs(info["iters"] - ref["iters"]) <= max(2, 0.005 * ref["iters"])


def test_server_admission_by_memory_budget():
    # a budget that holds one context of the 32x64x128 grid (8.4 MB of vectors)
    # and a small one, but not two of the large grid: the second large request
    # waits for the first to retire, then reuses its context
    reqs = requests([GRIDS[6], GRIDS[6], GRIDS[4]])
    ref = alone(reqs, P.FP64)
    out, peak, stats = run_server(reqs, P.FP64, max_slots=4, budget=16.5e6)
    info = [o[1] for o in out]
    print(f"\n[serving budget] peak active {peak}, used {stats['used_bytes'] / 1e6:.2f} MB of "
          f"{stats['budget_bytes'] / 1e6:.2f} MB", flush=True)
    assert info[1]["t_admit"] >= info[0]["t_done"]
    assert peak <= 2
    assert stats["used_bytes"] <= stats["budget_bytes"]
    assert stats["cached_contexts"] == 2
    for (phi_a, st_a, it_a, _), (phi_s, inf) in zip(ref, out):
        assert inf["status"] == st_a and inf["iters"] == it_a and np.array_equal(phi_s, phi_a)


def test_server_edge_cases():
    case = GRIDS[4]
    rf, tf, pf = make_faces(*case)
    nr, nt, np_ = case[:3]
    br = magnetograms.br_bipoles(tf, pf, 30, seed=5)
    bad = br.copy()
    bad[2, 3] = np.inf
    with P.Server(precision=P.FP64, max_slots=2) as sv:
        ids = {
            "zero": sv.submit(rf, tf, pf, np.zeros((nt, np_)), 1e-10, 100),
            "cap": sv.submit(rf, tf, pf, br, 1e-10, 5),
            "inf": sv.submit(rf, tf, pf, bad, 1e-10, 100),
            "maxit0": sv.submit(rf, tf, pf, br, 1e-10, 0),
            "fixed": sv.submit(rf, tf, pf, br, 0.0, 37),
        }
        with pytest.raises(P.Pot3dError):
            sv.submit(rf[:2], tf, pf, br, 1e-10, 10)
        for _ in range(1000):
            if sv.step()[2] == len(ids):
                break
        res = {k: sv.take(v) for k, v in ids.items()}
        assert P.pot3d_server_result(sv.sv, ids["zero"])[0] == P.EINVAL   # forgotten after take
        assert sv.stats()["active"] == 0 and sv.stats()["queued"] == 0
    phi, info = res["zero"]
    assert info["status"] == P.OK and info["iters"] == 0 and np.all(phi == 0)
    assert res["cap"][1]["status"] == P.ENOCONV and res["cap"][1]["iters"] == 5
    assert res["inf"][1]["status"] == P.EBREAKDOWN and res["inf"][1]["iters"] == 0
    assert res["maxit0"][1]["status"] == P.ENOCONV and res["maxit0"][1]["iters"] == 0
    assert res["fixed"][1]["status"] == P.ENOCONV and res["fixed"][1]["iters"] == 37
    with P.Solver(rf, tf, pf) as s:
        for key, (b, tol, maxit) in {"cap": (br, 1e-10, 5), "fixed": (br, 0.0, 37)}.items():
            phi_a, st_a, it_a, _ = s.solve(b, tol, maxit)
            assert np.array_equal(res[key][0], phi_a) and res[key][1]["iters"] == it_a


def test_server_cache_budget():
    # 1 byte: no two solves share a replay; 0: no limit.  Results unchanged.
    reqs = requests([GRIDS[4], GRIDS[5], GRIDS[3], GRIDS[4]])
    ref = alone(reqs, P.FP64)
    for budget, want_peak in ((1.0, 1), (0.0, 4)):
        with P.Server(precision=P.FP64, max_slots=4) as sv:
            sv.set_cache_budget(budget)
            ids = [sv.submit(rf, tf, pf, br, tol, maxit) for _, rf, tf, pf, br, tol, maxit in reqs]
            peak = 0
            for _ in range(100_000):
                active, _, finished = sv.step()
                peak = max(peak, active)
                if finished == len(ids):
                    break
            out = [sv.take(rid) for rid in ids]
            with pytest.raises(P.Pot3dError):
                sv.set_cache_budget(-1.0)
        assert peak == want_peak, (budget, peak)
        for (phi_a, st_a, it_a, _), (phi_s, info) in zip(ref, out):
            assert info["status"] == st_a and info["iters"] == it_a and np.array_equal(phi_s, phi_a)


def test_server_small_requests_pass_a_waiting_large_one():
    """Streaming budget 250 kB: two 6x10x40 solves (96 kB each in the one-sweep
    form) fit side by side, a 20x37x101 solve (3.1 MB) fits only alone.  Small
    requests queued behind the large one are admitted before it, up to 8 of
    them, then it waits at the head; every result is still bitwise the single
    solve's."""
    small, large = GRIDS[3], GRIDS[4]
    reqs = requests([small, large] + [small] * 10)
    ref = alone(reqs, P.FP64)
    with P.Server(precision=P.FP64, max_slots=4) as sv:
        sv.set_cache_budget(250e3)
        ids = [sv.submit(rf, tf, pf, br, tol, maxit) for _, rf, tf, pf, br, tol, maxit in reqs]
        for _ in range(100_000):
            if sv.step()[2] == len(ids):
                break
        out = [sv.take(rid) for rid in ids]
    t_admit = [o[1]["t_admit"] for o in out]
    before = sum(t < t_admit[1] for t in t_admit[2:])
    print(f"\n[serving] small requests admitted before the waiting large one: {before}", flush=True)
    assert 1 <= before <= 8
    assert all(t >= t_admit[1] for t in t_admit[2 + before:])
    for (phi_a, st_a, it_a, _), (phi_s, info) in zip(ref, out):
        assert info["status"] == st_a == P.OK and info["iters"] == it_a and np.array_equal(phi_s, phi_a)
