"""GPU: the field B = -grad Phi on the cell faces (pot3d_field_device) against
the oracle's, computed from the same (GPU) Phi.

Bars: each component elementwise within 1e-13 of its max |B| (each value is
one difference times a reciprocal: a few roundings); the discrete Gauss law
on the GPU output (net outward flux = A Phi - b, with A and b from the
oracle) within 1e-12 of the flux scale.
"""
import numpy as np
import pytest

import oracle
from paper_1709_01126_amd import pot3d as P
from workloads import magnetograms

from test_gpu_parity import GRIDS, dev, gpu_solve, label, make_faces
from test_oracle_field import net_outward_flux

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

UPPER = pytest.mark.parametrize("upper", [P.UPPER_SOURCE_SURFACE, P.UPPER_CLOSED_WALL], ids=["source_surface", "closed_wall"])


def compare(phi, rf, tf, pf, br, closed_wall, fields):
    ref = oracle.field(rf, tf, pf, phi, br, closed_wall)
    for name, g, r in zip(("Br", "Bt", "Bp"), fields, ref):
        assert g.shape == r.shape, name
        err = np.abs(g - r).max() / np.abs(r).max()
        assert err <= 1e-13, (name, err)
    net, scale = net_outward_flux(rf, tf, pf, *fields)
    coef = oracle.assemble(rf, tf, pf, closed_wall)
    b = oracle.rhs(rf, tf, pf, br, closed_wall)
    assert np.all(np.abs(net - (oracle.matvec(coef, phi) - b)) <= 1e-12 * scale.max())


@UPPER
@pytest.mark.parametrize("case", GRIDS[2:], ids=label)
def test_field_matches_oracle(case, upper):
    rf, tf, pf = make_faces(*case)
    br = magnetograms.br_bipoles(tf, pf, 25, seed=6) + 0.1
    with P.Solver(rf, tf, pf, upper_bc=upper) as s:
        with pytest.raises(P.Pot3dError):
            s.field()   # no solution yet
        phi, st, it, _ = gpu_solve(s, br, 1e-10, 100_000)
        fields = [f.cpu().numpy() for f in s.field()]
        # after pot3d_rhs_device the b plane is no longer the solve's
        b = torch.empty(case[:3], dtype=torch.float64, device="cuda:0")
        s.rhs(dev(br), b)
        with pytest.raises(P.Pot3dError):
            s.field()
    assert st == P.OK
    compare(phi, rf, tf, pf, br, upper == P.UPPER_CLOSED_WALL, fields)


def test_field_full_size_151x301x601():
    from workloads import C151
    rf, tf, pf = C151.faces()
    br = C151.br((rf, tf, pf))
    with P.Solver(rf, tf, pf) as s:
        phi, st, it, _ = gpu_solve(s, br, 0.0, 20)
        fields = [f.cpu().numpy() for f in s.field()]
    ref = oracle.field(rf, tf, pf, phi, br)
    for name, g, r in zip(("Br", "Bt", "Bp"), fields, ref):
        err = np.abs(g - r).max() / np.abs(r).max()
        print(f"[field full size] {name} max rel diff {err:.2e}", flush=True)
        assert err <= 1e-13, (name, err)
