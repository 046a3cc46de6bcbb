"""The isentropic vortex workload against its analytic solution, through the
C-ABI: 50,176 P2 nodes on the deforming periodic square, Ma 0.3 along the
diagonal, strength 5, 2000 steps, FP64 and FP32 beside the oracle.

The analytic solution is the inviscid vortex translated with the mean flow.
At Re_R = 100 the run is viscous, so the solver's distance from it is the
method's (viscous decay plus discretisation), the same for the oracle and the
GPU: the test checks that the GPU's distance equals the oracle's (FP64 to
1e-9 of it, FP32 to 1e-3 of it), that FP32 stays within 1e-5 relative density
of the oracle after the 2000 steps, and that the vortex is still there where
the mean flow has carried it (its density dip has decayed by less than half,
its minimum within R / 4 of the analytic centre)."""

import numpy as np
import pytest
from conftest import rel_fields

from paper_2002_04353_amd import cases

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def alelb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_2002_04353_amd import alelb as A
    A.load()
    return A


def _distance(rho, ux, uy, ref):
    """L2 distances of density and velocity from the analytic fields, relative
    to the vortex's own deviation from the free stream."""
    ar, au, av, U = ref
    d_rho = np.sqrt(np.mean((rho - ar) ** 2) / np.mean((ar - 1.0) ** 2))
    d_u = np.sqrt(np.mean((ux - au) ** 2 + (uy - av) ** 2) / np.mean((au - U[0]) ** 2 + (av - U[1]) ** 2))
    return d_rho, d_u


def test_vortex_2000_steps_against_the_analytic_solution(alelb, oracle_mod):
    c = cases.vortex()
    steps = 2000
    assert c["steps"] == steps
    v = c["vortex"]
    p = c["params"]
    o = oracle_mod.Oracle(c["mesh"].arrays(), p)
    o.init_fields(**c["init"])
    o.step(steps)
    t = steps * p["dt"]
    code, x, _, _, _ = o.move_mesh(t)
    assert code == 0
    ar, au, av, _ = cases.vortex_fields(x[:, 0], x[:, 1], t, v["L"], v["U"], v["R"], v["beta"], v["T_inf"])
    ref = (ar, au, av, v["U"])
    om = o.fields()
    d_o = _distance(om[0], om[1], om[2], ref)
    print(f"oracle vs analytic after {steps} steps: density {d_o[0]:.4e} velocity {d_o[1]:.4e}", flush=True)
    # The vortex is still there and where the mean flow has carried it: its
    # density dip has decayed (viscously) by less than half, and its minimum
    # lies within R / 4 of the analytic centre on the periodic box.
    dip = (1.0 - om[0].min()) / (1.0 - ar.min())
    L, U, R = v["L"], v["U"], v["R"]
    xc = np.mod(0.5 * L + np.array(U) * t, L)
    dc = np.mod(x[int(np.argmin(om[0]))] - xc + 0.5 * L, L) - 0.5 * L
    print(f"  dip {dip:.3f} of the analytic one, minimum {np.hypot(*dc):.2f} from its centre (R = {R})", flush=True)
    assert 0.5 < dip < 1.02
    assert np.hypot(*dc) < 0.25 * R
    for prec in ("fp64", "fp32"):
        s = alelb.Solver(c["mesh"].arrays(), p, precision=prec)
        s.init_fields(**c["init"])
        s.step(steps)
        gm = s.fields()
        s.close()
        d_g = _distance(gm[0], gm[1], gm[2], ref)
        rho_err = float(np.max(np.abs(gm[0] - om[0]) / om[0]))
        print(f"{prec} vs analytic: density {d_g[0]:.4e} velocity {d_g[1]:.4e}; "
              f"vs oracle: max rel density {rho_err:.2e}, fields {rel_fields(gm, om):.2e}", flush=True)
        tol = 1e-9 if prec == "fp64" else 1e-3
        assert abs(d_g[0] / d_o[0] - 1.0) < tol and abs(d_g[1] / d_o[1] - 1.0) < tol
        assert rho_err < (1e-12 if prec == "fp64" else 1e-5)
