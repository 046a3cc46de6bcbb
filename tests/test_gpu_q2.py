"""9-node quadrilateral meshes (the paper's element, Sec. III) on the GPU
against the FP64 CPU oracle, through the C-ABI.

Same bar as the triangle path: FP64 within 1e-12 relative per array,
missing-direction masks exact (integer decisions), FP32 within 1e-5 relative
density after 1000 steps.  Quadrilateral handles run the one-wave streaming
schedule only.
"""

import numpy as np
import pytest
from conftest import assert_forces_match, rel_fields

from paper_2002_04353_amd import cases

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32_RHO = 1e-5


@pytest.fixture(scope="module")
def alelb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_2002_04353_amd import alelb as A
    A.load()
    return A




def _pair(alelb, oracle_mod, c, precision="fp64", flags=0, oflags=0):
    s = alelb.Solver(c["mesh"].arrays(), c["params"], precision=precision, flags=flags | alelb.F_KEEP_MASKS)
    o = oracle_mod.Oracle(c["mesh"].arrays(), c["params"], flags=oflags)
    s.init_fields(**c["init"])
    o.init_fields(**c["init"])
    return s, o


SMALL = {
    "uniform_paper": lambda: cases.uniform(nx=25, ny=20, paper=True, elem="q2"),
    "vortex": lambda: cases.small("vortex", n=28, beta=2.0, elem="q2"),
    "plunge": lambda: cases.small("plunge", elem="q2"),
    "pitch_blend": lambda: cases.pitch(n_nodes=20_000, first=0.5, Ma=0.3, Re=2e3, A_deg=10.0, k=2.0, h_c=0.1,
                                       phase_h=0.5, r0_c=0.5, r1_c=3.0, elem="q2", mesh_kw=cases.SMALL_QUADS),
}


@pytest.mark.parametrize("name", list(SMALL))
def test_q2_one_step_parity_fp64(alelb, oracle_mod, name):
    c = SMALL[name]()
    print(f"q2 case {name} nodes {c['mesh'].n_nodes}", flush=True)
    s, o = _pair(alelb, oracle_mod, c)
    s.step(1)
    o.step(1)
    gs, gmw, gmf = s.streamed(masks=True)
    os_, omw, omf = o.streamed()
    np.testing.assert_array_equal(gmw, omw)
    np.testing.assert_array_equal(gmf, omf)
    assert rel_fields(gs, os_) < TOL64
    gp, gm, gt, gstep = s.state()
    op, om, ot, ostep = o.state()
    assert gstep == ostep == 1 and abs(gt - ot) < 1e-14
    assert rel_fields(gm, om) < TOL64
    W, Xa = s.correction()
    oW, oXa = o.correction()
    assert np.abs(W - oW).max() <= max(TOL64 * np.abs(oW).max(), 1e-15)
    assert np.abs(Xa - oXa).max() <= max(TOL64 * np.abs(oXa).max(), 1e-13)
    assert rel_fields(gp, op) < TOL64
    s.close()


@pytest.mark.parametrize("name", list(SMALL))
def test_q2_multi_step_parity_fp64(alelb, oracle_mod, name):
    c = SMALL[name]()
    print(f"q2 case {name} nodes {c['mesh'].n_nodes}", flush=True)
    s, o = _pair(alelb, oracle_mod, c)
    for k in range(4):
        s.step(25)
        o.step(25)
        gp, gm, _, _ = s.state()
        op, om, _, _ = o.state()
        print(f"{name} step {25 * (k + 1)}: rel diff pops {rel_fields(gp, op):.2e} macros {rel_fields(gm, om):.2e}", flush=True)
        assert rel_fields(gm, om) < TOL64, name
        assert rel_fields(gp, op) < TOL64, name
    if c["mesh"].wall_edges.shape[0]:
        fg, fo = s.forces(), o.forces()
        assert_forces_match(fg, fo, c["params"]["chord"])
    s.close()


def test_q2_propagation_only_parity(alelb, oracle_mod):
    c = SMALL["pitch_blend"]()
    s, o = _pair(alelb, oracle_mod, c, flags=alelb.F_NO_COLLIDE, oflags=oracle_mod.F_NO_COLLIDE)
    s.step(3)
    o.step(3)
    assert rel_fields(s.state()[0], o.state()[0]) < TOL64
    s.close()


def test_q2_fp32_density_after_1000_steps(alelb, oracle_mod):
    """The vortex workload on quadrilaterals (112 x 112 vertices, 50,176
    nodes): FP32 within 1e-5 relative density of the oracle after 1000 steps."""
    c = cases.vortex(elem="q2")
    print(f"q2 vortex nodes {c['mesh'].n_nodes}", flush=True)
    o = oracle_mod.Oracle(c["mesh"].arrays(), c["params"])
    o.init_fields(**c["init"])
    o.step(1000)
    orho = o.fields()[0]
    for prec, tol in (("fp32", TOL32_RHO), ("fp64", TOL64)):
        s = alelb.Solver(c["mesh"].arrays(), c["params"], precision=prec)
        s.init_fields(**c["init"])
        s.step(1000)
        err = float(np.max(np.abs(s.fields()[0] - orho) / orho))
        print(f"{prec}: max rel density error after 1000 steps {err:.3e}", flush=True)
        assert err < tol, (prec, err)
        s.close()


def test_q2_full_size_plunge_one_step_from_gpu_state(alelb, oracle_mod):
    """Plunging NACA0012 on the full-size quadrilateral mesh (~190k nodes):
    200 FP32 steps on the GPU, then one FP64 step from that state on both
    sides."""
    c = cases.plunge(elem="q2")
    print(f"q2 plunge nodes {c['mesh'].n_nodes}", flush=True)
    s32 = alelb.Solver(c["mesh"].arrays(), c["params"], precision="fp32", flags=alelb.F_CHECK_FINITE)
    s32.init_fields(**c["init"])
    s32.step(200)
    pops, mac, t, st = s32.state()
    s32.close()
    s = alelb.Solver(c["mesh"].arrays(), c["params"], precision="fp64", flags=alelb.F_KEEP_MASKS)
    o = oracle_mod.Oracle(c["mesh"].arrays(), c["params"])
    s.set_state(pops, mac, t, st)
    o.set_state(pops, mac, t, st)
    s.step(1)
    o.step(1)
    _, gmw, gmf = s.streamed(masks=True)
    _, omw, omf = o.streamed()
    np.testing.assert_array_equal(gmw, omw)
    np.testing.assert_array_equal(gmf, omf)
    gp, gm, _, _ = s.state()
    op, om, _, _ = o.state()
    assert rel_fields(gp, op) < TOL64
    assert rel_fields(gm, om) < TOL64
    fg, fo = s.forces(), o.forces()
    assert_forces_match(fg, fo, c["params"]["chord"])
    s.close()


def _batch_vs_alone(alelb, cs, steps=20):
    alone = []
    for c in cs:
        s = alelb.Solver(c["mesh"].arrays(), c["params"], precision="fp64")
        s.init_fields(**c["init"])
        s.step(steps)
        alone.append(s.state()[0])
        s.close()
    for flags in (0, alelb.F_GRAPH):
        s = alelb.Solver([c["mesh"].arrays() for c in cs], [c["params"] for c in cs], precision="fp64",
                         flags=flags)
        s.init_fields(**cases.concat_init([c["init"] for c in cs]))
        s.step(steps)
        pops = s.state()[0]
        off = 0
        for c, ref in zip(cs, alone):
            n = c["mesh"].n_nodes
            np.testing.assert_array_equal(pops[:, off:off + n], ref)
            off += n
        s.close()


def test_q2_batch_and_graph_match_single_runs(alelb):
    """Quadrilateral cases batched advance exactly as each alone (periodic
    vortices on different meshes; airfoils at different pitch amplitudes),
    and graph replay matches eager launches bit for bit."""
    _batch_vs_alone(alelb, [cases.small("vortex", n=20, beta=2.0, elem="q2"),
                            cases.small("vortex", n=24, beta=3.0, seed=5, elem="q2")])
    b1 = SMALL["pitch_blend"]()
    b2 = dict(b1)
    p = list(b1["params"]["motion_p"])
    p[0] *= 0.5
    b2["params"] = dict(b1["params"], motion_p=p)
    _batch_vs_alone(alelb, [b1, b2])


def test_q2_schedule_rules(alelb):
    c = cases.small("vortex", n=20, elem="q2")
    s = alelb.Solver(c["mesh"].arrays(), c["params"], precision="fp32")
    s.init_fields(**c["init"])
    with pytest.raises(alelb.AleLbError) as e:
        s.set_schedule(waves=4, rings=1)
    assert e.value.code == alelb.EUNSUPPORTED
    assert s.autotune(reps=3)["waves"] == 0
    s.step(5)
    ref = s.state()[0]
    # every one-wave group count gives the same state
    for g in (1, 4, 8):
        t = alelb.Solver(c["mesh"].arrays(), c["params"], precision="fp32")
        t.set_schedule(0, 0, 128, 0, g)
        t.init_fields(**c["init"])
        t.step(5)
        np.testing.assert_array_equal(t.state()[0], ref)
        t.close()
    assert np.isfinite(s.fields()).all()
    s.close()
