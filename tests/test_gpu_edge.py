"""Degenerate and ragged inputs on the GPU, through the C-ABI.

- A 3 x 3 periodic mesh (36 nodes: fewer than one streaming tile, padded to
  1792 slots, elements that touch their own periodic images) of triangles and
  of quadrilaterals, from a perturbed state: FP64 within 1e-12 of the oracle
  after 20 steps, masks identical; FP32 density within 1e-5.
- step(0) changes nothing.
- A batch of that tiny case with a larger one of the other size class
  advances each exactly as on its own.
- The largest batch, 255 cases (the case index is one byte), in both schedule
  families: sampled cases at both ends and the middle within 1e-12 of the
  oracle; 256 cases are refused.
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




def _tiny(elem, n=3, seed=5):
    c = cases.uniform(nx=n, ny=n, paper=True, elem=elem)
    rng = np.random.default_rng(seed)
    N = c["mesh"].n_nodes
    init = c["init"]
    u = c["params"]["u_inf"][0]
    c["init"] = dict(rho=init["rho"] * (1 + 0.01 * rng.standard_normal(N)),
                     ux=init["ux"] + 0.01 * u * rng.standard_normal(N),
                     uy=0.01 * u * rng.standard_normal(N),
                     T=init["T"] * (1 + 0.01 * rng.standard_normal(N)))
    return c


@pytest.mark.parametrize("elem", ["p2", "q2"])
def test_mesh_smaller_than_one_tile(alelb, oracle_mod, elem):
    c = _tiny(elem)
    print(f"tiny {elem}: {c['mesh'].n_nodes} nodes", flush=True)
    s = alelb.Solver(c["mesh"].arrays(), c["params"], precision="fp64", flags=alelb.F_KEEP_MASKS)
    o = oracle_mod.Oracle(c["mesh"].arrays(), c["params"])
    assert s.info()["slots"] == 1792
    s.init_fields(**c["init"])
    o.init_fields(**c["init"])
    s.step(20)
    o.step(20)
    _, gmw, gmf = s.streamed(masks=True)
    _, omw, omf = o.streamed()
    np.testing.assert_array_equal(gmw, omw)
    np.testing.assert_array_equal(gmf, omf)
    gp, gm, _, gst = s.state()
    op, om, _, ost = o.state()
    assert gst == ost == 20
    assert rel_fields(gp, op) < TOL64 and rel_fields(gm, om) < TOL64
    s.close()
    s = alelb.Solver(c["mesh"].arrays(), c["params"], precision="fp32")
    s.init_fields(**c["init"])
    s.step(20)
    orho = o.fields()[0]
    assert float(np.max(np.abs(s.fields()[0] - orho) / orho)) < TOL32_RHO
    s.close()


def test_step_zero_changes_nothing(alelb):
    c = _tiny("p2")
    s = alelb.Solver(c["mesh"].arrays(), c["params"], precision="fp64", flags=alelb.F_GRAPH)
    s.init_fields(**c["init"])
    s.step(3)
    before = s.state()
    s.step(0)
    after = s.state()
    np.testing.assert_array_equal(before[0], after[0])
    np.testing.assert_array_equal(before[1], after[1])
    assert before[2:] == after[2:]
    s.close()


def test_tiny_and_larger_case_in_one_batch(alelb):
    cs = [_tiny("p2"), cases.small("vortex", n=20, beta=2.0)]
    alone = []
    for c in cs:
        s = alelb.Solver(c["mesh"].arrays(), c["params"], precision="fp64")
        s.init_fields(**c["init"])
        s.step(10)
        alone.append(s.state()[0])
        s.close()
    s = alelb.Solver([c["mesh"].arrays() for c in cs], [c["params"] for c in cs], precision="fp64",
                     flags=alelb.F_GRAPH)
    s.init_fields(**cases.concat_init([c["init"] for c in cs]))
    s.step(10)
    pops = s.state()[0]
    n0 = cs[0]["mesh"].n_nodes
    np.testing.assert_array_equal(pops[:, :n0], alone[0])
    np.testing.assert_array_equal(pops[:, n0:], alone[1])
    s.close()


def test_set_times_per_case(alelb):
    cs = [_tiny("p2"), _tiny("p2", seed=6)]
    s = alelb.Solver([c["mesh"].arrays() for c in cs], [c["params"] for c in cs], precision="fp64")
    s.init_fields(**cases.concat_init([c["init"] for c in cs]))
    lib = alelb.load()
    import ctypes as C
    bad = np.array([1.0, np.nan])
    assert lib.ale_lb_set_times(s.h, bad.ctypes.data_as(C.c_void_p), 2) == alelb.EINVAL
    assert lib.ale_lb_set_times(s.h, bad.ctypes.data_as(C.c_void_p), 1) == alelb.EINVAL
    s.set_times([0.5, 0.75])
    np.testing.assert_array_equal(s.times(), [0.5, 0.75])
    dt = cs[0]["params"]["dt"]
    s.step(2)
    np.testing.assert_allclose(s.times(), [0.5 + 2 * dt, 0.75 + 2 * dt], rtol=0, atol=1e-15)
    s.close()


def test_largest_batch(alelb, oracle_mod):
    cs = [_tiny("p2", seed=100 + k) for k in range(255)]
    meshes = [c["mesh"].arrays() for c in cs]
    params = [c["params"] for c in cs]
    init = cases.concat_init([c["init"] for c in cs])
    n = cs[0]["mesh"].n_nodes
    ref = {}
    for k in (0, 127, 254):
        o = oracle_mod.Oracle(meshes[k], params[k])
        o.init_fields(**cs[k]["init"])
        o.step(10)
        ref[k] = o.state()
    for sched in (None, (2, 1, 256, 0, 3)):
        print(f"255 cases, schedule {sched}", flush=True)
        s = alelb.Solver(meshes, params, precision="fp64", flags=alelb.F_GRAPH)
        assert s.info()["slots"] == 255 * 1792
        if sched:
            s.set_schedule(*sched)
        s.init_fields(**init)
        s.step(10)
        pops, mac, _, step = s.state()
        assert step == 10
        for k, (op, om, _, _) in ref.items():
            sl = slice(k * n, (k + 1) * n)
            assert rel_fields(pops[:, sl], op) < TOL64 and rel_fields(mac[:, sl], om) < TOL64, (sched, k)
        s.close()
    with pytest.raises(alelb.AleLbError) as e:
        alelb.Solver(meshes + meshes[:1], params + params[:1], precision="fp64")
    assert e.value.code == alelb.EINVAL
