"""Batched cases and graph replay on the GPU, through the C-ABI.

A batch advances independent cases (own mesh, time step, viscosity, free
stream and motion parameters) with every launch.  Each case must match the
FP64 oracle run on that case alone to 1e-12 relative, and a case must give
bit-identical results inside a batch and on its own (the kernels do the same
arithmetic in the same order).  Replaying the captured two-step graph must give
bit-identical results to eager launches.
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


@pytest.fixture(scope="module")
def ens():
    # four meshes of uneven size (about 21k-27k nodes: the airfoil surface
    # resolution sets the smallest mesh), each padded to a multiple of 1792 slots
    return cases.ensemble(n_cases=4, n_min=2000, n_max=20_000, seed=7)




def _split(arr, sizes):
    out, o = [], 0
    for n in sizes:
        out.append(arr[..., o:o + n])
        o += n
    return out


def test_batch_parity_per_case_fp64(alelb, oracle_mod, ens):
    ms = [m.arrays() for m in ens["meshes"]]
    sizes = [m.n_nodes for m in ens["meshes"]]
    print(f"batch sizes {sizes}", flush=True)
    s = alelb.Solver(ms, ens["params"], precision="fp64", flags=alelb.F_KEEP_MASKS)
    info = s.info()
    assert info["cases"] == 4 and info["nodes"] == sum(sizes) and info["slots"] % 1792 == 0
    s.init_fields(**cases.concat_init(ens["inits"]))
    os_ = []
    for c in range(4):
        o = oracle_mod.Oracle(ms[c], ens["params"][c])
        o.init_fields(**ens["inits"][c])
        os_.append(o)
    for rnd in range(2):
        s.step(20)
        for o in os_:
            o.step(20)
        gp, gm, _, gstep = s.state()
        assert gstep == 20 * (rnd + 1)
        gps, gms = _split(gp, sizes), _split(gm, sizes)
        for c, o in enumerate(os_):
            op, om, ot, _ = o.state()
            print(f"case {c} step {20 * (rnd + 1)}: pops {rel_fields(gps[c], op):.2e} macros {rel_fields(gms[c], om):.2e}",
                  flush=True)
            assert rel_fields(gms[c], om) < TOL64, c
            assert rel_fields(gps[c], op) < TOL64, c
    _, mw, mf = s.streamed(masks=True)
    for c, (w, f) in enumerate(zip(_split(mw, sizes), _split(mf, sizes))):
        _, ow, of = os_[c].streamed()
        np.testing.assert_array_equal(w, ow)
        np.testing.assert_array_equal(f, of)
    t = s.times()
    fb = s.forces_batch()
    for c, o in enumerate(os_):
        assert abs(t[c] - 40 * ens["params"][c]["dt"]) < 1e-12
        fo = o.forces()
        assert_forces_match(fb[c], fo, ens["params"][c]["chord"])
    s.close()


def test_case_in_batch_is_bit_identical_to_case_alone(alelb, ens):
    ms = [m.arrays() for m in ens["meshes"]]
    sizes = [m.n_nodes for m in ens["meshes"]]
    b = alelb.Solver(ms, ens["params"], precision="fp32")
    b.init_fields(**cases.concat_init(ens["inits"]))
    b.step(30)
    bp = _split(b.state()[0], sizes)
    for c in (0, 3):
        s = alelb.Solver(ms[c], ens["params"][c], precision="fp32")
        s.init_fields(**ens["inits"][c])
        s.step(30)
        np.testing.assert_array_equal(s.state()[0], bp[c])
        s.close()
    b.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_graph_replay_is_bit_identical_to_eager(alelb, ens, precision):
    ms = [m.arrays() for m in ens["meshes"]]
    init = cases.concat_init(ens["inits"])
    eager = alelb.Solver(ms, ens["params"], precision=precision)
    graph = alelb.Solver(ms, ens["params"], precision=precision, flags=alelb.F_GRAPH, stream=0)
    for s in (eager, graph):
        s.init_fields(**init)
    # odd and even counts, with reads (host synchronisation) between replays
    for n in (7, 6, 1, 9):
        eager.step(n)
        graph.step(n)
        ep, em, et, es = eager.state()
        gp, gm, gt, gs = graph.state()
        print(f"{precision} after +{n}: step {gs}", flush=True)
        assert es == gs and et == gt
        np.testing.assert_array_equal(gp, ep)
        np.testing.assert_array_equal(gm, em)
        np.testing.assert_array_equal(graph.times(), eager.times())
    eager.close()
    graph.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_split_batch_on_two_streams_is_bit_identical(alelb, ens, precision):
    """ALE_LB_F_PIPELINE runs the two halves of the batch staggered on two
    streams; every step must give exactly the serial launches' state, also
    with error checks inside the run and host reads in between."""
    ms = [m.arrays() for m in ens["meshes"]]
    init = cases.concat_init(ens["inits"])
    serial = alelb.Solver(ms, ens["params"], precision=precision)
    split = alelb.Solver(ms, ens["params"], precision=precision,
                         flags=alelb.F_PIPELINE | alelb.F_GRAPH | alelb.F_CHECK_FINITE, check_every=3)
    for s in (serial, split):
        s.init_fields(**init)
    for n in (5, 1, 8):
        serial.step(n)
        split.step(n)
        sp, sm, st, ss = serial.state()
        pp, pm, pt, ps = split.state()
        assert ss == ps and st == pt
        np.testing.assert_array_equal(pp, sp)
        np.testing.assert_array_equal(pm, sm)
        np.testing.assert_array_equal(split.times(), serial.times())
    fs, fp = serial.forces_batch(), split.forces_batch()
    assert [f["cl"] for f in fs] == [f["cl"] for f in fp]
    serial.close()
    split.close()


def test_batch_fp32_density_after_1000_steps(alelb, oracle_mod, ens):
    """FP32 batch within 1e-5 relative density of the FP64 oracle, per case,
    after 1000 steps."""
    ms = [m.arrays() for m in ens["meshes"]]
    sizes = [m.n_nodes for m in ens["meshes"]]
    s = alelb.Solver(ms, ens["params"], precision="fp32", flags=alelb.F_GRAPH, stream=0)
    s.init_fields(**cases.concat_init(ens["inits"]))
    s.step(1000)
    rho = _split(s.fields()[0], sizes)
    for c in range(len(sizes)):
        o = oracle_mod.Oracle(ms[c], ens["params"][c])
        o.init_fields(**ens["inits"][c])
        o.step(1000)
        orho = o.fields()[0]
        err = float(np.max(np.abs(rho[c] - orho) / orho))
        print(f"case {c} ({sizes[c]} nodes): FP32 max rel density error {err:.3e}", flush=True)
        assert err < TOL32_RHO, (c, err)
    s.close()
