"""Launch schedules on the GPU, through the C-ABI.

Two families of schedules compute a step.
- One-wave: the streaming kernel walks and gathers in global memory with 1, 4
  or 8 node groups per workgroup, and k_collide forms f* in full.
- Tile: the tile kernel stages each tile's element patch in LDS (128 or 256
  nodes per tile, patch radius 1 or 2, a node's nine directions in 1, 2 or 3
  groups of threads), fuses the part of the collision the
  node's own moments fix, and k_grad2 leaves the correction X for the next
  step to add as it stages.

Within a family every schedule (including the node-kernel block 64/128/256,
and LDS caps that send some or all tiles to the global path) computes the
same values in the same order: the states must be bit-identical.  Across the
families the walks start from different elements (the last step's element,
or the node's owner), so a departure point on a shared edge may be taken from
either neighbour; the two agree to round-off.  Switching family in the middle
of a run converts the state exactly.  Every tile schedule matches the FP64
oracle at 1e-12 per field.
"""

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


@pytest.fixture(scope="module")
def ens():
    return cases.ensemble(n_cases=3, n_min=2000, n_max=40_000, seed=5)


ONE_WAVE = [  # (waves, rings, node_block, lds_limit, groups)
    (0, 0, 128, 0, 4), (0, 0, 64, 0, 8), (0, 0, 256, 0, 1),
]
TILE_REF = (4, 1, 256, 0, 1)
TILES = [  # groups: direction groups of the tile kernel
    (2, 1, 64, 0, 1), (2, 2, 256, 0, 2), (4, 2, 128, 0, 3), (2, 1, 256, 0, 3), (4, 1, 64, 0, 2),
    (4, 1, 256, 4096, 1),   # no room for any patch: every tile on the global path
    (4, 1, 256, 36000, 1),  # a cap below the largest patches: some tiles on the global path
]


def _run(alelb, meshes, params, init, precision, sched, steps, switch=None):
    s = alelb.Solver(meshes, params, precision=precision)
    if sched is not None:
        s.set_schedule(*sched)
    s.init_fields(**init)
    if switch is None:
        s.step(steps)
    else:
        s.step(steps // 2)
        s.set_schedule(*switch)
        s.step(steps - steps // 2)
    pops, mac, t, n = s.state()
    info = s.info()
    s.close()
    return pops, mac, info


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_schedules_within_a_family_are_bit_identical(alelb, ens, precision):
    ms = [m.arrays() for m in ens["meshes"]]
    init = cases.concat_init(ens["inits"])
    for ref, family in ((None, ONE_WAVE), (TILE_REF, TILES)):
        ref_p, ref_m, _ = _run(alelb, ms, ens["params"], init, precision, ref, 12)
        for sched in family:
            p, m, info = _run(alelb, ms, ens["params"], init, precision, sched, 12)
            print(f"{precision} schedule {sched}: global-path tiles {info['global_tiles']}", flush=True)
            np.testing.assert_array_equal(p, ref_p, err_msg=str(sched))
            np.testing.assert_array_equal(m, ref_m, err_msg=str(sched))
            if sched[3] == 4096:
                assert info["global_tiles"] > 0


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_families_agree_and_switch_exactly(alelb, ens, precision):
    ms = [m.arrays() for m in ens["meshes"]]
    init = cases.concat_init(ens["inits"])
    tol = 1e-13 if precision == "fp64" else 2e-6
    one_p, one_m, _ = _run(alelb, ms, ens["params"], init, precision, None, 12)
    til_p, til_m, _ = _run(alelb, ms, ens["params"], init, precision, TILE_REF, 12)
    d = max(rel_fields(til_p, one_p), rel_fields(til_m, one_m))
    print(f"{precision}: tile vs one-wave after 12 steps {d:.2e} "
          f"(bit-identical: {np.array_equal(til_p, one_p)})", flush=True)
    assert d < tol
    # a switch of family converts the state exactly: 6 steps each way equal
    # 6 steps of the first family, a checkpoint blob, and 6 of the second
    for first, second in ((None, TILE_REF), (TILE_REF, (0, 0, 256, 0, 4))):
        p, m, _ = _run(alelb, ms, ens["params"], init, precision, first, 12, switch=second)
        a = alelb.Solver(ms, ens["params"], precision=precision)
        if first is not None:
            a.set_schedule(*first)
        a.init_fields(**init)
        a.step(6)
        blob = a.save_state()
        a.close()
        b = alelb.Solver(ms, ens["params"], precision=precision)
        b.set_schedule(*second)
        b.load_state(blob)
        b.step(6)
        np.testing.assert_array_equal(b.state()[0], p)
        np.testing.assert_array_equal(b.state()[1], m)
        b.close()


@pytest.mark.parametrize("name", ["plunge", "pitch_blend", "vortex"])
def test_tile_schedule_matches_oracle(alelb, oracle_mod, name):
    c = {"plunge": lambda: cases.small("plunge", n_nodes=12000),
         "pitch_blend": lambda: cases.pitch(n_nodes=12000, first=0.5, Ma=0.3, Re=2e3, A_deg=10.0, k=2.0,
                                            h_c=0.1, phase_h=0.5, r0_c=0.5, r1_c=3.0),
         "vortex": lambda: cases.small("vortex", n=28, beta=2.0)}[name]()
    s = alelb.Solver(c["mesh"].arrays(), c["params"], precision="fp64", flags=alelb.F_KEEP_MASKS)
    s.set_schedule(*TILE_REF)
    o = oracle_mod.Oracle(c["mesh"].arrays(), c["params"])
    s.init_fields(**c["init"])
    o.init_fields(**c["init"])
    s.step(1)
    o.step(1)
    gs, gmw, gmf = s.streamed(masks=True)
    os_, omw, omf = o.streamed()
    np.testing.assert_array_equal(gmw, omw)
    np.testing.assert_array_equal(gmf, omf)
    assert rel_fields(gs, os_) < 1e-12
    W, Xa = s.correction()
    oW, oXa = o.correction()
    assert rel_fields(W, oW) < 1e-12 and rel_fields(Xa, oXa) < 1e-12
    for k in range(3):
        s.step(20)
        o.step(20)
        gp, gm, _, _ = s.state()
        op, om, _, _ = o.state()
        print(f"{name} step {1 + 20 * (k + 1)}: pops {rel_fields(gp, op):.2e} macros {rel_fields(gm, om):.2e}",
              flush=True)
        assert rel_fields(gp, op) < 1e-12 and rel_fields(gm, om) < 1e-12
    s.close()


def test_schedules_on_a_periodic_mesh(alelb):
    c = cases.small("vortex", n=28, beta=2.0)
    for ref, family in ((None, [(0, 0, 256, 0, 8)]),
                        (TILE_REF, [(2, 1, 64, 0, 3), (4, 2, 128, 0, 2), (4, 1, 256, 30000, 1)])):
        ref_p, ref_m, _ = _run(alelb, c["mesh"].arrays(), c["params"], c["init"], "fp64", ref, 10)
        for sched in family:
            p, m, info = _run(alelb, c["mesh"].arrays(), c["params"], c["init"], "fp64", sched, 10)
            print(f"vortex schedule {sched}: global-path tiles {info['global_tiles']}", flush=True)
            np.testing.assert_array_equal(p, ref_p, err_msg=str(sched))
            np.testing.assert_array_equal(m, ref_m, err_msg=str(sched))


def test_autotune_choice_and_cache(alelb, ens):
    ms = [m.arrays() for m in ens["meshes"]]
    init = cases.concat_init(ens["inits"])
    s = alelb.Solver(ms, ens["params"], precision="fp32")
    s.init_fields(**init)
    s.autotune(reps=0)  # drop any cached choice of this bucket
    ch = s.autotune(reps=3)
    print(f"autotune: {ch}", flush=True)
    assert ch["waves"] in (0, 2, 4) and ch["node_block"] in (64, 128, 256) and not ch["cached"]
    assert ch["groups"] in ((1, 4, 8) if ch["waves"] == 0 else (1, 2, 3))
    assert ch["ms"] > 0
    sched = (ch["waves"], ch["rings"], ch["node_block"], 0, ch["groups"])
    ref_p, _, _ = _run(alelb, ms, ens["params"], init, "fp32", sched, 8)
    s.step(8)
    np.testing.assert_array_equal(s.state()[0], ref_p)
    s2 = alelb.Solver(ms, ens["params"], precision="fp32")
    ch2 = s2.autotune(reps=3)
    assert ch2["cached"] and (ch2["waves"], ch2["rings"], ch2["node_block"], ch2["groups"]) == \
        (ch["waves"], ch["rings"], ch["node_block"], ch["groups"])
    s.close()
    s2.close()


@pytest.mark.parametrize("name", ["vortex", "pitch_blend"])
def test_fp32_correction_fields_against_oracle(alelb, oracle_mod, name):
    """W and X after one FP32 step against the FP64 oracle's, in both families.

    With an FP32 state on triangles the correction passes read FP32-rounded
    copies of the element gradient coefficients and node coordinates.  Their
    error is then that of the FP32 moments they differentiate (a relative
    1e-7, amplified where the fields vary little across an element), far below
    the order-one error of a wrong coefficient, node or slot.  The vortex
    exercises the sine-deformation metric on a periodic mesh, the pitching
    case the blend zone, where J at a node depends on its coordinates.
    Measured: vortex W 4.3e-5, X 1.3e-4; pitching W 3.6e-6, X 5.0e-6, the same
    to three digits as with the FP64 records."""
    c = {"vortex": lambda: cases.small("vortex", n=28, beta=2.0),
         "pitch_blend": lambda: cases.pitch(n_nodes=12000, first=0.5, Ma=0.3, Re=2e3, A_deg=10.0, k=2.0,
                                            h_c=0.1, phase_h=0.5, r0_c=0.5, r1_c=3.0)}[name]()
    o = oracle_mod.Oracle(c["mesh"].arrays(), c["params"])
    o.init_fields(**c["init"])
    o.step(1)
    oW, oXa = o.correction()
    for sched in (None, TILE_REF):
        s = alelb.Solver(c["mesh"].arrays(), c["params"], precision="fp32", flags=alelb.F_KEEP_MASKS)
        if sched:
            s.set_schedule(*sched)
        s.init_fields(**c["init"])
        s.step(1)
        W, Xa = s.correction()
        eW, eX = rel_fields(W, oW), rel_fields(Xa, oXa)
        print(f"{name} schedule {sched}: W {eW:.2e} X {eX:.2e}", flush=True)
        assert eW < 1e-3 and eX < 1e-3, (name, sched, eW, eX)
        s.close()
