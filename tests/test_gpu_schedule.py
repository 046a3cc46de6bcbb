"""Launch schedules on the GPU, through the C-ABI.

Every schedule (one-wave streaming kernel with 1, 4 or 8 node groups,
direction-major streaming, or patch tiles of 28, 56 or 112 nodes with patch
radius 1 or 2, node-kernel block 64/128/256) computes
the same values in the same order, so the states must be bit-identical to
the default schedule's, also when an LDS cap sends some or all tiles to the
global path.  The autotuner must pick one of them and reuse its choice for a
second handle in the same mesh-size bucket.
"""

import numpy as np
import pytest

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


SCHEDULES = [  # (waves, rings, node_block, lds_limit[, groups])
    (0, 0, 128, 0, 4), (0, 0, 64, 0, 8),  # one wave, 4 or 8 node groups sharing the metric phase
    (9, 0, 256, 0), (9, 0, 64, 0),  # direction-major streaming
    (4, 1, 64, 0), (4, 2, 256, 0), (8, 1, 128, 0), (8, 2, 256, 0), (16, 1, 256, 0), (16, 2, 64, 0),
    (8, 1, 256, 2048),    # no room for any patch: every tile on the global path
    (16, 1, 256, 20000),  # caps below the largest patches: some tiles on the global path
]


def _run(alelb, meshes, params, init, precision, sched, steps):
    s = alelb.Solver(meshes, params, precision=precision)
    if sched is not None:
        s.set_schedule(*sched)
    s.init_fields(**init)
    s.step(steps)
    pops, mac, t, n = s.state()
    info = s.info()
    s.close()
    return pops, mac, info


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_every_schedule_is_bit_identical(alelb, ens, precision):
    ms = [m.arrays() for m in ens["meshes"]]
    init = cases.concat_init(ens["inits"])
    ref_p, ref_m, _ = _run(alelb, ms, ens["params"], init, precision, None, 12)
    for sched in SCHEDULES:
        p, m, info = _run(alelb, ms, ens["params"], init, precision, sched, 12)
        print(f"{precision} schedule {sched}: global-path tiles {info['global_tiles']}", flush=True)
        np.testing.assert_array_equal(p, ref_p, err_msg=str(sched))
        np.testing.assert_array_equal(m, ref_m, err_msg=str(sched))
        if sched[3] == 2048:
            assert info["global_tiles"] > 0


def test_schedules_on_a_periodic_mesh(alelb):
    c = cases.small("vortex", n=28, beta=2.0)
    ref_p, ref_m, _ = _run(alelb, c["mesh"].arrays(), c["params"], c["init"], "fp64", None, 10)
    for sched in ((0, 0, 256, 0, 8), (9, 0, 128, 0), (4, 1, 64, 0), (16, 2, 128, 0), (8, 1, 256, 6000)):
        p, m, info = _run(alelb, c["mesh"].arrays(), c["params"], c["init"], "fp64", sched, 10)
        print(f"vortex schedule {sched}: global-path tiles {info['global_tiles']}", flush=True)
        np.testing.assert_array_equal(p, ref_p, err_msg=str(sched))
        np.testing.assert_array_equal(m, ref_m, err_msg=str(sched))


def test_autotune_choice_and_cache(alelb, ens):
    ms = [m.arrays() for m in ens["meshes"]]
    init = cases.concat_init(ens["inits"])
    ref_p, _, _ = _run(alelb, ms, ens["params"], init, "fp32", None, 8)
    s = alelb.Solver(ms, ens["params"], precision="fp32")
    s.init_fields(**init)
    s.autotune(reps=0)  # drop any cached choice of this bucket
    ch = s.autotune(reps=3)
    print(f"autotune: {ch}", flush=True)
    assert ch["waves"] in (0, 9, 4, 8, 16) and ch["node_block"] in (64, 128, 256) and not ch["cached"]
    assert ch["groups"] in (1, 4, 8) and (ch["groups"] == 1 or ch["waves"] == 0)
    assert ch["ms"] > 0
    s.step(8)
    np.testing.assert_array_equal(s.state()[0], ref_p)
    s2 = alelb.Solver(ms, ens["params"], precision="fp32")
    ch2 = s2.autotune(reps=3)
    assert ch2["cached"] and (ch2["waves"], ch2["rings"], ch2["node_block"], ch2["groups"]) == \
        (ch["waves"], ch["rings"], ch["node_block"], ch["groups"])
    s.close()
    s2.close()
