"""The entry point that allocates nothing, through the C-ABI:
ale_lb_forces_noalloc() against ale_lb_forces_batch() on two calls in a row,
the second on a smaller batch (fewer cases, fewer wall-edge workgroups), each
in both precisions.  The two entry points run the same kernels on the same
partial-sum layout, so the sums must agree bit for bit; the scratch array
keeps the first call's partials, which the second must not see."""

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


def _raw(f):
    return np.array([f["F_p"][0], f["F_p"][1], f["F_v"][0], f["F_v"][1], f["M_p"], f["M_v"]])


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_forces_noalloc_matches_forces_batch(alelb, precision):
    import torch
    big = cases.ensemble(n_cases=3, n_min=2000, n_max=20_000, seed=7)
    small = cases.ensemble(n_cases=1, n_min=2000, n_max=2000, seed=8)
    out = torch.full((6 * 3,), float("nan"), dtype=torch.float64, device="cuda")
    blocks = []
    for ens, steps in ((big, 7), (small, 3)):
        ms = [m.arrays() for m in ens["meshes"]]
        n = len(ms)
        s = alelb.Solver(ms, ens["params"], precision=precision)
        s.init_fields(**cases.concat_init(ens["inits"]))
        s.step(steps)
        ref = np.stack([_raw(f) for f in s.forces_batch()])
        s.forces_noalloc(out.data_ptr(), n)
        torch.cuda.synchronize()
        got = out.cpu().numpy()[:6 * n].reshape(n, 6)
        blocks.append(sum(-(-len(m.wall_edges) // 256) for m in ens["meshes"]))
        print(f"{precision}: {n} cases, {blocks[-1]} wall-edge workgroups, max |diff| {np.abs(got - ref).max():.3e}",
              flush=True)
        assert np.all(np.abs(ref) > 0)
        np.testing.assert_array_equal(got, ref)
        with pytest.raises(alelb.AleLbError) as e:
            s.forces_noalloc(out.data_ptr(), n - 1)
        assert e.value.code == alelb.EINVAL
        with pytest.raises(alelb.AleLbError) as e:
            s.forces_noalloc(0, n)
        assert e.value.code == alelb.EINVAL
        s.close()
    assert blocks[1] < blocks[0]
