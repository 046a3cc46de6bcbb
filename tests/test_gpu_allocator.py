"""The optional device allocator of ale_lb_params_t, through the C-ABI: a
handle whose every device allocation goes through the caller's functions
(here torch's caching allocator) computes what a default handle computes,
bit for bit, under both schedule families and through the state calls; it
returns every block it took when it is destroyed, also after a create that
fails for want of memory."""

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


class Pool:
    """Counts the blocks taken from torch's caching allocator."""

    def __init__(self, fail_after=None):
        import torch
        self.torch = torch
        self.live = {}
        self.calls = 0
        self.fail_after = fail_after

    def alloc(self, n):
        self.calls += 1
        if self.fail_after is not None and self.calls > self.fail_after:
            return 0
        p = self.torch.cuda.caching_allocator_alloc(n)
        self.live[p] = n
        return p

    def free(self, p):
        assert p in self.live, "freed a block it did not take"
        del self.live[p]
        self.torch.cuda.caching_allocator_delete(p)


@pytest.mark.parametrize("sched", [None, (4, 1, 256, 0, 3)])
def test_allocator_hook_matches_default(alelb, sched):
    c = cases.small("plunge", n_nodes=12000)
    pool = Pool()
    ref = alelb.Solver(c["mesh"].arrays(), c["params"], precision="fp32")
    s = alelb.Solver(c["mesh"].arrays(), c["params"], precision="fp32", allocator=(pool.alloc, pool.free))
    for h in (ref, s):
        if sched is not None:
            h.set_schedule(*sched)
        h.init_fields(**c["init"])
        h.step(8)
    blob = s.save_state()
    assert blob == ref.save_state()
    np.testing.assert_array_equal(s.state()[0], ref.state()[0])
    np.testing.assert_array_equal(s.fields(), ref.fields())
    print(f"schedule {sched}: {pool.calls} allocations, {len(pool.live)} live, "
          f"{sum(pool.live.values())} bytes", flush=True)
    assert pool.live and pool.calls > len(pool.live)  # the state calls' scratch copies came and went
    ref.close()
    s.close()
    assert not pool.live


def test_allocator_failure_returns_every_block(alelb):
    c = cases.small("plunge", n_nodes=12000)
    pool = Pool(fail_after=5)
    with pytest.raises(alelb.AleLbError) as e:
        alelb.Solver(c["mesh"].arrays(), c["params"], precision="fp32", allocator=(pool.alloc, pool.free))
    assert e.value.code == alelb.ENOMEM
    assert pool.calls == 6 and not pool.live
