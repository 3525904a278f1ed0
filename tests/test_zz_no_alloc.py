"""The allocation-free objective forward (drg_objective_fwd_noalloc) against
drg_objective_fwd: the same loss bit for bit, on two calls in a row with
the second on a smaller similarity (the static scratch keeps the first
call's contents), on the column-blocked path and on the row kernels, and
the size limit of the static scratch (marked gpu)."""
import numpy as np
import pytest

from paper_2008_07799_amd import gen
from tests.gpu_util import ctx, dev_graph, say

pytestmark = pytest.mark.gpu


def test_noalloc_forward_matches_allocating_forward():
    import torch
    from paper_2008_07799_amd import drgraph as d
    c = ctx()
    cases = [("rmat13 k=2 (column-blocked)", gen.rmat(13, 16, seed=1), 2, True),
             ("rmat12 k=2", gen.rmat(12, 8, seed=3), 2, False),
             ("grid32 k=3", gen.grid(32, 32), 3, False)]
    for name, g, k, blocked in cases:
        say("noalloc objective", name)
        rp, col = dev_graph(g)
        sim = d.drg_build_similarity(c, rp, col, k)
        assert sim.blocked == blocked
        y = torch.from_numpy(np.random.default_rng(g.n).uniform(-3, 3, (g.n, 2))
                             .astype(np.float32)).cuda()
        for M, b, seed, it in ((5, 1, 0, 0), (3, 2, 9, 4)):
            want = d.drg_objective_fwd(c, sim, y, M=M, b=b, gamma=0.1, seed=seed, iter=it)
            got = torch.full((), float("nan"), dtype=torch.float32, device="cuda")
            d.drg_objective_fwd_noalloc(c, sim, y, got, M=M, b=b, gamma=0.1, seed=seed, iter=it)
            c.synchronize()
            say("  ", M, b, float(want), float(got))
            assert torch.equal(got, want)
        sim.close()


def test_noalloc_forward_rejects_oversized_similarity():
    import torch
    from paper_2008_07799_amd import drgraph as d
    c = ctx()
    n = (1 << 20) + 1
    g = gen.canonical_csr(n, np.array([0]), np.array([1]))
    rp, col = dev_graph(g)
    sim = d.drg_build_similarity(c, rp, col, 1)
    y = torch.zeros((n, 2), dtype=torch.float32, device="cuda")
    loss = torch.zeros((), dtype=torch.float32, device="cuda")
    with pytest.raises(d.DrgError) as e:
        d.drg_objective_fwd_noalloc(c, sim, y, loss)
    assert e.value.status == d.DRG_E_INVALID
    sim.close()
