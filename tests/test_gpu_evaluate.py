"""GPU neighbourhood preservation (Sec. 4.1, Eq. NP) against the oracle's
brute force, node by node (marked gpu): bit-exact, since both sides select
the nearest nodes by the same FP64 squared distances (ties by id) and count
the same sets.  Random layouts, layouts with many exact distance ties, and
a real layout; graph neighbourhoods are the similarity rows at k = k_eval."""
import numpy as np
import pytest

from paper_2008_07799_amd import gen
from tests.gpu_util import ctx, dev_graph, say, to_y

pytestmark = pytest.mark.gpu


def _np_gpu(c, sim, y, nodes):
    import torch
    from paper_2008_07799_amd import drgraph as d
    yt = to_y(y)
    nt = torch.from_numpy(np.ascontiguousarray(nodes, np.int32)).cuda()
    return d.drg_neighbourhood_preservation(c, sim, yt, nt).cpu().numpy()


@pytest.mark.parametrize("name,k", [("grid32", 2), ("er300", 2), ("rmat12", 2), ("ba2000", 3),
                                    ("isolated", 2)])
def test_np_matches_oracle(oracle_lib, name, k):
    from oracle import evaluate
    from paper_2008_07799_amd import drgraph as d
    graphs = {
        "grid32": gen.grid(32, 32),
        "er300": gen.random_graph(300, 0.02, seed=1),
        "rmat12": gen.rmat(12, 8, seed=3),
        "ba2000": gen.ba(2000, 3, seed=2),
        "isolated": gen.canonical_csr(50, np.array([0, 1, 2, 10, 11]), np.array([1, 2, 3, 11, 12])),
    }
    g = graphs[name]
    say("np", name, k)
    c = ctx()
    rp, col = dev_graph(g)
    sim = d.drg_build_similarity(c, rp, col, k)
    prp, pcol, _ = oracle_lib.khop(g, k)
    nodes = np.arange(g.n, dtype=np.int32)
    rng = np.random.default_rng(7)
    layouts = {
        "random": rng.uniform(-3, 3, size=(g.n, 2)).astype(np.float32),
        # coarse lattice: many coincident points and equal distances
        "ties": np.round(rng.uniform(-3, 3, size=(g.n, 2)) * 2).astype(np.float32) / 2,
    }
    yl = np.empty((g.n, 2), np.float32)
    import torch
    yt = torch.empty((g.n, 2), dtype=torch.float32, device="cuda")
    d.drg_layout(c, rp, col, d.layout_params(k=k, M=5, b=1, T=60, min_nodes=50, seed=3), yt)
    yl[:] = yt.cpu().numpy()
    layouts["layout"] = yl
    for tag, y in layouts.items():
        got = _np_gpu(c, sim, y, nodes)
        want = evaluate.np_per_node(y.astype(np.float64), prp, pcol, nodes)
        act = want >= 0
        say("  ", tag, "NP", float(want[act].mean()) if act.any() else None)
        assert np.array_equal(got, want), tag


def test_np_bad_nodes_rejected():
    import torch
    from paper_2008_07799_amd import drgraph as d
    g = gen.grid(8, 8)
    c = ctx()
    rp, col = dev_graph(g)
    sim = d.drg_build_similarity(c, rp, col, 2)
    y = torch.zeros((g.n, 2), dtype=torch.float32, device="cuda")
    bad = torch.tensor([0, g.n], dtype=torch.int32, device="cuda")
    with pytest.raises(d.DrgError) as e:
        d.drg_neighbourhood_preservation(c, sim, y, bad)
    assert e.value.status == d.DRG_E_INVALID


@pytest.mark.parametrize("name", ["grid32", "er300", "rmat12", "isolated"])
def test_stress_sums_match_oracle(oracle_lib, name):
    """Per-source stress sums (A, B, P) of the GPU search against the
    oracle's shortest paths: P exact, A and B within 1e-12."""
    import torch
    from oracle import evaluate
    from paper_2008_07799_amd import drgraph as d
    graphs = {
        "grid32": gen.grid(32, 32),
        "er300": gen.random_graph(300, 0.02, seed=1),   # several components
        "rmat12": gen.rmat(12, 8, seed=3),
        "isolated": gen.canonical_csr(50, np.array([0, 1, 2, 10, 11]), np.array([1, 2, 3, 11, 12])),
    }
    g = graphs[name]
    say("stress", name)
    c = ctx()
    rp, col = dev_graph(g)
    y = np.random.default_rng(9).uniform(-2, 2, size=(g.n, 2)).astype(np.float32)
    src = np.random.default_rng(1).choice(g.n, size=min(g.n, 40), replace=False).astype(np.int32)
    got, est = d.drg_stress_sampled(c, rp, col, to_y(y), torch.from_numpy(src).cuda())
    got = got.cpu().numpy()
    want = evaluate.stress_terms(g, y.astype(np.float64), src)
    assert np.array_equal(got[:, 2], want[:, 2])
    np.testing.assert_allclose(got[:, :2], want[:, :2], rtol=1e-12, atol=0)
    ref = evaluate.stress(g, y.astype(np.float64), src)
    say("  sampled stress", est, ref)
    assert abs(est - ref) <= 1e-10 * max(1e-30, abs(ref))
