"""Batched layout (marked gpu): every graph of a batch comes out bit for bit
as its single-graph layout (drg_layout with the same parameters), on mixed
batches that cover one-level and multilevel graphs, edge-less graphs, graphs
with isolated nodes, different exponents, seeds and iteration counts; the
recorded run replays to the same result; bad batches are rejected."""
import numpy as np
import pytest

from paper_2008_07799_amd import gen
from tests.gpu_util import ctx, dev_graph, say

pytestmark = pytest.mark.gpu


def _edgeless(n):
    return gen.canonical_csr(n, np.zeros(0, np.int64), np.zeros(0, np.int64), f"empty{n}")


def _single(g, p):
    import torch
    from paper_2008_07799_amd import drgraph as d
    rp, col = dev_graph(g)
    y = torch.empty((g.n, 2), dtype=torch.float32, device="cuda")
    d.drg_layout(ctx(), rp, col, p, y)
    return y.cpu().numpy()


def _params(i, g, T, k):
    from paper_2008_07799_amd import drgraph as d
    b = 3 if g.name.startswith("grid") else (1 if g.name.startswith("ba") else 2)
    return d.layout_params(k=k, M=5, b=b, T=T, seed=100 + i, min_nodes=200, gamma=0.1)


def _check_batch(graphs, params):
    import torch
    from paper_2008_07799_amd import drgraph as d
    devs = [dev_graph(g) for g in graphs]
    batch = d.drg_batch_create(ctx(), devs, params)
    y = torch.empty((batch.n_total, 2), dtype=torch.float32, device="cuda")
    batch.run(ctx(), y)
    got = y.cpu().numpy()
    say("  batch", len(graphs), "graphs", batch.n_total, "nodes", batch.nnz, "entries",
        "levels", batch.levels)
    assert np.all(np.isfinite(got))
    for c, (g, p) in enumerate(zip(graphs, params)):
        want = _single(g, p)
        part = got[batch.base[c]:batch.base[c + 1]]
        same = np.array_equal(part, want)
        if not same:
            say("  graph", c, g.name, "max diff", float(np.max(np.abs(part - want))))
        assert same, f"graph {c} ({g.name}) differs from its single-graph layout"
    return batch, y


@pytest.mark.parametrize("k,blocked", [(1, False), (2, False), (3, False), (2, True), (3, True)])
def test_mixed_batch_equals_single_graph_layouts(monkeypatch, k, blocked):
    """blocked=True forces the column-blocked sweep (small blocks, so every
    graph spans several, and small work items, so that the batch sweeps runs
    of several items per workgroup) on every graph with edges, alone and in
    the batch."""
    say("batch mixed k", k, "blocked" if blocked else "")
    if blocked:
        monkeypatch.setenv("DRG_SWEEP_BLOCKED", "1")
        monkeypatch.setenv("DRG_BLOCK_BITS", "8")
        monkeypatch.setenv("DRG_BLK_CHUNK_BITS", "12")
    graphs = [
        gen.grid_deleted(700, 0.05, 0, sub=0),
        gen.ba(1500, 3, 0, sub=1),
        gen.grid(32, 32),
        _edgeless(5),
        gen.random_graph(300, 0.01, seed=4),   # isolated nodes
        gen.ba(600, 3, 0, sub=5),
        gen.grid_deleted(2500, 0.05, 0, sub=6),
        gen.rmat(11, 8, seed=3),
    ]
    Ts = [40, 60, 30, 10, 50, 0, 60, 45]
    params = [_params(i, g, T, k) for i, (g, T) in enumerate(zip(graphs, Ts))]
    batch, y = _check_batch(graphs, params)
    assert max(batch.levels) > 1 and min(batch.levels) == 1
    # a replay of the recorded run gives the same coordinates
    import torch
    y2 = torch.empty_like(y)
    batch.run(ctx(), y2)
    assert torch.equal(y, y2)


def test_sweep_forms_agree(monkeypatch):
    """Row form, windowed form (small LDS chunks) and the tuned choice give
    the same bits; the tuner reports every candidate it timed."""
    import torch
    from paper_2008_07799_amd import drgraph as d
    say("batch sweep forms")
    graphs = [gen.ba(3000, 3, 0, sub=2), gen.grid_deleted(2000, 0.05, 0, sub=3),
              gen.random_graph(400, 0.01, seed=5), gen.ba(900, 3, 0, sub=4)]
    params = [_params(i, g, 30, 3) for i, g in enumerate(graphs)]
    devs = [dev_graph(g) for g in graphs]
    outs = []
    for env in ({"DRG_BATCH_SWEEP": "row"},
                {"DRG_BATCH_SWEEP": "win", "DRG_WIN_RPL": "2", "DRG_WIN_CH": "300"},
                {"DRG_BATCH_SWEEP": "win", "DRG_WIN_RPL": "8", "DRG_WIN_CH": "8192"},
                {}):
        for k in ("DRG_BATCH_SWEEP", "DRG_WIN_RPL", "DRG_WIN_CH"):
            monkeypatch.delenv(k, raising=False)
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        b = d.drg_batch_create(ctx(), devs, params)
        y = torch.empty((b.n_total, 2), dtype=torch.float32, device="cuda")
        b.run(ctx(), y)
        outs.append(y.cpu().numpy())
        tune = b.tuning()
        say("  ", env, tune)
        if env:
            assert tune["chosen"] == -1
        else:
            assert len(tune["candidates"]) >= 2 and 0 <= tune["chosen"] < len(tune["candidates"])
            assert tune["candidates"][0][0] == 0  # the row form is always a candidate
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_single_graph_batch_and_one_shot():
    import torch
    from paper_2008_07799_amd import drgraph as d
    say("batch of one")
    g = gen.ba(3000, 3, 0, sub=9)
    p = _params(0, g, 80, 3)
    _check_batch([g], [p])
    y = torch.empty((g.n, 2), dtype=torch.float32, device="cuda")
    d.drg_layout_batched(ctx(), [dev_graph(g)], p, y)
    assert np.array_equal(y.cpu().numpy(), _single(g, p))


def test_full_size_batch_sampled_graphs():
    """512 graphs, log-uniform 500..50,000 nodes (grids minus 5% of edges and
    Barabasi-Albert m=3), k=3, 300 iterations: the smallest, the median and the
    largest graph of each kind against their single-graph layouts."""
    import torch
    from paper_2008_07799_amd import drgraph as d
    say("batch full size")
    graphs = gen.batch_graphs(512)
    params = [_params(i, g, 300, 3) for i, g in enumerate(graphs)]
    for p in params:
        p.min_nodes = 1000
    devs = [dev_graph(g) for g in graphs]
    batch = d.drg_batch_create(ctx(), devs, params)
    y = torch.empty((batch.n_total, 2), dtype=torch.float32, device="cuda")
    batch.run(ctx(), y)
    got = y.cpu().numpy()
    say("  nodes", batch.n_total, "entries", batch.nnz, "max levels", max(batch.levels))
    assert np.all(np.isfinite(got))
    sizes = np.array([g.n for g in graphs])
    picks = set()
    for parity in (0, 1):
        idx = np.arange(parity, 512, 2)
        order = idx[np.argsort(sizes[idx], kind="stable")]
        picks.update([int(order[0]), int(order[len(order) // 2]), int(order[-1])])
    for c in sorted(picks):
        want = _single(graphs[c], params[c])
        assert np.array_equal(got[batch.base[c]:batch.base[c + 1]], want), graphs[c].name


def test_bad_batches_are_rejected():
    import torch
    from paper_2008_07799_amd import drgraph as d
    say("batch errors")
    g1, g2 = gen.grid(8, 8), gen.ba(200, 3, 0, sub=1)
    devs = [dev_graph(g1), dev_graph(g2)]
    with pytest.raises(d.DrgError) as e:
        d.drg_batch_create(ctx(), devs, [d.layout_params(k=2), d.layout_params(k=3)])
    assert e.value.status == d.DRG_E_INVALID
    with pytest.raises(d.DrgError) as e:
        d.drg_batch_create(ctx(), devs, d.layout_params(mode=d.DRG_MODE_ASYNC))
    assert e.value.status == d.DRG_E_UNSUPPORTED
    rp, col = dev_graph(g2)
    bad = col.clone()
    bad[3] = g2.n + 7  # outside graph 2's own id range
    with pytest.raises(d.DrgError) as e:
        d.drg_batch_create(ctx(), [devs[0], (rp, bad)], d.layout_params(k=2))
    assert e.value.status == d.DRG_E_GRAPH
    y = torch.empty((g1.n + g2.n, 2), dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError):
        d.drg_layout_batched(ctx(), devs, d.layout_params(k=2), y[:-1])


def test_batch_matches_oracle_layouts(oracle_lib):
    """Every graph of a mixed batch against the oracle's own layout of that
    graph (drgo.layout, FP64) with the same parameters: one-level and
    multilevel graphs, exponents 1..3, different seeds and iteration counts,
    an isolated node.  Coordinates within 1e-4 normwise on the graphs whose
    trajectory is conditioned for it (grids and random geometric graphs:
    the oracle's own FP32-rounded run stays within ~1e-5); the power-law
    graph (Barabasi-Albert, b = 1), whose trajectory amplifies rounding to
    O(0.05) within 30 iterations, by final objective within 1% and NP within
    0.01."""
    import torch
    from oracle import evaluate
    from paper_2008_07799_amd import drgraph as d
    f32 = lambda v: float(np.float32(v))  # noqa: E731  (parameters cross the ABI as FP32)
    cases = [  # graph, k, b, T, eta0, min_nodes, seed, compare
        (gen.grid_deleted(700, 0.05, 0, sub=0), 3, 3, 30, 0.25, 200, 101, "coords"),
        (gen.rgg(3000, 0.04, seed=1), 3, 2, 30, 0.5, 200, 102, "coords"),
        (gen.grid(32, 32), 3, 3, 20, 0.25, 1 << 30, 103, "coords"),
        (gen.canonical_csr(40, np.arange(0, 38), np.arange(1, 39)), 2, 2, 25, 0.5, 10, 104,
         "coords"),
        (gen.ba(1500, 3, 0, sub=1), 2, 1, 150, 1.0, 200, 105, "stats"),
    ]
    devs, params = [], []
    for g, k, b, T, eta0, mn, seed, _ in cases:
        devs.append(dev_graph(g))
        params.append(d.layout_params(k=k, M=5, b=b, T=T, eta0=eta0, min_nodes=mn, seed=seed))
    ks = {c[1] for c in cases}
    batches = []
    for k in sorted(ks):  # k is one per batch (one union similarity)
        idx = [i for i, c in enumerate(cases) if c[1] == k]
        batch = d.drg_batch_create(ctx(), [devs[i] for i in idx], [params[i] for i in idx])
        y = torch.empty((batch.n_total, 2), dtype=torch.float32, device="cuda")
        batch.run(ctx(), y)
        batches.append((idx, batch, y.cpu().numpy()))
    for idx, batch, got in batches:
        for pos, i in enumerate(idx):
            g, k, b, T, eta0, mn, seed, how = cases[i]
            part = got[batch.base[pos]:batch.base[pos + 1]].astype(np.float64)
            yr, rsim, rh = oracle_lib.layout(g, k=k, M=5, b=b, T=T, eta0=f32(eta0),
                                             gamma=f32(0.1), gamma_coarsest=f32(0.01),
                                             min_nodes=mn, seed=seed, return_all=True)
            assert batch.levels[pos] == rh.levels
            if how == "coords":
                err = float(np.abs(part - yr).max() / np.abs(yr).max())
                say("  batch graph", i, g.name, "levels", rh.levels, "err", err)
                assert err < 1e-4
            else:
                o_g = evaluate.objective_eval(rsim, part, M=5, b=b, gamma=0.1)
                o_r = evaluate.objective_eval(rsim, yr, M=5, b=b, gamma=0.1)
                np_g = evaluate.neighbourhood_preservation(g, part)
                np_r = evaluate.neighbourhood_preservation(g, yr)
                say("  batch graph", i, g.name, "objective", o_g, o_r, "NP", np_g, np_r)
                assert abs(o_g - o_r) <= 0.01 * abs(o_r)
                assert abs(np_g - np_r) <= 0.01
        batch.close()
