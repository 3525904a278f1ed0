"""Full-size checks on the R-MAT 2^20 input of the benchmark (2^20 nodes,
16 * 2^20 generated edges), in the benchmark's launch configuration
(marked gpu).

k = 2: the similarity holds 2.4e10 entries, far beyond what the oracle can
take whole, so sampled rows (18 to 4,934 entries, the longest spread over
all 128 column blocks) are checked one by one against the oracle's
rows-only similarity (Sec. 3.2.1): pattern, hops, FP64 values, 1/Z and
sampling weights bit for bit, qt within 1e-12; then one FP32 synchronous
step without negatives from a seeded state, on those rows, within 2e-6
normwise of the FP64 oracle.  Over all rows, properties that hold at any
size: qt sums to the number of non-isolated nodes (each conditional
distribution sums to one), and the attraction forces of the step add up to
zero force and zero torque (every pair acts on both ends with opposite
sign, the clip included).

k = 1 (the paper's own neighbourhood order): the whole similarity and one
whole synchronous step with negatives against the oracle."""
import numpy as np
import pytest

from paper_2008_07799_amd import gen
from tests.gpu_util import ctx, dev_graph, normwise_rel, say, to_y

pytestmark = pytest.mark.gpu

_G = {}


def _rmat20():
    if "g" not in _G:
        say("  generating R-MAT 2^20")
        _G["g"] = gen.rmat(20, 16, seed=0)
    return _G["g"]


def _sample_rows(g, seed=20):
    """Rows of the k = 2 check: non-isolated nodes whose oracle rows are cheap
    (the 1/Z of every column costs a search from that column), plus an
    isolated node."""
    deg = np.diff(g.row_ptr).astype(np.int64)
    act = np.nonzero(deg > 0)[0]
    est2 = np.zeros(g.n, np.int64)
    est2[act] = np.add.reduceat(deg[g.col], g.row_ptr[:-1][act])
    rng = np.random.default_rng(seed)
    picks = []
    for lo, hi, m, cost in ((0, 300, 2, 4e8), (300, 3000, 2, 1.5e9)):
        cand = rng.permutation(np.nonzero((deg > 0) & (est2 > lo) & (est2 <= hi))[0])
        taken = 0
        for v in cand:
            nb = g.col[g.row_ptr[v]:g.row_ptr[v + 1]]
            two = np.unique(np.concatenate([nb] + [g.col[g.row_ptr[u]:g.row_ptr[u + 1]] for u in nb]))
            if est2[two].sum() <= cost:  # what the searches from the row's columns cost
                picks.append(int(v))
                taken += 1
                if taken == m:
                    break
    # one long row (thousands of entries over most of the 128 column blocks,
    # its heaviest block segments spanning several waves): the cheapest for
    # the oracle among 60 candidates whose rows reach 5,000..60,000 entries
    cand = rng.permutation(np.nonzero((deg > 0) & (est2 > 5000) & (est2 <= 60000))[0])[:60]
    costs = []
    for v in cand:
        nb = g.col[g.row_ptr[v]:g.row_ptr[v + 1]]
        two = np.unique(np.concatenate([nb] + [g.col[g.row_ptr[u]:g.row_ptr[u + 1]] for u in nb]))
        costs.append(est2[two].sum())
    picks.append(int(cand[int(np.argmin(costs))]))
    picks.append(int(rng.choice(np.nonzero(deg == 0)[0])))
    return np.array(picks, np.int32)


def test_rmat20_k2_sampled_rows_and_invariants(oracle_lib):
    import torch
    from paper_2008_07799_amd import drgraph as d
    g = _rmat20()
    src = _sample_rows(g)
    say("rmat20 k=2 rows", src.tolist())
    c = ctx()
    rp, col = dev_graph(g)
    sim = d.drg_build_similarity(c, rp, col, 2)
    assert sim.blocked  # the benchmark's sweep path
    got = sim.export_rows(src)
    want = oracle_lib.similarity_rows(g, 2, src)
    say("  row lengths", got["row_len"].tolist())
    assert np.array_equal(got["row_len"], np.diff(want["row_ptr"]))
    assert np.array_equal(got["col"], want["col"])
    assert np.array_equal(got["hop"], want["hop"])
    assert np.array_equal(got["P"], want["P"])
    assert np.array_equal(got["invZ"], want["invZ"])
    assert np.array_equal(got["W"], want["W"])
    np.testing.assert_allclose(got["qt"], want["qt"], rtol=1e-12, atol=0)
    # every row: qt sums to N_a
    per = sim.export(values=False, pattern=False)
    n_active = int(np.count_nonzero(np.diff(per["row_ptr"])))
    assert n_active == sim.n_active
    assert abs(per["qt"].sum() - n_active) <= 1e-9 * n_active
    # one FP32 step without negatives, from a seeded state
    y0 = np.random.default_rng(3).uniform(-3, 3, size=(g.n, 2)).astype(np.float32)
    y = to_y(y0)
    eta = 0.9
    d.drg_layout_step(c, sim, None, y, M=0, b=1, gamma=0.1, eta=eta, clip=4.0, level=0,
                      seed=7, iter=0)
    y1 = y.cpu().numpy()
    # the oracle's step of the sampled rows: a pattern over all nodes whose
    # only non-empty rows are the sampled ones
    order = np.argsort(src)
    lens = np.zeros(g.n, np.int64)
    lens[src] = np.diff(want["row_ptr"])
    prp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    pc = np.concatenate([want["col"][want["row_ptr"][r]:want["row_ptr"][r + 1]] for r in order])
    pP = np.concatenate([want["P"][want["row_ptr"][r]:want["row_ptr"][r + 1]] for r in order])
    qt = np.zeros(g.n, np.float64)
    qt[src] = want["qt"]
    rs = oracle_lib.Sim(g.n, 2, 1.0, prp, pc.astype(np.int32), np.zeros(len(pc), np.uint8),
                        np.zeros(2), np.zeros(g.n), np.zeros(g.n), pP, qt,
                        np.zeros(g.n, np.uint64), np.zeros(g.n + 1, np.uint64))
    yr = y0.astype(np.float64)
    oracle_lib.iter_sync(rs, yr, None, 0, 1, 0.1, eta, 4.0, 7, 0)
    err = normwise_rel(y1[src], yr[src])
    say("  sampled-row step err", err)
    assert err < 2e-6
    assert np.array_equal(y1[src[-1]], y0[src[-1]])  # the isolated node stays
    # neighbourhood preservation of the sampled rows at full size (k_eval = 2)
    from oracle import evaluate
    nodes = torch.from_numpy(src).cuda()
    np_gpu = d.drg_neighbourhood_preservation(c, sim, to_y(y0), nodes).cpu().numpy()
    np_ref = evaluate.np_per_node(y0.astype(np.float64), prp, pc, src)
    say("  NP of the sampled rows", np_gpu.tolist())
    assert np.array_equal(np_gpu, np_ref)
    # all rows: zero net attraction force and torque
    qf = per["qt"].astype(np.float32).astype(np.float64)
    gvec = (y1.astype(np.float64) - y0.astype(np.float64)) * qf[:, None] / np.float64(np.float32(eta))
    scale = np.abs(gvec).sum()
    net = np.abs(gvec.sum(axis=0)).max()
    yy = y0.astype(np.float64)
    torque = abs((yy[:, 0] * gvec[:, 1] - yy[:, 1] * gvec[:, 0]).sum())
    say("  net force", net, "torque", torque, "scale", scale)
    assert net <= 1e-6 * scale
    assert torque <= 1e-6 * scale * np.abs(yy).max()
    del torch


def test_rmat20_k1_whole_similarity_and_step(oracle_lib):
    from paper_2008_07799_amd import drgraph as d
    g = _rmat20()
    say("rmat20 k=1")
    c = ctx()
    rp, col = dev_graph(g)
    sim = d.drg_build_similarity(c, rp, col, 1)
    rsim = oracle_lib.similarity(g, 1)
    ex = sim.export()
    assert np.array_equal(ex["row_ptr"], rsim.row_ptr)
    assert np.array_equal(ex["col"], rsim.col)
    assert np.array_equal(ex["hop"], rsim.hop)
    assert np.array_equal(ex["P"], rsim.P)
    assert np.array_equal(ex["invZ"], rsim.invZ)
    assert np.array_equal(ex["W"], rsim.W)
    np.testing.assert_allclose(ex["qt"], rsim.qt, rtol=1e-12, atol=0)
    y0 = np.random.default_rng(4).uniform(-3, 3, size=(g.n, 2)).astype(np.float32)
    y = to_y(y0)
    d.drg_layout_step(c, sim, None, y, M=5, b=1, gamma=0.1, eta=0.9, clip=4.0, level=0,
                      seed=9, iter=2)
    yr = y0.astype(np.float64)
    oracle_lib.iter_sync(rsim, yr, None, 5, 1, 0.1, 0.9, 4.0, 9, 2)
    err = normwise_rel(y.cpu().numpy(), yr)
    say("  whole step err", err)
    assert err < 2e-6
    # neighbourhood preservation (k_eval = 1 here: the rows of this
    # similarity) of 64 nodes at full size
    import torch
    from oracle import evaluate
    nodes = np.random.default_rng(5).choice(g.n, size=64, replace=False).astype(np.int32)
    y1 = y.cpu().numpy()
    np_gpu = d.drg_neighbourhood_preservation(c, sim, y, torch.from_numpy(nodes).cuda())
    np_ref = evaluate.np_per_node(y1.astype(np.float64), rsim.row_ptr, rsim.col, nodes)
    assert np.array_equal(np_gpu.cpu().numpy(), np_ref)


def test_rmat16_k2_whole_step_default_blocks(oracle_lib):
    """R-MAT 2^16 (edge factor 16), k = 2: 3.6e8 pattern entries, rows up to
    45k entries, so at the default 8192-column blocks every long row spans
    eight blocks and, inside a block, several windows and waves of the flat
    sweep.  One whole synchronous FP32 step with negatives from a seeded state
    on the column-blocked path vs the FP64 oracle over all rows, and the same
    at the coarse level of a two-level hierarchy."""
    from paper_2008_07799_amd import drgraph as d
    say("rmat16 k=2 whole step")
    g = gen.rmat(16, 16, seed=2)
    c = ctx()
    rp, col = dev_graph(g)
    sim = d.drg_build_similarity(c, rp, col, 2)
    assert sim.blocked
    rsim = oracle_lib.similarity(g, 2)
    assert sim.nnz == rsim.nnz
    say("  nnz", sim.nnz, "longest row", int(np.diff(rsim.row_ptr).max()))
    y0 = np.random.default_rng(6).uniform(-3, 3, size=(g.n, 2)).astype(np.float32)
    y = to_y(y0)
    d.drg_layout_step(c, sim, None, y, M=5, b=1, gamma=0.1, eta=0.9, clip=4.0, level=0,
                      seed=4, iter=11)
    assert c.last_sweep() == d.DRG_SWEEP_BLOCKED
    yr = y0.astype(np.float64)
    oracle_lib.iter_sync(rsim, yr, None, 5, 1, float(np.float32(0.1)), float(np.float32(0.9)),
                         4.0, 4, 11)
    err = normwise_rel(y.cpu().numpy(), yr)
    say("  level 0 err", err)
    assert err < 2e-6
    h = d.drg_coarsen(c, rp, col, seed=0, rho=0.8, min_nodes=1000, max_levels=2)
    rh = oracle_lib.hierarchy(g, 0, 0.8, 1000, 2)
    assert h.sizes == rh.sizes and h.levels == 2
    y1 = np.random.default_rng(7).uniform(-3, 3, size=(h.sizes[1], 2)).astype(np.float32)
    y = to_y(y1)
    d.drg_layout_step(c, sim, h, y, M=5, b=1, gamma=0.1, eta=0.9, clip=4.0, level=1,
                      seed=4, iter=12)
    yr = y1.astype(np.float64)
    oracle_lib.iter_sync(rsim, yr, rh.cmaps[1], 5, 1, float(np.float32(0.1)),
                         float(np.float32(0.9)), 4.0, 4, 12)
    err = normwise_rel(y.cpu().numpy(), yr)
    say("  level 1 err", err)
    assert err < 2e-6
