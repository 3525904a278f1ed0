"""Weighted graphs (future work in Sec. 6; Eq. NS with the graph distance
GD the shortest path of at most k edges under positive symmetric lengths)
against the oracle (marked gpu).

Bars: the distances, E, Z and the sampling table use IEEE operations in the
same order on both sides, so 1/Z, P~ (FP64) and W are bit-exact; qt within
1e-12 (summation order); steps, objective and end to end as for unweighted
graphs."""
import numpy as np
import pytest

from paper_2008_07799_amd import gen
from tests.gpu_util import ctx, dev_graph, normwise_rel, say, to_y, zeros_y

pytestmark = pytest.mark.gpu

CASES = {
    "rmat12_k2": (lambda: gen.rmat(12, 8, seed=3), 2),
    "rgg20k_k3": (lambda: gen.rgg(20000, 0.0125, seed=4), 3),
    "grid32_k3": (lambda: gen.grid(32, 32), 3),
    "ba2000_k2": (lambda: gen.ba(2000, 3, seed=2), 2),
    "er300_k1": (lambda: gen.random_graph(300, 0.02, seed=1), 1),
    "rmat12_k4": (lambda: gen.rmat(12, 4, seed=5), 4),
    "rmat13_k2": (lambda: gen.rmat(13, 16, seed=1), 2),
    "isolated_k2": (lambda: gen.canonical_csr(50, np.array([0, 1, 2, 10, 11]),
                                              np.array([1, 2, 3, 11, 12])), 2),
}


def _both(name, sigma=1.0, seed=0):
    import torch
    from paper_2008_07799_amd import drgraph as d
    maker, k = CASES[name]
    g = maker()
    ln = gen.edge_lengths(g, seed)
    rp, col = dev_graph(g)
    sim = d.drg_build_similarity_weighted(ctx(), rp, col, torch.from_numpy(ln).cuda(), k, sigma)
    return g, k, ln, sim


@pytest.mark.parametrize("name", list(CASES))
def test_similarity_bit_exact(oracle_lib, name):
    say("weighted similarity", name)
    g, k, ln, sim = _both(name, sigma=1.5)
    assert not sim.blocked
    ref = oracle_lib.similarity_weighted(g, ln, k, 1.5)
    got = sim.export()
    assert np.array_equal(got["row_ptr"], ref.row_ptr)
    assert np.array_equal(got["col"][:ref.nnz], ref.col)
    assert np.array_equal(got["hop"][:ref.nnz], ref.hop)
    assert np.array_equal(got["P"][:ref.nnz], ref.P)
    assert np.array_equal(got["invZ"], ref.invZ)
    assert np.array_equal(got["W"], ref.W)
    assert np.allclose(got["qt"], ref.qt, rtol=1e-12, atol=0)
    say("  nnz", ref.nnz)


def test_unit_lengths_and_bad_lengths():
    import torch
    from paper_2008_07799_amd import drgraph as d
    say("weighted: unit lengths, rejects")
    g = gen.rmat(12, 8, seed=3)
    rp, col = dev_graph(g)
    c = ctx()
    ones = torch.ones(g.nnz, dtype=torch.float64, device="cuda")
    w = d.drg_build_similarity_weighted(c, rp, col, ones, 2, 1.0).export()
    u = d.drg_build_similarity(c, rp, col, 2, 1.0).export()
    # Z is summed entry by entry here and by hop histogram there: P~ agrees
    # to rounding, so each quantised entry of W may differ by one
    assert np.array_equal(w["col"], u["col"]) and np.array_equal(w["hop"], u["hop"])
    assert np.allclose(w["P"], u["P"], rtol=1e-12, atol=0)
    dW = np.abs(w["W"].astype(np.int64) - u["W"].astype(np.int64))
    assert np.all(dW <= np.diff(u["row_ptr"]))
    ln = gen.edge_lengths(g, 0)
    for bad in ("zero", "negative", "nan", "inf", "asymmetric"):
        b = ln.copy()
        if bad == "zero":
            b[5] = 0.0
        elif bad == "negative":
            b[5] = -1.0
        elif bad == "nan":
            b[5] = np.nan
        elif bad == "inf":
            b[5] = np.inf
        else:
            b[5] *= 1.5
        with pytest.raises(d.DrgError):
            d.drg_build_similarity_weighted(c, rp, col, torch.from_numpy(b).cuda(), 2)


@pytest.mark.parametrize("name", ["rmat12_k2", "rgg20k_k3", "rmat13_k2"])
def test_one_step_every_level(oracle_lib, name):
    from paper_2008_07799_amd import drgraph as d
    say("weighted step", name)
    g, k, ln, sim = _both(name)
    c = ctx()
    rp, col = dev_graph(g)
    h = d.drg_coarsen(c, rp, col, seed=1, rho=0.8, min_nodes=20, max_levels=3)
    rsim = oracle_lib.similarity_weighted(g, ln, k)
    rh = oracle_lib.hierarchy(g, 1, 0.8, 20, 3)
    rng = np.random.default_rng(9)
    gam, eta = float(np.float32(0.1)), float(np.float32(0.9))
    for l in range(h.levels):
        for dim in (2, 3):
            for b in (1, 2.5):
                y0 = rng.uniform(-3, 3, size=(h.sizes[l], dim)).astype(np.float32)
                yr = y0.astype(np.float64)
                oracle_lib.iter_sync(rsim, yr, None if l == 0 else rh.cmaps[l], 7, b, gam, eta,
                                     4.0, 11, 3 + l)
                y = to_y(y0)
                d.drg_layout_step(c, sim, h, y, M=7, b=b, gamma=0.1, eta=0.9, clip=4.0,
                                  level=l, seed=11, iter=3 + l)
                assert c.last_sweep() == d.DRG_SWEEP_ROW
                err = normwise_rel(y.cpu().numpy(), yr)
                y64 = to_y(y0, np.float64)
                d.drg_layout_step(c, sim, h, y64, M=7, b=b, gamma=0.1, eta=0.9, clip=4.0,
                                  level=l, seed=11, iter=3 + l)
                err64 = normwise_rel(y64.cpu().numpy(), yr)
                say("  level", l, "dim", dim, "b", b, "err", err, "fp64", err64)
                assert err < 2e-6
                assert err64 < 1e-12


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("f64", [True, False])
def test_objective_and_gradient(oracle_lib, dim, f64):
    from paper_2008_07799_amd import drgraph as d
    say("weighted objective", dim, "f64" if f64 else "f32")
    g, k, ln, sim = _both("rmat13_k2")
    rsim = oracle_lib.similarity_weighted(g, ln, k)
    y0 = np.random.default_rng(3).uniform(-3, 3, size=(g.n, dim))
    if not f64:
        y0 = y0.astype(np.float32).astype(np.float64)
    y = to_y(y0, np.float64 if f64 else np.float32)
    kw = dict(M=5, b=2, gamma=0.1, seed=4, iter=2)
    loss = float(d.drg_objective_fwd(ctx(), sim, y, **kw).cpu())
    grad = d.drg_objective_bwd(ctx(), sim, y, **kw).cpu().numpy().astype(np.float64)
    rloss = oracle_lib.objective(rsim, y0, 5, 2, 0.1, 4, 2)
    rgrad = oracle_lib.objective_grad(rsim, y0, 5, 2, 0.1, 4, 2)
    el = abs(loss - rloss) / abs(rloss)
    eg = normwise_rel(grad, rgrad)
    say("  loss err", el, "grad err", eg)
    assert el < (1e-12 if f64 else 1e-5)
    assert eg < (1e-10 if f64 else 1e-5)
    rows, cols, P = d.drg_sim_coo(ctx(), sim)
    assert np.allclose(P.cpu().numpy().astype(np.float64), rsim.P, rtol=1e-6, atol=1e-37)


@pytest.mark.parametrize("mode", [0, 1])
def test_full_layout_statistics(oracle_lib, mode):
    """R-MAT 2^13, edge factor 16, lengths uniform in [0.2, 3), k=2, M=5,
    b=1, T=300, coarsened until < 1000 nodes: the library's schedule over
    the weighted similarity (sync; async = the Hogwild row form) against the
    oracle's sync layout."""
    from oracle import evaluate
    from paper_2008_07799_amd import drgraph as d
    say("weighted layout mode", mode)
    g, k, ln, sim = _both("rmat13_k2")
    c = ctx()
    rp, col = dev_graph(g)
    h = d.drg_coarsen(c, rp, col, seed=0, rho=0.8, min_nodes=1000, max_levels=64)
    p = d.layout_params(k=2, M=5, b=1, T=300, min_nodes=1000, seed=0, mode=mode)
    y = zeros_y(g.n)
    d.drg_layout_run(c, sim, h, p, y)
    assert c.last_sweep() == (d.DRG_SWEEP_ROW_ASYNC if mode else d.DRG_SWEEP_ROW)
    yg = y.cpu().numpy().astype(np.float64)
    yr, rsim, _ = oracle_lib.layout(g, k=2, M=5, b=1, T=300, min_nodes=1000, seed=0,
                                    lengths=ln, return_all=True)
    obj_g = evaluate.objective_eval(rsim, yg, M=5, b=1, gamma=0.1)
    obj_r = evaluate.objective_eval(rsim, yr, M=5, b=1, gamma=0.1)
    np_g = evaluate.neighbourhood_preservation(g, yg)
    np_r = evaluate.neighbourhood_preservation(g, yr)
    say("  objective", obj_g, obj_r, "NP", np_g, np_r)
    assert abs(obj_g - obj_r) <= 0.01 * abs(obj_r)
    assert abs(np_g - np_r) <= 0.01
