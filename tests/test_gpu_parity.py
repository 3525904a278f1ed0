"""GPU library vs the CPU oracle on the same seeded inputs (marked gpu).

Bars: integer and index work (BFS rows, hops, sampling weights, coarsening
maps, coarse graphs, initial coordinates) bit-exact; the FP64 similarity
values bit-exact (same operations in the same order on both sides); layout
coordinates within 1e-4 normwise relative of the FP64 oracle after 50
synchronous iterations.  The layout dynamics amplify rounding differences
(repulsion between near-coincident nodes), so the 50-iteration trajectories
are checked with the FP64 instance of the same kernels; the FP32 kernels are
checked step by step from identical states at every level (one FP32 rounding
of the step, bar 2e-6), over 50 iterations where the dynamics are tame, and
end to end by objective and neighbourhood preservation."""
import math

import numpy as np
import pytest

from paper_2008_07799_amd import gen
from tests.gpu_util import (ctx, dev_graph, hogwild_vs_oracle_spread, normwise_rel, say,
                            to_y, zeros_y)

pytestmark = pytest.mark.gpu


def _graphs_small():
    return {
        "grid32": gen.grid(32, 32),
        "er300": gen.random_graph(300, 0.02, seed=1),
        "ba2000": gen.ba(2000, 3, seed=2),
        "rmat12": gen.rmat(12, 8, seed=3),
        "rgg20k": gen.rgg(20000, 0.0125, seed=4),
        "isolated": gen.canonical_csr(50, np.array([0, 1, 2, 10, 11]), np.array([1, 2, 3, 11, 12])),
    }


def test_init_layout_bit_exact(oracle_lib):
    from paper_2008_07799_amd import drgraph as d
    c = ctx()
    for n, seed, level in [(1, 0, 0), (5000, 0, 0), (777, 3, 2), (4096, 2**40 + 5, 7)]:
        say("init", n, seed, level)
        y = zeros_y(n)
        d.drg_init_layout(c, n, seed, level, y)
        ref = oracle_lib.init(n, seed, level)
        assert np.array_equal(y.cpu().numpy().astype(np.float64), ref)


@pytest.mark.parametrize("name,k", [("grid32", 3), ("er300", 1), ("er300", 2), ("er300", 3),
                                    ("er300", 4), ("ba2000", 3), ("rmat12", 2), ("rgg20k", 3),
                                    ("isolated", 2), ("rmat12", 1)])
def test_similarity_matches_oracle(oracle_lib, name, k):
    from paper_2008_07799_amd import drgraph as d
    say("similarity", name, k)
    g = _graphs_small()[name]
    rp, col = dev_graph(g)
    sim = d.drg_build_similarity(ctx(), rp, col, k, 1.0, validate=True)
    got = sim.export()
    ref = oracle_lib.similarity(g, k, 1.0)
    assert sim.nnz == ref.nnz and sim.n_active == ref.n_active
    assert np.array_equal(got["row_ptr"], ref.row_ptr)
    assert np.array_equal(got["col"], ref.col)
    assert np.array_equal(got["hop"], ref.hop)
    assert np.array_equal(got["e"], ref.e)
    assert np.array_equal(got["invZ"], ref.invZ)
    assert np.array_equal(got["P"], ref.P)
    assert np.array_equal(got["W"], ref.W)
    assert np.allclose(got["qt"], ref.qt, rtol=1e-12, atol=0)
    sim.close()


def test_bad_input_is_rejected():
    import torch
    from paper_2008_07799_amd import drgraph as d
    c = ctx()
    say("bad inputs")
    asym_rp = torch.tensor([0, 1, 1], dtype=torch.int32, device="cuda")
    asym_col = torch.tensor([1], dtype=torch.int32, device="cuda")
    with pytest.raises(d.DrgError) as e:
        d.drg_build_similarity(c, asym_rp, asym_col, 2, validate=True)
    assert e.value.status == d.DRG_E_GRAPH
    loop_rp = torch.tensor([0, 2, 3], dtype=torch.int32, device="cuda")
    loop_col = torch.tensor([0, 1, 0], dtype=torch.int32, device="cuda")
    with pytest.raises(d.DrgError) as e:
        d.drg_build_similarity(c, loop_rp, loop_col, 2, validate=True)
    assert e.value.status == d.DRG_E_GRAPH
    oob_rp = torch.tensor([0, 1, 2], dtype=torch.int32, device="cuda")
    oob_col = torch.tensor([1, 7], dtype=torch.int32, device="cuda")
    with pytest.raises(d.DrgError) as e:
        d.drg_build_similarity(c, oob_rp, oob_col, 2)
    assert e.value.status == d.DRG_E_GRAPH
    rp, col = dev_graph(gen.grid(4, 4))
    for k in (0, 5):
        with pytest.raises(d.DrgError) as e:
            d.drg_build_similarity(c, rp, col, k)
        assert e.value.status == d.DRG_E_INVALID
    with pytest.raises(d.DrgError) as e:
        d.drg_coarsen(c, rp, col, 0, rho=1.5)
    assert e.value.status == d.DRG_E_INVALID


@pytest.mark.parametrize("name", ["grid32", "ba2000", "rmat12", "rgg20k", "isolated"])
def test_coarsening_matches_oracle(oracle_lib, name):
    from paper_2008_07799_amd import drgraph as d
    say("coarsen", name)
    g = _graphs_small()[name]
    rp, col = dev_graph(g)
    h = d.drg_coarsen(ctx(), rp, col, seed=7, rho=0.8, min_nodes=20, max_levels=64)
    ref = oracle_lib.hierarchy(g, seed=7, rho=0.8, min_nodes=20, max_levels=64)
    assert h.sizes == ref.sizes
    for l in range(1, h.levels):
        got = h.export(l, g.n)
        assert np.array_equal(got["map"], ref.maps[l - 1])
        assert np.array_equal(got["cmap"], ref.cmaps[l])
        assert np.array_equal(got["row_ptr"], ref.graphs[l].row_ptr)
        assert np.array_equal(got["col"], ref.graphs[l].col)
    h.close()


def _run_steps(oracle_lib, g, k, M, b, gamma, iters, T, seed=0, max_levels=1, min_nodes=10,
               mode=0, f64=False, eta0=1.0):
    """Both sides run the same schedule over `iters` of the T iterations,
    starting at the coarsest level and refining in between."""
    import torch
    from paper_2008_07799_amd import drgraph as d
    c = ctx()
    dt = torch.float64 if f64 else torch.float32
    rp, col = dev_graph(g)
    sim = d.drg_build_similarity(c, rp, col, k)
    h = d.drg_coarsen(c, rp, col, seed=seed, rho=0.8, min_nodes=min_nodes,
                      max_levels=max_levels)
    rsim = oracle_lib.similarity(g, k)
    rh = oracle_lib.hierarchy(g, seed, 0.8, min_nodes, max_levels)
    assert h.sizes == rh.sizes
    Lc = h.levels
    y = zeros_y(h.sizes[-1], dt)
    d.drg_init_layout(c, h.sizes[-1], seed, Lc - 1, y)
    yr = oracle_lib.init(rh.sizes[-1], seed, Lc - 1)
    done = 0
    gi = 0
    for (l, Tl, gam) in oracle_lib.schedule(T, Lc, gamma, 0.01):
        if done >= iters:
            break
        cm = None if l == 0 else rh.cmaps[l]
        gam = float(np.float32(gam))  # the step parameters cross the ABI as FP32
        for t in range(Tl):
            if done >= iters:
                break
            eta = float(np.float32(oracle_lib.eta_at(eta0, t, Tl)))
            d.drg_layout_step(c, sim, h, y, M=M, b=b, gamma=gam, eta=eta, clip=4.0, level=l,
                              mode=mode, seed=seed, iter=gi)
            oracle_lib.iter_sync(sim=rsim, y=yr, cmap=cm, M=M, b=b, gamma=gam, eta=eta,
                                 clip=4.0, seed=seed, it=gi)
            gi += 1
            done += 1
        if l > 0 and done < iters:
            yf = zeros_y(h.sizes[l - 1], dt)
            d.drg_prolong(c, h, l, y, yf)
            y = yf
            yr = yr[rh.maps[l - 1]].copy()
    return y.cpu().numpy(), yr, sim, h, rsim, rh


@pytest.mark.parametrize("name,k,b", [("grid32", 3, 3), ("er300", 2, 2), ("rmat12", 2, 1),
                                      ("rgg20k", 3, 2), ("isolated", 2, 2)])
def test_one_step_matches_oracle(oracle_lib, name, k, b):
    say("one step", name, k, b)
    g = _graphs_small()[name]
    y, yr, *_ = _run_steps(oracle_lib, g, k, 5, b, 0.1, 1, 300)
    err = normwise_rel(y, yr)
    say("  err", err)
    assert err < 2e-6


@pytest.mark.parametrize("name,k,b", [("rmat12", 2, 1), ("rgg20k", 3, 2), ("ba2000", 3, 1)])
def test_one_step_every_level_from_same_state(oracle_lib, name, k, b):
    """FP32 step at each level from one random FP32 state, in sync mode."""
    from paper_2008_07799_amd import drgraph as d
    say("one step per level", name)
    g = _graphs_small()[name]
    c = ctx()
    rp, col = dev_graph(g)
    sim = d.drg_build_similarity(c, rp, col, k)
    h = d.drg_coarsen(c, rp, col, seed=1, rho=0.8, min_nodes=20, max_levels=64)
    rsim = oracle_lib.similarity(g, k)
    rh = oracle_lib.hierarchy(g, 1, 0.8, 20, 64)
    assert h.levels >= 2
    rng = np.random.default_rng(5)
    for l in range(h.levels):
        y0 = rng.uniform(-3, 3, size=(h.sizes[l], 2)).astype(np.float32)
        y = to_y(y0)
        d.drg_layout_step(c, sim, h, y, M=7, b=b, gamma=0.1, eta=0.9, clip=4.0, level=l,
                          seed=11, iter=3 + l)
        yr = y0.astype(np.float64)
        oracle_lib.iter_sync(rsim, yr, None if l == 0 else rh.cmaps[l], 7, b, 0.1, 0.9, 4.0,
                             11, 3 + l)
        err = normwise_rel(y.cpu().numpy(), yr)
        say("  level", l, "err", err)
        assert err < 2e-6


def test_fp64_instance_one_step_is_tight(oracle_lib):
    say("fp64 one step")
    g = _graphs_small()["rmat12"]
    y, yr, *_ = _run_steps(oracle_lib, g, 2, 5, 1, 0.1, 1, 100, f64=True)
    err = normwise_rel(y, yr)
    say("  err", err)
    assert err < 1e-12


# Step size of the 32x32 grid workload (k=3, M=5, b=3, T=300, one level): the
# largest of 1, 1/2, 1/3, 1/4 at which the oracle's own 50-iteration
# trajectory moves by less than a fifth of the 1e-4 bar when its state is
# rounded to FP32 after every iteration (tests/test_oracle_forces.py measures
# this on the CPU: 0.78 at 1, 1e-5 at 1/4).
C1_ETA0 = 0.25


@pytest.mark.parametrize("case", ["grid32", "rgg_multilevel", "rmat_multilevel"])
def test_sync_50_iterations_fp64_instance(oracle_lib, case):
    """50 synchronous iterations of the schedule, FP64 instance vs oracle:
    grid32 (k=3, M=5, b=3, single level, the grid workload's step size); RGG
    (k=3, M=10, b=2, three levels, 60 iterations so two refinements happen);
    R-MAT (k=2, M=5, b=1)."""
    say("sync50 fp64", case)
    if case == "grid32":
        y, yr, *_ = _run_steps(oracle_lib, gen.grid(32, 32), 3, 5, 3, 0.1, 50, 300, f64=True,
                               eta0=C1_ETA0)
    elif case == "rgg_multilevel":
        y, yr, sim, h, *_ = _run_steps(oracle_lib, gen.rgg(20000, 0.0125, seed=4), 3, 10, 2, 0.1,
                                       60, 60, max_levels=3, f64=True)
        assert h.levels == 3
    else:
        y, yr, sim, h, *_ = _run_steps(oracle_lib, gen.rmat(12, 8, seed=3), 2, 5, 1, 0.1, 50,
                                       100, max_levels=64, min_nodes=100, f64=True)
        assert h.levels >= 2
    err = normwise_rel(y, yr)
    say("  err", err)
    assert err < 1e-4


def test_sync_50_iterations_fp32_grid32(oracle_lib):
    """The 32x32 grid workload itself (k=3, M=5, b=3, T=300, one level, seed
    0, sync) on the FP32 product path, at the same step size as the FP64
    test: within 1e-4 of the FP64 oracle after 50 iterations.  The row-form
    sweep computes every pair in FP64 from the FP32 records, so the FP32
    trajectory differs from the oracle's by the rounding of the stored
    coordinates only."""
    from paper_2008_07799_amd import drgraph as d
    say("sync50 fp32 grid32")
    y, yr, *_ = _run_steps(oracle_lib, gen.grid(32, 32), 3, 5, 3, 0.1, 50, 300, eta0=C1_ETA0)
    assert ctx().last_sweep() == d.DRG_SWEEP_ROW
    err = normwise_rel(y, yr)
    say("  err", err)
    assert err < 1e-4


def test_sync_50_iterations_fp32_coarse_levels(oracle_lib):
    """FP32 over the first 50 iterations of a three-level RGG schedule
    (coarsest level), where the averaged steps keep the dynamics tame."""
    say("sync50 fp32 rgg coarse")
    y, yr, sim, h, *_ = _run_steps(oracle_lib, gen.rgg(20000, 0.0125, seed=4), 3, 10, 2, 0.1,
                                   50, 300, max_levels=3)
    err = normwise_rel(y, yr)
    say("  err", err)
    assert err < 1e-4


def test_sync_is_deterministic():
    from paper_2008_07799_amd import drgraph as d
    say("determinism")
    c = ctx()
    g = gen.rmat(12, 8, seed=3)
    rp, col = dev_graph(g)
    p = d.layout_params(k=2, M=5, b=1, T=40, min_nodes=100, seed=3)
    y1 = zeros_y(g.n)
    y2 = zeros_y(g.n)
    d.drg_layout(c, rp, col, p, y1)
    d.drg_layout(c, rp, col, p, y2)
    assert np.array_equal(y1.cpu().numpy(), y2.cpu().numpy())


@pytest.mark.parametrize("case,mode", [("grid32", 0), ("grid32", 1), ("rmat13", 0),
                                       ("rmat13", 1)])
def test_full_layout_statistics(oracle_lib, case, mode):
    """End to end (FP32 sync, FP32 async) vs the oracle's sync layout with the
    same parameters: final sampled objective within 1% and NP within 0.01.
    grid32 is the grid workload (k=3, M=5, b=3, T=300, one level, its step
    size); its async run is the Hogwild row sweep, held to the distribution
    of the oracle's layouts over seeds.  R-MAT 2^13, edge factor
    16, k=2, M=5, b=1, T=300, coarsened until < 1000 nodes, is above the
    column-blocked threshold: its async run is the Hogwild form of the
    blocked sweep.  Across seeds the oracle's own final objective varies by
    about 0.1% and NP by about 0.0015 on that family.  The form that ran is
    checked through drg_ctx_last_sweep."""
    from oracle import evaluate
    from paper_2008_07799_amd import drgraph as d
    say("full layout stats", case, "mode", mode)
    if case == "grid32":
        g = gen.grid(32, 32)
        kw = dict(k=3, M=5, b=3, T=300, max_levels=1, eta0=C1_ETA0)
        want = d.DRG_SWEEP_ROW_ASYNC if mode else d.DRG_SWEEP_ROW
    else:
        g = gen.rmat(13, 16, seed=1)
        kw = dict(k=2, M=5, b=1, T=300, min_nodes=1000)
        want = d.DRG_SWEEP_BLOCKED_ASYNC if mode else d.DRG_SWEEP_BLOCKED
    c = ctx()
    rp, col = dev_graph(g)
    p = d.layout_params(seed=0, mode=mode, **kw)
    y = zeros_y(g.n)
    d.drg_layout(c, rp, col, p, y)
    assert c.last_sweep() == want
    yg = y.cpu().numpy().astype(np.float64)
    yr, rsim, _ = oracle_lib.layout(g, seed=0, return_all=True, **kw)
    M, b = kw["M"], kw["b"]
    obj_g = evaluate.objective_eval(rsim, yg, M=M, b=b, gamma=0.1)
    obj_r = evaluate.objective_eval(rsim, yr, M=M, b=b, gamma=0.1)
    np_g = evaluate.neighbourhood_preservation(g, yg)
    np_r = evaluate.neighbourhood_preservation(g, yr)
    say("  objective", obj_g, obj_r, "NP", np_g, np_r)
    if case == "grid32" and mode == 1:
        # a Hogwild run is one draw of a random process; on this workload the
        # oracle's own layouts vary by about 7% in objective across seeds
        def run(seed):
            yy = zeros_y(g.n)
            d.drg_layout(c, rp, col, d.layout_params(seed=seed, mode=1, **kw), yy)
            assert c.last_sweep() == want
            return yy.cpu().numpy()
        hogwild_vs_oracle_spread(oracle_lib, g, kw, run)
        return
    assert abs(obj_g - obj_r) <= 0.01 * abs(obj_r)
    assert abs(np_g - np_r) <= 0.01


def test_blocked_async_many_blocks_statistics(oracle_lib, monkeypatch):
    """The asynchronous form of the blocked sweep (rows moved stage by stage,
    Sec. 3.2.2's updates seen by the later stages) on a pattern cut into 16
    column blocks of 512 nodes, as on large graphs where a stage's work items
    span many blocks and a row's partials come from items of several
    workgroups: R-MAT 2^13, edge factor 16, k=2, M=5, b=1, T=300, coarsened
    until < 1000 nodes, 4 stages; end to end against the oracle's sync
    layout, objective within 1% and NP within 0.01 (the oracle's own final
    objective varies by about 0.1% across seeds on this graph)."""
    from oracle import evaluate
    from paper_2008_07799_amd import drgraph as d
    monkeypatch.setenv("DRG_SWEEP_BLOCKED", "1")
    monkeypatch.setenv("DRG_BLOCK_BITS", "9")
    monkeypatch.setenv("DRG_ASYNC_STAGES", "4")
    say("blocked async, 16 blocks")
    g = gen.rmat(13, 16, seed=1)
    kw = dict(k=2, M=5, b=1, T=300, min_nodes=1000)
    c = ctx()
    rp, col = dev_graph(g)
    y = zeros_y(g.n)
    d.drg_layout(c, rp, col, d.layout_params(seed=0, mode=1, **kw), y)
    assert c.last_sweep() == d.DRG_SWEEP_BLOCKED_ASYNC
    yg = y.cpu().numpy().astype(np.float64)
    assert np.isfinite(yg).all()
    yr, rsim, _ = oracle_lib.layout(g, seed=0, return_all=True, **kw)
    obj_g = evaluate.objective_eval(rsim, yg, M=5, b=1, gamma=0.1)
    obj_r = evaluate.objective_eval(rsim, yr, M=5, b=1, gamma=0.1)
    np_g = evaluate.neighbourhood_preservation(g, yg)
    np_r = evaluate.neighbourhood_preservation(g, yr)
    say("  objective", obj_g, obj_r, "NP", np_g, np_r)
    assert abs(obj_g - obj_r) <= 0.01 * abs(obj_r)
    assert abs(np_g - np_r) <= 0.01


def test_async_level_weights_follow_the_hierarchy(monkeypatch):
    """A coarse level's anchor weights (each level node's members' q~
    summed) are computed once per (hierarchy, level) and reused by later
    asynchronous steps.  Checked through a case where the asynchronous step
    has a deterministic counterpart: the blocked sweep in one stage and
    without negatives takes every attraction from the records staged at the
    step's start, as the synchronous step does, so each level node moves as
    in the synchronous step up to the order of its FP32 additions.  Two
    hierarchies of one similarity in turn, every coarse level, two
    asynchronous steps (the second on the stored weights) per level."""
    from paper_2008_07799_amd import drgraph as d
    monkeypatch.setenv("DRG_SWEEP_BLOCKED", "1")
    monkeypatch.setenv("DRG_BLOCK_BITS", "9")
    monkeypatch.setenv("DRG_ASYNC_STAGES", "1")
    say("async level weights across hierarchies")
    g = gen.rmat(12, 8, seed=3)
    c = ctx()
    rp, col = dev_graph(g)
    sim = d.drg_build_similarity(c, rp, col, 2)
    assert sim.blocked
    hs = [d.drg_coarsen(c, rp, col, seed=s, rho=0.8, min_nodes=50, max_levels=3) for s in (1, 2)]
    assert all(h.levels >= 2 for h in hs)
    rng = np.random.default_rng(8)
    kw = dict(M=0, b=1, gamma=0.1, eta=0.9, clip=4.0, seed=4, iter=1)
    for h in (hs[0], hs[1], hs[0]):
        for l in range(1, h.levels):
            y0 = rng.uniform(-3, 3, size=(h.sizes[l], 2)).astype(np.float32)
            ys = to_y(y0)
            d.drg_layout_step(c, sim, h, ys, level=l, mode=d.DRG_MODE_SYNC, **kw)
            step_s = ys.cpu().numpy().astype(np.float64) - y0
            for rep in range(2):
                ya = to_y(y0)
                d.drg_layout_step(c, sim, h, ya, level=l, mode=d.DRG_MODE_ASYNC, **kw)
                assert c.last_sweep() == d.DRG_SWEEP_BLOCKED_ASYNC
                step_a = ya.cpu().numpy().astype(np.float64) - y0
                err = normwise_rel(step_a, step_s)
                say("  level", l, "rep", rep, "step error", err)
                assert err < 1e-4


@pytest.mark.parametrize("bits,form", [(8, "flat2"), (10, "flat2"), (10, "flat4"), (12, "flat4"),
                                       (8, "rows0"), (8, "rows16"), (10, "rows32"),
                                       (10, "rows64")])
def test_blocked_sweep_every_level(oracle_lib, monkeypatch, bits, form):
    """The LDS-staged sweep over the column-blocked pattern (forced on, with
    small blocks so a small graph spans many): the flat form with 1, 2 or 4
    chunks per lane and the row form with lanes per segment chosen per item or
    forced; one FP32 step per level from the same state vs the oracle, and
    bit-identical reruns."""
    from paper_2008_07799_amd import drgraph as d
    monkeypatch.setenv("DRG_SWEEP_BLOCKED", "1")
    monkeypatch.setenv("DRG_BLOCK_BITS", str(bits))
    if form.startswith("flat"):
        monkeypatch.setenv("DRG_BLK_FLAT", form[4:])
    else:
        monkeypatch.setenv("DRG_BLK_FLAT", "0")
        monkeypatch.setenv("DRG_BLK_LANES", form[4:])
    say("blocked sweep, bits", bits, form)
    g = _graphs_small()["rmat12"]
    c = ctx()
    rp, col = dev_graph(g)
    sim = d.drg_build_similarity(c, rp, col, 2)
    h = d.drg_coarsen(c, rp, col, seed=1, rho=0.8, min_nodes=20, max_levels=64)
    rsim = oracle_lib.similarity(g, 2)
    rh = oracle_lib.hierarchy(g, 1, 0.8, 20, 64)
    rng = np.random.default_rng(6)
    for l in range(h.levels):
        y0 = rng.uniform(-3, 3, size=(h.sizes[l], 2)).astype(np.float32)
        outs = []
        for rep in range(2):
            y = to_y(y0)
            d.drg_layout_step(c, sim, h, y, M=5, b=1, gamma=0.1, eta=0.9, clip=4.0, level=l,
                              seed=2, iter=7)
            outs.append(y.cpu().numpy())
        assert np.array_equal(outs[0], outs[1])
        yr = y0.astype(np.float64)
        oracle_lib.iter_sync(rsim, yr, None if l == 0 else rh.cmaps[l], 5, 1, 0.1, 0.9, 4.0, 2, 7)
        err = normwise_rel(outs[0], yr)
        say("  level", l, "err", err)
        assert err < 2e-6


@pytest.mark.parametrize("name,k,b", [("grid32", 3, 3), ("er300", 2, 2), ("rmat12", 2, 1),
                                      ("ba2000", 3, 1), ("rgg20k", 3, 2)])
def test_windowed_sweep_is_bit_identical_to_row_sweep(monkeypatch, name, k, b):
    """The LDS-windowed sweep keeps every lane's order of terms: five sync
    steps per level (from the same start) equal the global-gather row sweep
    bit for bit, for every rows-per-group setting and a small LDS chunk."""
    from paper_2008_07799_amd import drgraph as d
    say("windowed vs row sweep", name, k)
    g = _graphs_small()[name]
    c = ctx()
    rp, col = dev_graph(g)
    sim = d.drg_build_similarity(c, rp, col, k)
    h = d.drg_coarsen(c, rp, col, seed=1, rho=0.8, min_nodes=50, max_levels=3)
    rng = np.random.default_rng(11)
    starts = [rng.uniform(-3, 3, size=(h.sizes[l], 2)).astype(np.float32) for l in range(h.levels)]

    def run():
        outs = []
        for l in range(h.levels):
            y = to_y(starts[l])
            for it in range(5):
                d.drg_layout_step(c, sim, h, y, M=5, b=b, gamma=0.1, eta=0.5, clip=4.0, level=l,
                                  seed=3, iter=it)
            outs.append(y.cpu().numpy())
        return outs

    monkeypatch.setenv("DRG_SWEEP_BLOCKED", "0")
    monkeypatch.setenv("DRG_SWEEP_WINDOW", "0")
    want = run()
    monkeypatch.setenv("DRG_SWEEP_WINDOW", "1")
    for rpl, ch in ((1, 8192), (2, 300), (4, 8192), (8, 1000)):
        monkeypatch.setenv("DRG_WIN_RPL", str(rpl))
        monkeypatch.setenv("DRG_WIN_CH", str(ch))
        got = run()
        for l in range(h.levels):
            assert np.array_equal(got[l], want[l]), (rpl, ch, l)
