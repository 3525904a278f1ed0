"""Layouts in R^3 (Sec. 3.1: positions in R^2 or R^3) on the GPU against
the oracle's 3-D functions (marked gpu): the initial layout bit for bit;
one FP32 step per level from the same state within 2e-6 (also on a graph
whose 2-D steps use the column-blocked copy: 3-D runs the row sweep); the
FP64 instance within 1e-12 for one step and 1e-4 after 50 iterations; the
objective and its gradient (FP64 1e-12 / 1e-10, FP32 1e-5); a whole
schedule equal to the host-driven one bit for bit; end to end, sync and
async, by objective and NP against the oracle's 3-D layout."""
import numpy as np
import pytest

from paper_2008_07799_amd import gen
from tests.gpu_util import ctx, dev_graph, hogwild_vs_oracle_spread, normwise_rel, say, to_y

pytestmark = pytest.mark.gpu


def _z(n, dtype=None):
    import torch
    return torch.zeros((n, 3), dtype=dtype or torch.float32, device="cuda")


def test_init_3d_bit_exact(oracle_lib):
    import torch
    from paper_2008_07799_amd import drgraph as d
    c = ctx()
    for n, seed, level in [(1, 0, 0), (5000, 0, 0), (777, 3, 2)]:
        for dt in (torch.float32, torch.float64):
            y = _z(n, dt)
            d.drg_init_layout(c, n, seed, level, y)
            assert np.array_equal(y.cpu().numpy().astype(np.float64),
                                  oracle_lib.init(n, seed, level, dim=3))


@pytest.mark.parametrize("name,k,b", [("grid16", 3, 3), ("er300", 2, 2), ("rmat12", 2, 1),
                                      ("rgg8k", 3, 2), ("rmat13_blocked", 2, 1)])
def test_one_3d_step_every_level(oracle_lib, name, k, b):
    from paper_2008_07799_amd import drgraph as d
    g = {"grid16": gen.grid(16, 16), "er300": gen.random_graph(300, 0.02, seed=1),
         "rmat12": gen.rmat(12, 8, seed=3), "rgg8k": gen.rgg(8000, 0.02, seed=4),
         "rmat13_blocked": gen.rmat(13, 16, seed=1)}[name]
    say("3-D step", name)
    c = ctx()
    rp, col = dev_graph(g)
    sim = d.drg_build_similarity(c, rp, col, k)
    assert sim.blocked == (name == "rmat13_blocked")
    h = d.drg_coarsen(c, rp, col, seed=1, rho=0.8, min_nodes=20, max_levels=3)
    rsim = oracle_lib.similarity(g, k)
    rh = oracle_lib.hierarchy(g, 1, 0.8, 20, 3)
    rng = np.random.default_rng(5)
    for l in range(h.levels):
        y0 = rng.uniform(-3, 3, size=(h.sizes[l], 3)).astype(np.float32)
        y = to_y(y0)
        d.drg_layout_step(c, sim, h, y, M=7, b=b, gamma=0.1, eta=0.9, clip=4.0, level=l,
                          seed=11, iter=3 + l)
        assert c.last_sweep() == d.DRG_SWEEP_ROW
        yr = y0.astype(np.float64)
        oracle_lib.iter_sync(rsim, yr, None if l == 0 else rh.cmaps[l], 7, b,
                             float(np.float32(0.1)), float(np.float32(0.9)), 4.0, 11, 3 + l)
        err = normwise_rel(y.cpu().numpy(), yr)
        say("  level", l, "err", err)
        assert err < 2e-6
        y64 = to_y(y0, np.float64)
        d.drg_layout_step(c, sim, h, y64, M=7, b=b, gamma=0.1, eta=0.9, clip=4.0, level=l,
                          seed=11, iter=3 + l)
        assert normwise_rel(y64.cpu().numpy(), yr) < 1e-12


def test_3d_fp64_50_iterations(oracle_lib):
    """Three-level RGG (k=3, M=10, b=2): the FP64 instance's schedule in
    R^3 within 1e-4 of the oracle after 50 iterations (two refinements)."""
    import torch
    from paper_2008_07799_amd import drgraph as d
    g = gen.rgg(8000, 0.02, seed=4)
    c = ctx()
    rp, col = dev_graph(g)
    sim = d.drg_build_similarity(c, rp, col, 3)
    h = d.drg_coarsen(c, rp, col, seed=0, rho=0.8, min_nodes=10, max_levels=3)
    rsim = oracle_lib.similarity(g, 3)
    rh = oracle_lib.hierarchy(g, 0, 0.8, 10, 3)
    assert h.levels == 3
    y = _z(h.sizes[-1], torch.float64)
    d.drg_init_layout(c, h.sizes[-1], 0, 2, y)
    yr = oracle_lib.init(rh.sizes[-1], 0, 2, dim=3)
    gi = 0
    for (l, Tl, gam) in oracle_lib.schedule(50, 3, 0.1, 0.01):
        gam = float(np.float32(gam))
        for t in range(Tl):
            eta = float(np.float32(oracle_lib.eta_at(1.0, t, Tl)))
            d.drg_layout_step(c, sim, h, y, M=10, b=2, gamma=gam, eta=eta, clip=4.0, level=l,
                              seed=0, iter=gi)
            oracle_lib.iter_sync(rsim, yr, None if l == 0 else rh.cmaps[l], 10, 2, gam, eta, 4.0,
                                 0, gi)
            gi += 1
        if l > 0:
            yf = _z(h.sizes[l - 1], torch.float64)
            d.drg_prolong(c, h, l, y, yf)
            y = yf
            yr = yr[rh.maps[l - 1]].copy()
    err = normwise_rel(y.cpu().numpy(), yr)
    say("  3-D FP64 50 iterations err", err)
    assert err < 1e-4


@pytest.mark.parametrize("name", ["er300", "rmat13_blocked"])
def test_3d_objective_and_gradient(oracle_lib, name):
    import torch
    from paper_2008_07799_amd import drgraph as d
    g = gen.random_graph(300, 0.02, seed=1) if name == "er300" else gen.rmat(13, 16, seed=1)
    c = ctx()
    rp, col = dev_graph(g)
    sim = d.drg_build_similarity(c, rp, col, 2)
    rsim = oracle_lib.similarity(g, 2)
    y0 = np.random.default_rng(9).uniform(-2, 2, size=(g.n, 3))
    for b in (1, 3):
        want = oracle_lib.objective(rsim, y0, 5, b, 0.1, 4, 2)
        gwant = oracle_lib.objective_grad(rsim, y0, 5, b, 0.1, 4, 2)
        y64 = to_y(y0, np.float64)
        got = float(d.drg_objective_fwd(c, sim, y64, M=5, b=b, gamma=0.1, seed=4, iter=2))
        assert abs(got - want) <= 1e-12 * abs(want)
        g64 = d.drg_objective_bwd(c, sim, y64, M=5, b=b, gamma=0.1, seed=4, iter=2)
        assert normwise_rel(g64.cpu().numpy(), gwant) < 1e-10
        y32 = to_y(y0)
        got32 = float(d.drg_objective_fwd(c, sim, y32, M=5, b=b, gamma=0.1, seed=4, iter=2))
        g32 = d.drg_objective_bwd(c, sim, y32, M=5, b=b, gamma=0.1, seed=4, iter=2)
        want32 = oracle_lib.objective(rsim, y0.astype(np.float32).astype(np.float64), 5, b, 0.1,
                                      4, 2)
        say("  3-D objective", name, b, got, want, got32)
        assert abs(got32 - want32) <= 1e-5 * abs(want32)
        assert normwise_rel(g32.cpu().numpy(), gwant) < 1e-5
    # through the autograd form, with a term on the third coordinate
    y = to_y(y0).requires_grad_()
    loss = -d.objective(y, c, sim, M=5, b=1, gamma=0.1, seed=4, iter=2) + (y[:, 2] ** 2).sum()
    loss.backward()
    gref = -oracle_lib.objective_grad(rsim, y0, 5, 1, 0.1, 4, 2)
    gref[:, 2] += 2 * y0[:, 2]
    assert normwise_rel(y.grad.cpu().numpy(), gref) < 1e-5
    del torch


@pytest.mark.parametrize("name", ["grid16", "rgg8k"])
def test_3d_schedule_equals_step_by_step(name):
    from paper_2008_07799_amd import drgraph as d
    g = gen.grid(16, 16) if name == "grid16" else gen.rgg(8000, 0.02, seed=4)
    c = ctx()
    rp, col = dev_graph(g)
    sim = d.drg_build_similarity(c, rp, col, 2)
    h = d.drg_coarsen(c, rp, col, seed=2, rho=0.8, min_nodes=50, max_levels=3)
    T = 30
    p = d.layout_params(k=2, M=5, b=2, T=T, min_nodes=50, max_levels=3, seed=2, eta0=0.5, dim=3)
    want = _z(g.n)
    d.drg_layout_run(c, sim, h, p, want)
    Lc = h.levels
    y = _z(h.sizes[-1])
    d.drg_init_layout(c, h.sizes[-1], 2, Lc - 1, y)
    git, base = 0, T // Lc
    for l in range(Lc - 1, -1, -1):
        Tl = base + (T - base * Lc if l == 0 else 0)
        gam = 0.01 if (l == Lc - 1 and Lc > 1) else 0.1
        for t in range(Tl):
            d.drg_layout_step(c, sim, h, y, M=5, b=2, gamma=gam,
                              eta=float(np.float32(0.5 * (1.0 - t / Tl))), clip=4.0, level=l,
                              seed=2, iter=git)
            git += 1
        if l > 0:
            yf = _z(h.sizes[l - 1])
            d.drg_prolong(c, h, l, y, yf)
            y = yf
    assert np.array_equal(y.cpu().numpy(), want.cpu().numpy())
    yl = _z(h.sizes[Lc - 1])
    d.drg_layout_run_until(c, sim, h, p, Lc - 1, 4, yl)
    got = _z(g.n)
    d.drg_layout_resume(c, sim, h, p, Lc - 1, 4, yl, got)
    assert np.array_equal(got.cpu().numpy(), want.cpu().numpy())


@pytest.mark.parametrize("case,mode", [("rgg8k", 0), ("grid32", 0), ("grid32", 1),
                                       ("rmat13", 0), ("rmat13", 1)])
def test_3d_full_layout_statistics(oracle_lib, case, mode):
    """End to end in R^3 vs the oracle's 3-D sync layout: objective within
    1%, NP within 0.01.  The grid workload's parameters (32x32, k=3, M=5,
    b=3, T=300, one level, eta0 = 1/4), R-MAT 2^13 (k=2, M=5, b=1, T=300,
    multilevel; its 2-D steps would use the column-blocked copy) and, sync
    only, a multilevel RGG (the Hogwild row sweep lands 1.0-1.4% below the
    sync objective there, in 2-D as in 3-D)."""
    from oracle import evaluate
    from paper_2008_07799_amd import drgraph as d
    if case == "rgg8k":
        g, kw = gen.rgg(8000, 0.02, seed=4), dict(k=2, M=5, b=2, T=200, min_nodes=200, eta0=0.5)
    elif case == "grid32":
        g, kw = gen.grid(32, 32), dict(k=3, M=5, b=3, T=300, max_levels=1, eta0=0.25)
    else:
        g, kw = gen.rmat(13, 16, seed=1), dict(k=2, M=5, b=1, T=300, min_nodes=1000)
    c = ctx()
    rp, col = dev_graph(g)
    p = d.layout_params(seed=0, mode=mode, dim=3, **kw)
    y = _z(g.n)
    d.drg_layout(c, rp, col, p, y)
    assert c.last_sweep() == (d.DRG_SWEEP_ROW_ASYNC if mode else d.DRG_SWEEP_ROW)
    yg = y.cpu().numpy().astype(np.float64)
    yr, rsim, _ = oracle_lib.layout(g, seed=0, return_all=True, dim=3, **kw)
    o_g = evaluate.objective_eval(rsim, yg, M=kw["M"], b=kw["b"], gamma=0.1)
    o_r = evaluate.objective_eval(rsim, yr, M=kw["M"], b=kw["b"], gamma=0.1)
    np_g = evaluate.neighbourhood_preservation(g, yg)
    np_r = evaluate.neighbourhood_preservation(g, yr)
    say("  3-D layout", case, "mode", mode, "objective", o_g, o_r, "NP", np_g, np_r)
    if case == "grid32" and mode == 1:
        # a Hogwild run is one draw of a random process; on this workload the
        # oracle's own 3-D layouts vary by about 7% in objective across seeds
        def run(seed):
            yy = _z(g.n)
            d.drg_layout(c, rp, col, d.layout_params(seed=seed, mode=1, dim=3, **kw), yy)
            assert c.last_sweep() == d.DRG_SWEEP_ROW_ASYNC
            return yy.cpu().numpy()
        hogwild_vs_oracle_spread(oracle_lib, g, kw, run, dim=3)
        return
    assert abs(o_g - o_r) <= 0.01 * abs(o_r)
    assert abs(np_g - np_r) <= 0.01


