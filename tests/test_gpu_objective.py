"""The sampled objective and its hand-written backward (marked gpu).

Bars: negatives bit-exact vs the oracle's draws; FP64 instance within 1e-12
(loss, relative) and 1e-10 (gradient, normwise) of the FP64 oracle; FP32
within 1e-5; FP64 central differences (h = 1e-6) on 64 coordinates of the
R-MAT 2^18 workload within 1e-5 of the backward; deterministic backward."""
import numpy as np
import pytest

from paper_2008_07799_amd import gen
from tests.gpu_util import ctx, dev_graph, normwise_rel, say, to_y

pytestmark = pytest.mark.gpu

CASES = {
    "rmat12": (lambda: gen.rmat(12, 8, seed=3), 2, 1),
    "grid32": (lambda: gen.grid(32, 32), 3, 3),
    "er300": (lambda: gen.random_graph(300, 0.02, seed=1), 2, 2),
}


def _sim(g, k):
    from paper_2008_07799_amd import drgraph as d
    rp, col = dev_graph(g)
    return d.drg_build_similarity(ctx(), rp, col, k)


@pytest.mark.parametrize("name", ["rmat12", "grid32"])
def test_negatives_bit_exact(oracle_lib, name):
    from paper_2008_07799_amd import drgraph as d
    say("negatives", name)
    maker, k, b = CASES[name]
    g = maker()
    sim = _sim(g, k)
    rsim = oracle_lib.similarity(g, k)
    M, seed, it = 7, 5, 9
    got = d.drg_sample_negatives(ctx(), sim, M, seed, it).cpu().numpy()
    active = np.diff(rsim.row_ptr) > 0
    for i in range(g.n):
        for m in range(M):
            want = oracle_lib.draw(rsim, oracle_lib.neg_word(seed, it, i, m)) if active[i] else -1
            assert got[i, m] == want


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("f64", [True, False])
def test_objective_and_gradient_match_oracle(oracle_lib, name, f64):
    import torch
    from paper_2008_07799_amd import drgraph as d
    say("objective", name, "f64" if f64 else "f32")
    maker, k, b = CASES[name]
    g = maker()
    sim = _sim(g, k)
    rsim = oracle_lib.similarity(g, k)
    rng = np.random.default_rng(3)
    y0 = rng.uniform(-3, 3, size=(g.n, 2))
    if not f64:
        y0 = y0.astype(np.float32).astype(np.float64)
    y = to_y(y0, np.float64 if f64 else np.float32)
    kw = dict(M=5, b=b, gamma=0.1, seed=4, iter=2)
    loss = float(d.drg_objective_fwd(ctx(), sim, y, **kw).cpu())
    grad = d.drg_objective_bwd(ctx(), sim, y, **kw).cpu().numpy().astype(np.float64)
    rloss = oracle_lib.objective(rsim, y0, 5, b, 0.1, 4, 2)
    rgrad = oracle_lib.objective_grad(rsim, y0, 5, b, 0.1, 4, 2)
    el = abs(loss - rloss) / abs(rloss)
    eg = normwise_rel(grad, rgrad)
    say("  loss err", el, "grad err", eg)
    assert el < (1e-12 if f64 else 1e-5)
    assert eg < (1e-10 if f64 else 1e-5)
    dl = torch.tensor(0.25, dtype=y.dtype, device="cuda")
    g2 = d.drg_objective_bwd(ctx(), sim, y, dl, **kw).cpu().numpy().astype(np.float64)
    assert np.array_equal(g2, (0.25 * torch.from_numpy(grad).to(y.dtype)).numpy().astype(np.float64)) \
        or normwise_rel(g2, 0.25 * grad) < 1e-7


def test_objective_rmat14_fp64_vs_oracle(oracle_lib):
    """R-MAT 2^14 (edge factor 16), k=2: the FP64 instance vs the oracle."""
    from paper_2008_07799_amd import drgraph as d
    say("objective rmat14 fp64")
    g = gen.rmat(14, 16, seed=2)
    sim = _sim(g, 2)
    rsim = oracle_lib.similarity(g, 2)
    y0 = np.random.default_rng(4).uniform(-5, 5, size=(g.n, 2))
    y = to_y(y0, np.float64)
    kw = dict(M=5, b=1, gamma=0.1, seed=0, iter=1)
    loss = float(d.drg_objective_fwd(ctx(), sim, y, **kw).cpu())
    grad = d.drg_objective_bwd(ctx(), sim, y, **kw).cpu().numpy()
    rloss = oracle_lib.objective(rsim, y0, 5, 1, 0.1, 0, 1)
    rgrad = oracle_lib.objective_grad(rsim, y0, 5, 1, 0.1, 0, 1)
    say("  loss", loss, rloss, "grad err", normwise_rel(grad, rgrad))
    assert abs(loss - rloss) <= 1e-12 * abs(rloss)
    assert normwise_rel(grad, rgrad) < 1e-10


def test_backward_is_deterministic():
    from paper_2008_07799_amd import drgraph as d
    say("bwd determinism")
    g = gen.rmat(12, 8, seed=3)
    sim = _sim(g, 2)
    y = to_y(np.random.default_rng(1).uniform(-2, 2, size=(g.n, 2)))
    a = d.drg_objective_bwd(ctx(), sim, y, M=5, b=1, gamma=0.1, seed=1, iter=1).cpu().numpy()
    b = d.drg_objective_bwd(ctx(), sim, y, M=5, b=1, gamma=0.1, seed=1, iter=1).cpu().numpy()
    assert np.array_equal(a, b)


def test_autograd_gradcheck_small():
    import torch
    from paper_2008_07799_amd import drgraph as d
    say("gradcheck")
    g = gen.random_graph(40, 0.12, seed=2)
    sim = _sim(g, 2)
    y = torch.from_numpy(np.random.default_rng(2).uniform(-2, 2, size=(g.n, 2))).cuda()
    y.requires_grad_(True)
    f = lambda t: d.objective(t, ctx(), sim, M=5, b=2, gamma=0.1, seed=3, iter=0)
    assert torch.autograd.gradcheck(f, (y,), eps=1e-6, atol=1e-6, rtol=1e-5)


def test_autograd_with_anchor_term():
    """loss = -L^/N_a + lam * mean over anchors of ||y_a - t_a||^2: the torch
    gradient equals -bwd/N_a plus the anchor term's own gradient."""
    import torch
    from paper_2008_07799_amd import drgraph as d
    say("anchor loss")
    g = gen.rmat(12, 8, seed=3)
    sim = _sim(g, 2)
    rng = np.random.default_rng(6)
    y = torch.from_numpy(rng.uniform(-2, 2, size=(g.n, 2)).astype(np.float32)).cuda()
    y.requires_grad_(True)
    idx = torch.from_numpy(rng.choice(g.n, size=g.n // 100, replace=False)).cuda()
    tgt = torch.from_numpy(rng.uniform(-1, 1, size=(idx.numel(), 2)).astype(np.float32)).cuda()
    L = d.objective(y, ctx(), sim, M=5, b=1, gamma=0.1, seed=0, iter=0)
    loss = -L / sim.n_active + 1.0 * ((y[idx] - tgt) ** 2).sum(dim=1).mean()
    loss.backward()
    want = -d.drg_objective_bwd(ctx(), sim, y.detach(), M=5, b=1, gamma=0.1, seed=0,
                                iter=0) / sim.n_active
    anchor = torch.zeros_like(want)
    anchor[idx] = 2.0 * (y.detach()[idx] - tgt) / idx.numel()
    assert torch.allclose(y.grad, want + anchor, rtol=1e-5, atol=1e-7)


def test_c5_central_differences_and_precision():
    """R-MAT 2^18, edge factor 8, k=2, M=5, b=1: FP64 central differences
    (h = 1e-6) on 64 random coordinates vs the FP64 backward; differences of
    the per-row values are summed so rows the perturbation does not touch
    cancel exactly.  FP32 loss and gradient vs the FP64 instance."""
    import torch
    from paper_2008_07799_amd import drgraph as d
    say("C5 FD")
    g = gen.rmat(18, 8, seed=0)
    sim = _sim(g, 2)
    rng = np.random.default_rng(8)
    y0 = rng.uniform(-5, 5, size=(g.n, 2))
    y = to_y(y0, np.float64)
    kw = dict(M=5, b=1, gamma=0.1, seed=0, iter=0)
    grad = d.drg_objective_bwd(ctx(), sim, y, **kw).cpu().numpy()
    act = np.nonzero(np.diff(sim.export(values=False)["row_ptr"]) > 0)[0]
    picks = rng.choice(act, size=32, replace=False)
    h = 1e-6
    worst = 0.0
    for i in picks:
        for c in (0, 1):
            yp = y.clone()
            ym = y.clone()
            yp[i, c] += h
            ym[i, c] -= h
            rp_ = d.drg_objective_fwd(ctx(), sim, yp, rows=True, **kw).cpu().numpy()
            rm_ = d.drg_objective_fwd(ctx(), sim, ym, rows=True, **kw).cpu().numpy()
            fd = float(np.sum(rp_ - rm_)) / (2 * h)
            err = abs(fd - grad[i, c]) / max(1.0, abs(grad[i, c]))
            worst = max(worst, err)
    say("  worst FD rel err", worst)
    assert worst < 1e-5
    y32 = y.float()
    l64 = float(d.drg_objective_fwd(ctx(), sim, y32.double(), **kw).cpu())
    l32 = float(d.drg_objective_fwd(ctx(), sim, y32, **kw).cpu())
    g64 = d.drg_objective_bwd(ctx(), sim, y32.double(), **kw).cpu().numpy()
    g32 = d.drg_objective_bwd(ctx(), sim, y32, **kw).cpu().numpy()
    say("  fp32 loss err", abs(l32 - l64) / abs(l64), "grad err", normwise_rel(g32, g64))
    assert abs(l32 - l64) <= 1e-5 * abs(l64)
    assert normwise_rel(g32, g64) < 1e-5


@pytest.mark.parametrize("name,bits", [("rmat12", 8), ("grid32", 6), ("er300", 6)])
def test_objective_on_blocked_layout_matches_oracle(oracle_lib, monkeypatch, name, bits):
    """FP32 objective and gradient through the column-blocked flat sweep (the
    path large graphs take; forced here with small blocks) vs the FP64 oracle,
    and vs the row kernels."""
    from paper_2008_07799_amd import drgraph as d
    say("objective blocked", name, bits)
    monkeypatch.setenv("DRG_SWEEP_BLOCKED", "1")
    monkeypatch.setenv("DRG_BLOCK_BITS", str(bits))
    maker, k, b = CASES[name]
    g = maker()
    sim = _sim(g, k)
    assert sim.blocked
    rsim = oracle_lib.similarity(g, k)
    rng = np.random.default_rng(5)
    y0 = rng.uniform(-3, 3, size=(g.n, 2)).astype(np.float32).astype(np.float64)
    y = to_y(y0, np.float32)
    kw = dict(M=5, b=b, gamma=0.1, seed=4, iter=2)
    loss = float(d.drg_objective_fwd(ctx(), sim, y, **kw).cpu())
    grad = d.drg_objective_bwd(ctx(), sim, y, **kw).cpu().numpy().astype(np.float64)
    rloss = oracle_lib.objective(rsim, y0, 5, b, 0.1, 4, 2)
    rgrad = oracle_lib.objective_grad(rsim, y0, 5, b, 0.1, 4, 2)
    say("  loss err", abs(loss - rloss) / abs(rloss), "grad err", normwise_rel(grad, rgrad))
    assert abs(loss - rloss) <= 1e-5 * abs(rloss)
    assert normwise_rel(grad, rgrad) < 1e-5
    monkeypatch.setenv("DRG_OBJ_BLOCKED", "0")
    loss_r = float(d.drg_objective_fwd(ctx(), sim, y, **kw).cpu())
    grad_r = d.drg_objective_bwd(ctx(), sim, y, **kw).cpu().numpy().astype(np.float64)
    assert abs(loss - loss_r) <= 1e-6 * abs(loss_r)
    assert normwise_rel(grad, grad_r) < 1e-6


def test_dynamic_graph_with_temporal_coherence():
    """A dynamic graph through the autograd form (the paper's Sec. 5 names a
    temporal-coherence term as the way to handle one): the graph at time t
    gains edges; starting from the layout of time t-1, Adam on
    -L^/N_a + lam * mean ||Y^t - Y^{t-1}||^2 (one fixed draw of negatives)
    keeps the new layout closer to the old one than lam = 0 does, while L^
    still improves in both runs."""
    import torch
    from paper_2008_07799_amd import drgraph as d
    say("dynamic graph")
    g1 = gen.ba(3000, 3, 0, sub=4)
    # time t: the same nodes plus 300 random new edges
    rng = np.random.default_rng(8)
    u = rng.integers(0, g1.n, 300)
    v = rng.integers(0, g1.n, 300)
    rows = np.repeat(np.arange(g1.n), np.diff(g1.row_ptr))
    g2 = gen.canonical_csr(g1.n, np.concatenate([rows, u]), np.concatenate([g1.col, v]), "ba+")
    c = ctx()
    rp1, col1 = dev_graph(g1)
    y_prev = torch.empty((g1.n, 2), dtype=torch.float32, device="cuda")
    d.drg_layout(c, rp1, col1, d.layout_params(k=2, M=5, b=1, T=200, seed=1), y_prev)
    sim2 = _sim(g2, 2)
    out = {}
    for lam in (0.0, 10.0):
        y = y_prev.clone().requires_grad_(True)
        opt = torch.optim.Adam([y], lr=0.01)
        # one fixed draw of negatives, so the objective is one smooth function
        L0 = float(d.objective(y.detach(), c, sim2, M=5, b=1, gamma=0.1, seed=0, iter=0))
        for it in range(60):
            opt.zero_grad()
            L = d.objective(y, c, sim2, M=5, b=1, gamma=0.1, seed=0, iter=0)
            loss = -L / sim2.n_active + lam * ((y - y_prev) ** 2).sum(dim=1).mean()
            loss.backward()
            opt.step()
        L1 = float(d.objective(y.detach(), c, sim2, M=5, b=1, gamma=0.1, seed=0, iter=0))
        drift = float(((y.detach() - y_prev) ** 2).sum(dim=1).mean())
        say("  lam", lam, "objective", L0, "->", L1, "drift", drift)
        assert L1 > L0
        out[lam] = drift
    assert out[10.0] < 0.5 * out[0.0]


def test_dynamic_graph_steps_match_oracle(oracle_lib):
    """The dynamic-graph form against the oracle: gradient descent on
    -L^(Y)/N_a + lam * mean ||Y - Y_prev||^2 for a graph that gained edges,
    from the previous layout, ten steps with fresh negatives each step,
    through the autograd form on the FP64 instance, vs the same steps taken
    on the CPU with the oracle's gradient (FP64) and the coherence term's
    closed-form gradient 2 lam (Y - Y_prev) / n: within 1e-9 after ten steps.
    One FP32 step: within 1e-5."""
    import torch
    from paper_2008_07799_amd import drgraph as d
    g1 = gen.ba(1500, 3, 0, sub=6)
    rng = np.random.default_rng(3)
    u = rng.integers(0, g1.n, 200)
    v = rng.integers(0, g1.n, 200)
    rows = np.repeat(np.arange(g1.n), np.diff(g1.row_ptr))
    g2 = gen.canonical_csr(g1.n, np.concatenate([rows, u]), np.concatenate([g1.col, v]), "ba+")
    c = ctx()
    sim2 = _sim(g2, 2)
    rsim2 = oracle_lib.similarity(g2, 2)
    na = rsim2.n_active
    y_prev = np.random.default_rng(4).uniform(-3, 3, size=(g1.n, 2))
    lam, lr = 5.0, 2.0
    yt = torch.from_numpy(y_prev.copy()).cuda()
    prev_t = torch.from_numpy(y_prev).cuda()
    yr = y_prev.copy()
    for it in range(10):
        y = yt.clone().requires_grad_(True)
        loss = (-d.objective(y, c, sim2, M=5, b=1, gamma=0.1, seed=0, iter=it) / na
                + lam * ((y - prev_t) ** 2).sum(dim=1).mean())
        loss.backward()
        yt = (y - lr * y.grad).detach()
        gr = (-oracle_lib.objective_grad(rsim2, yr, 5, 1, 0.1, 0, it) / na
              + 2.0 * lam * (yr - y_prev) / g1.n)
        yr = yr - lr * gr
    err = normwise_rel(yt.cpu().numpy(), yr)
    say("  dynamic FP64 ten steps err", err)
    assert err < 1e-9
    y32 = torch.from_numpy(y_prev.astype(np.float32)).cuda().requires_grad_(True)
    prev32 = torch.from_numpy(y_prev.astype(np.float32)).cuda()
    loss = (-d.objective(y32, c, sim2, M=5, b=1, gamma=0.1, seed=0, iter=0) / na
            + lam * ((y32 - prev32) ** 2).sum(dim=1).mean())
    loss.backward()
    y0 = y_prev.astype(np.float32).astype(np.float64)
    gr = -oracle_lib.objective_grad(rsim2, y0, 5, 1, 0.1, 0, 0) / na
    assert normwise_rel(y32.grad.cpu().numpy(), gr) < 1e-5
