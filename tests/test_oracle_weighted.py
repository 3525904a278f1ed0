"""Pins of the oracle's weighted-graph similarity (weighted graphs are named
as future work in Sec. 6; Eq. NS is written with the graph distance GD,
here the shortest path of at most k edges under positive symmetric edge
lengths).  Marked "not gpu"."""
import math

import numpy as np
import pytest

from paper_2008_07799_amd import gen


def _lengths(g, seed, lo=0.2, hi=3.0):
    return gen.edge_lengths(g, seed, lo, hi)


def _brute(g, ln, k, i):
    """min over walks of at most k edges from i, summed from i outwards."""
    best = {}

    def walk(u, d, depth):
        if depth == k:
            return
        for e in range(g.row_ptr[u], g.row_ptr[u + 1]):
            v = int(g.col[e])
            nd = d + float(ln[e])
            if v != i and nd < best.get(v, math.inf):
                best[v] = nd
            walk(v, nd, depth + 1)

    walk(i, 0.0, 0)
    return best


def test_exp_matches_libm(oracle_lib):
    L = oracle_lib.lib()
    xs = np.concatenate([-10.0 ** np.random.default_rng(0).uniform(-300, 2.85, 4000),
                         -np.random.default_rng(1).uniform(0, 1, 2000), [0.0, -1.0, -708.0]])
    for x in xs:
        got, want = L.drgo_exp_neg(float(x)), math.exp(float(x))
        assert abs(got - want) <= 2 * np.spacing(want), x
    assert L.drgo_exp_neg(-709.0) == 0.0 and L.drgo_exp_neg(0.0) == 1.0


@pytest.mark.parametrize("k", [1, 2, 3])
def test_distances_equal_brute_force_walks(oracle_lib, k):
    """Every entry's distance is the least walk length from either end,
    bit for bit (walk sums in the same order from the source)."""
    g = gen.random_graph(9, 0.35, seed=2)
    ln = _lengths(g, 3)
    s = oracle_lib.similarity_weighted(g, ln, k)
    for i in range(g.n):
        bi = _brute(g, ln, k, i)
        cols = s.col[s.row_ptr[i]:s.row_ptr[i + 1]]
        assert sorted(bi) == list(cols)
        for x, j in zip(range(s.row_ptr[i], s.row_ptr[i + 1]), cols):
            want = min(bi[int(j)], _brute(g, ln, k, int(j))[i])
            assert s.gd[x] == want


def test_unit_lengths_give_the_unweighted_similarity(oracle_lib):
    g = gen.rmat(10, 8, seed=1)
    ln = np.ones(len(g.col))
    for k in (1, 2, 3):
        s = oracle_lib.similarity_weighted(g, ln, k, 1.3)
        r = oracle_lib.similarity(g, k, 1.3)
        assert np.array_equal(s.gd, r.hop.astype(np.float64))
        # Z summed entry by entry here, hop histogram times e_d there
        assert np.allclose(s.P, r.P, rtol=1e-12, atol=0)
        assert np.allclose(s.qt, r.qt, rtol=1e-12, atol=0)


def test_path_closed_form_and_shortcut(oracle_lib):
    """On a path with lengths l_0, l_1, ... the distance over h <= k edges is
    the sum of the lengths in between; a long direct edge is bypassed when
    a two-edge route is shorter and allowed (k >= 2), not when k = 1."""
    n = 6
    u = np.arange(n - 1)
    g = gen.canonical_csr(n, u, u + 1)
    rows = np.repeat(np.arange(n), np.diff(g.row_ptr))
    seg = np.array([0.5, 1.25, 2.0, 0.75, 1.5])
    ln = seg[np.minimum(rows, g.col)]
    s = oracle_lib.similarity_weighted(g, ln, 3)
    for i in range(n):
        for x in range(s.row_ptr[i], s.row_ptr[i + 1]):
            j = int(s.col[x])
            a, b = min(i, j), max(i, j)
            assert s.gd[x] == pytest.approx(seg[a:b].sum(), rel=1e-15)
    # triangle 0-1-2 with a long 0-2 edge
    g = gen.canonical_csr(3, np.array([0, 1, 0]), np.array([1, 2, 2]))
    rows = np.repeat(np.arange(3), np.diff(g.row_ptr))
    ln = np.where((np.minimum(rows, g.col) == 0) & (np.maximum(rows, g.col) == 2), 5.0, 1.0)
    s1 = oracle_lib.similarity_weighted(g, ln, 1)
    s2 = oracle_lib.similarity_weighted(g, ln, 2)
    x02 = s1.row_ptr[0] + list(s1.col[s1.row_ptr[0]:s1.row_ptr[1]]).index(2)
    assert s1.gd[x02] == 5.0 and s2.gd[x02] == 2.0


def test_scale_invariance_symmetry_and_mass(oracle_lib):
    """Lengths and sigma scaled together leave P~ unchanged (to rounding);
    P~ is symmetric bit for bit; the row sums of NS_{.|i} give sum qt = N_a;
    W is the per-entry quantisation of P~."""
    g = gen.rgg(800, 0.08, seed=7)
    ln = _lengths(g, 5)
    s = oracle_lib.similarity_weighted(g, ln, 2, 1.0)
    t = oracle_lib.similarity_weighted(g, ln * 4.0, 2, 4.0)
    assert np.allclose(s.P, t.P, rtol=1e-13, atol=0)
    rows = np.repeat(np.arange(g.n), np.diff(s.row_ptr))
    key = {(int(r), int(c)): v for r, c, v in zip(rows, s.col, s.P)}
    for (r, c), v in key.items():
        assert key[(c, r)] == v
    assert s.qt.sum() == pytest.approx(s.n_active, rel=1e-12)
    W = np.zeros(g.n, np.uint64)
    np.add.at(W, rows, np.floor(s.P * 2.0 ** 32).astype(np.uint64))
    assert np.array_equal(W, s.W)


def test_weighted_layout_runs(oracle_lib):
    g = gen.grid(10, 10)
    ln = _lengths(g, 1)
    y, sim, _ = oracle_lib.layout(g, k=2, M=5, b=1, T=30, min_nodes=1 << 30, max_levels=1,
                                  lengths=ln, return_all=True)
    assert sim.gd is not None and np.all(np.isfinite(y))
