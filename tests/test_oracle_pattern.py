"""Pins of the oracle's sparse distance matrix and node similarity
(Sec. 3.2.1, Eq. NS).  Marked "not gpu"."""
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

from paper_2008_07799_amd import gen

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = []
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def _spd(g):
    A = sp.csr_matrix((np.ones(g.nnz), g.col, g.row_ptr), shape=(g.n, g.n))
    return shortest_path(A, method="D", unweighted=True, directed=False)


@pytest.mark.parametrize("k", [1, 2, 3, 4])
@pytest.mark.parametrize("sub", [0, 1, 2])
def test_khop_matches_all_pairs_bfs(oracle_lib, k, sub):
    """NNG(v, k) = {u != v : SPD(v, u) <= k} with hop = SPD, rows ascending."""
    g = gen.random_graph(120, 0.025, seed=11, sub=sub)
    D = _spd(g)
    rp, col, hop = oracle_lib.khop(g, k)
    for v in range(g.n):
        want = np.nonzero((D[v] >= 1) & (D[v] <= k))[0]
        got = col[rp[v]:rp[v + 1]]
        assert np.array_equal(got, want)
        assert np.array_equal(hop[rp[v]:rp[v + 1]], D[v, want].astype(np.uint8))


def test_khop_k1_is_adjacency(oracle_lib):
    g = gen.rmat(10, 8, seed=2)
    rp, col, hop = oracle_lib.khop(g, 1)
    assert np.array_equal(rp, g.row_ptr.astype(np.int64))
    assert np.array_equal(col, g.col)
    assert np.all(hop == 1)


def test_khop_grid32_count(oracle_lib):
    (row,) = _golden("grid32_k3_pattern.txt")
    rp, col, hop = oracle_lib.khop(gen.grid(32, 32), 3)
    assert int(rp[-1]) == int(row[1])
    # SPD on a grid is the Manhattan distance
    r, c = np.divmod(np.repeat(np.arange(1024), np.diff(rp)), 32)
    cr, cc = np.divmod(col, 32)
    assert np.array_equal(np.abs(r - cr) + np.abs(c - cc), hop.astype(np.int64))


def test_grid_normalisers(oracle_lib):
    rows = {r[0]: (int(r[1]), int(r[2]), int(r[3]), float(r[4]))
            for r in _golden("grid_normalisers.txt")}
    sim = oracle_lib.similarity(gen.grid(32, 32), 3, sigma=1.0)
    interior = 10 * 32 + 10
    assert sim.Z[interior] == pytest.approx(rows["interior"][3], rel=1e-15)
    assert sim.Z[0] == pytest.approx(rows["corner"][3], rel=1e-15)
    h = sim.hop[sim.row_ptr[0]:sim.row_ptr[1]]
    assert [int((h == d).sum()) for d in (1, 2, 3)] == list(rows["corner"][:3])


def test_k1_similarity_is_inverse_degree(oracle_lib):
    """With first-order neighbours every hop is 1, so NS_{j|i} = 1/deg_i
    whatever sigma is, and P~_ij = (1/deg_i + 1/deg_j)/2."""
    g = gen.rgg(2000, 0.04, seed=5)
    for sigma in (0.5, 1.0, 3.0):
        sim = oracle_lib.similarity(g, 1, sigma)
        deg = np.diff(g.row_ptr).astype(np.float64)
        i = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
        want = 0.5 * (1.0 / deg[i] + 1.0 / deg[sim.col])
        assert np.allclose(sim.P, want, rtol=1e-15, atol=0)


@pytest.mark.parametrize("k", [2, 3])
def test_similarity_invariants(oracle_lib, k):
    g = gen.ba(400, 3, seed=1)
    sim = oracle_lib.similarity(g, k, sigma=1.3)
    n = g.n
    i = np.repeat(np.arange(n), np.diff(sim.row_ptr))
    # e_d is the Gaussian of the hop value
    assert np.allclose(sim.e, np.exp(-np.arange(1, k + 1) ** 2 / (2 * 1.3 ** 2)), rtol=1e-15)
    # conditional similarities sum to one over each neighbourhood
    p_cond = sim.e[sim.hop - 1] * sim.invZ[i]
    rows = np.bincount(i, weights=p_cond, minlength=n)
    assert np.allclose(rows[np.diff(sim.row_ptr) > 0], 1.0, rtol=1e-12)
    # P~ = (p_{j|i} + p_{i|j}) / 2, symmetric bit for bit
    A = sp.csr_matrix((sim.P, sim.col, sim.row_ptr), shape=(n, n))
    assert (A != A.T).nnz == 0
    pc = sp.csr_matrix((p_cond, sim.col, sim.row_ptr), shape=(n, n))
    assert np.allclose(A.toarray(), 0.5 * (pc + pc.T).toarray(), rtol=1e-13, atol=0)
    # total mass: sum_i qt_i = N_a; each active qt_i >= 1/2
    assert sim.qt.sum() == pytest.approx(sim.n_active, rel=1e-12)
    assert np.all(sim.qt[np.diff(sim.row_ptr) > 0] >= 0.5 - 1e-12)
    # integer weights: truncations of P~ 2^32 summed per row, exact prefix
    W = np.array([sum(int(math.floor(p * 2**32)) for p in sim.P[sim.row_ptr[v]:sim.row_ptr[v + 1]])
                  for v in range(n)], dtype=object)
    assert all(int(a) == int(b) for a, b in zip(sim.W, W))
    assert int(sim.C[0]) == 0
    assert all(int(sim.C[v + 1]) - int(sim.C[v]) == int(sim.W[v]) for v in range(n))


def test_isolated_nodes_have_empty_rows(oracle_lib):
    g = gen.canonical_csr(8, np.array([0, 1, 2]), np.array([1, 2, 3]))
    sim = oracle_lib.similarity(g, 2)
    assert [int(x) for x in np.diff(sim.row_ptr)] == [2, 3, 3, 2, 0, 0, 0, 0]
    assert np.all(sim.qt[4:] == 0) and np.all(sim.W[4:] == 0) and np.all(sim.invZ[4:] == 0)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_similarity_rows_pinned(oracle_lib, k):
    """The rows-only similarity (for graphs too large to take whole): its rows
    are NNG(v, k) with hop = SPD (all-pairs BFS), and its values, 1/Z, qt and
    W equal the whole-graph similarity's rows bit for bit, for a subset of
    sources in any order (isolated nodes included)."""
    g = gen.random_graph(150, 0.02, seed=13, sub=k)
    D = _spd(g)
    full = oracle_lib.similarity(g, k)
    rng = np.random.default_rng(k)
    src = rng.choice(g.n, size=40, replace=False)
    iso = np.nonzero(np.diff(g.row_ptr) == 0)[0]
    if len(iso):
        src = np.concatenate([src, iso[:2]])
    rows = oracle_lib.similarity_rows(g, k, src)
    rp = rows["row_ptr"]
    for r, v in enumerate(src):
        want = np.nonzero((D[v] >= 1) & (D[v] <= k))[0]
        a, b = rp[r], rp[r + 1]
        assert np.array_equal(rows["col"][a:b], want)
        assert np.array_equal(rows["hop"][a:b], D[v, want].astype(np.uint8))
        fa, fb = full.row_ptr[v], full.row_ptr[v + 1]
        assert np.array_equal(rows["P"][a:b], full.P[fa:fb])
        assert rows["invZ"][r] == full.invZ[v]
        assert rows["qt"][r] == full.qt[v]
        assert rows["W"][r] == full.W[v]
