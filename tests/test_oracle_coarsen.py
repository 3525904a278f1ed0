"""Pins of the oracle's coarsening (Sec. 3.2.3, Fig. 3).  Marked "not gpu".

The oracle visits nodes in descending (priority, -id) order and turns each
still-unassigned node into a centre that absorbs its unassigned neighbours.
The tests check it against a different algorithm with the same unique
answer -- rounds of local decisions (a node is a centre iff no higher-
priority neighbour is a centre) -- using priorities from numpy's Philox."""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_2008_07799_amd import gen


def _priorities(n, seed, level):
    pri = np.zeros(n, dtype=object)
    for v in range(n):
        g = np.random.Philox(counter=(v + (level << 64) - 1) % (1 << 256),
                             key=seed | (2 << 64))
        pri[v] = int(g.random_raw(1)[0])
    return pri


def _rounds_reference(g, seed, level):
    n = g.n
    pri = _priorities(n, seed, level)
    key = [(pri[v], -v) for v in range(n)]
    state = np.zeros(n, np.int8)  # 0 undecided, 1 centre, 2 member
    while (state == 0).any():
        new = state.copy()
        for v in np.nonzero(state == 0)[0]:
            higher = [u for u in g.col[g.row_ptr[v]:g.row_ptr[v + 1]] if key[u] > key[v]]
            if any(state[u] == 1 for u in higher):
                new[v] = 2
            elif all(state[u] == 2 for u in higher):
                new[v] = 1
        state = new
    owner = np.arange(n)
    for v in range(n):
        if state[v] == 2:
            cs = [u for u in g.col[g.row_ptr[v]:g.row_ptr[v + 1]] if state[u] == 1]
            owner[v] = max(cs, key=lambda u: key[u])
    centres = np.nonzero(state == 1)[0]
    rank = -np.ones(n, np.int64)
    rank[centres] = np.arange(centres.size)
    return rank[owner], centres.size


@pytest.mark.parametrize("maker", [
    lambda: gen.random_graph(150, 0.03, seed=2, sub=0),
    lambda: gen.grid(9, 11),
    lambda: gen.ba(200, 3, seed=4),
    lambda: gen.canonical_csr(12, np.array([0, 1, 2, 7]), np.array([1, 2, 3, 8])),
])
@pytest.mark.parametrize("level", [0, 3])
def test_coarsen_matches_parallel_rounds(oracle_lib, maker, level):
    g = maker()
    m, nc = oracle_lib.coarsen_level(g, seed=5, level=level)
    m_ref, nc_ref = _rounds_reference(g, 5, level)
    assert nc == nc_ref
    assert np.array_equal(m, m_ref)


def test_coarsen_groups_are_stars(oracle_lib):
    g = gen.rgg(3000, 0.03, seed=1)
    m, nc = oracle_lib.coarsen_level(g, seed=0, level=0)
    A = sp.csr_matrix((np.ones(g.nnz), g.col, g.row_ptr), shape=(g.n, g.n)).tolil()
    assert m.min() == 0 and m.max() == nc - 1
    # each coarse node holds exactly one centre: the smallest-rank id chosen
    # as centre is a member of its own group and adjacent to all the others
    for a in np.unique(m)[:300]:
        members = np.nonzero(m == a)[0]
        centres = [c for c in members if all(c == u or A[c, u] for u in members)]
        assert centres, "group is not a star"


def test_contract_is_galerkin_pattern(oracle_lib):
    """Coarse edges = distinct {c(u), c(v)} with c(u) != c(v): the pattern of
    C^T A C without its diagonal."""
    g = gen.ba(500, 3, seed=7)
    m, nc = oracle_lib.coarsen_level(g, seed=1, level=0)
    gc = oracle_lib.contract(g, m, nc)
    A = sp.csr_matrix((np.ones(g.nnz), g.col, g.row_ptr), shape=(g.n, g.n))
    Cm = sp.csr_matrix((np.ones(g.n), (np.arange(g.n), m)), shape=(g.n, nc))
    Ac = (Cm.T @ A @ Cm).tolil()
    Ac.setdiag(0)
    Ac = Ac.tocsr()
    Ac.eliminate_zeros()
    Ac.sort_indices()
    assert np.array_equal(gc.row_ptr, Ac.indptr.astype(np.int32))
    assert np.array_equal(gc.col, Ac.indices.astype(np.int32))


def test_hierarchy_stop_rules(oracle_lib):
    g = gen.rgg(20000, 0.013, seed=3)
    h = oracle_lib.hierarchy(g, seed=0, rho=0.8, min_nodes=100, max_levels=64)
    sizes = [oracle_lib.n_active_csr(x) for x in h.graphs]
    for a, b in zip(sizes, sizes[1:]):
        assert b <= 0.8 * a
    assert sizes[-1] < 100 or oracle_lib.n_active_csr(
        oracle_lib.contract(h.graphs[-1], *oracle_lib.coarsen_level(h.graphs[-1], 0, h.levels - 1))
    ) > 0.8 * sizes[-1]
    # composed maps are compositions of the one-level maps
    for l in range(1, h.levels):
        assert np.array_equal(h.cmaps[l], h.maps[l - 1][h.cmaps[l - 1]])
    h3 = oracle_lib.hierarchy(g, seed=0, rho=0.8, min_nodes=100, max_levels=3)
    assert h3.levels == 3 and h3.sizes == h.sizes[:3]
