"""Pins of the oracle's node-wise sigma_i (Eq. NS gives every node its own
Gaussian; sigma_i calibrated to a perplexity as in t-SNE).  Marked "not gpu".

The oracle computes its logarithm from IEEE operations only (atanh series);
these tests check it against libm, and every calibrated row against numpy's
own entropy, so no pin uses the oracle's arithmetic to check itself."""
import math

import numpy as np
import pytest

from paper_2008_07799_amd import gen


def _ring(n):
    u = np.arange(n)
    return gen.canonical_csr(n, u, (u + 1) % n, "ring")


def test_log_matches_libm(oracle_lib):
    L = oracle_lib.lib()
    rng = np.random.default_rng(0)
    xs = np.concatenate([10.0 ** rng.uniform(-300, 300, 4000),
                         1.0 + rng.uniform(-1e-6, 1e-6, 500),
                         rng.uniform(0.5, 2.0, 2000),
                         [1.0, 2.0, 0.5, math.sqrt(0.5), math.sqrt(2.0), 5e-324, 1.7e308]])
    for x in xs:
        got, want = L.drgo_ln(float(x)), math.log(float(x))
        # a few ulps of the result plus the rounding of e * ln 2
        assert abs(got - want) <= 4 * np.spacing(abs(want)) + 1e-16 * abs(math.frexp(x)[1]) \
            + 1e-300, x
    assert L.drgo_ln(1.0) == 0.0


@pytest.mark.parametrize("k,U", [(2, 4.0), (2, 10.0), (3, 30.0), (3, 200.0)])
def test_rows_reach_the_perplexity(oracle_lib, k, U):
    """Every non-empty row of NS_{.|i} sums to 1 and has entropy ln U, or is
    at one end of the reachable range: uniform over NNG(i, k) when U is at
    least its size, all mass on hop 1 when U is below the hop-1 count."""
    g = gen.rmat(11, 8, seed=3)
    s = oracle_lib.similarity_perplexity(g, k, U)
    hit = ends = 0
    for i in range(g.n):
        a, b = s.row_ptr[i], s.row_ptr[i + 1]
        if a == b:
            assert s.t[i] == 1.0 and s.invZ[i] == 0.0
            continue
        hop = s.hop[a:b].astype(np.int64)
        p = s.A[i, hop - 1]
        assert p.sum() == pytest.approx(1.0, abs=1e-13)
        H = -float(np.sum(p * np.log(p, where=p > 0, out=np.zeros_like(p))))
        N, c1 = b - a, int(np.count_nonzero(hop == 1))
        if N <= U:
            assert s.t[i] == 1.0
            assert np.allclose(p, 1.0 / N, rtol=1e-14, atol=0)
            ends += 1
        elif U < c1:
            assert s.t[i] < 1e-19
            assert np.allclose(p[hop == 1], 1.0 / c1, rtol=1e-14)
            ends += 1
        else:
            assert H == pytest.approx(math.log(U), abs=1e-10)
            hit += 1
    assert hit > 100


def test_ring_at_the_perplexity_of_sigma_one_is_the_global_sigma(oracle_lib):
    """On a ring every node has two nodes at each hop, so the perplexity of
    sigma = 1 is the same for all: calibrated to it, every t_i is
    exp(-1/2) and P~ is the global-sigma similarity."""
    g = _ring(40)
    k = 3
    e = np.exp(-np.arange(1, k + 1) ** 2 / 2.0)
    p = e / (2 * e.sum())
    U = math.exp(-2 * float(np.sum(p * np.log(p))))
    s = oracle_lib.similarity_perplexity(g, k, U)
    ref = oracle_lib.similarity(g, k, 1.0)
    assert np.allclose(s.t, math.exp(-0.5), rtol=1e-12, atol=0)
    assert np.allclose(oracle_lib.node_sigma(s), 1.0, rtol=1e-11)
    assert np.array_equal(s.col, ref.col) and np.array_equal(s.hop, ref.hop)
    assert np.allclose(s.P, ref.P, rtol=1e-12, atol=0)
    assert np.allclose(s.qt, ref.qt, rtol=1e-12, atol=0)


def test_k1_is_the_inverse_degree_similarity(oracle_lib):
    """With k = 1 every neighbour sits at hop 1, so sigma_i has no effect:
    P~_ij = (1/deg_i + 1/deg_j) / 2 whatever the perplexity."""
    g = gen.ba(500, 3, seed=2)
    deg = np.diff(g.row_ptr).astype(np.float64)
    for U in (1.0, 3.0, 50.0):
        s = oracle_lib.similarity_perplexity(g, 1, U)
        for i in range(g.n):
            a, b = s.row_ptr[i], s.row_ptr[i + 1]
            want = (1.0 / deg[i] + 1.0 / deg[s.col[a:b]]) / 2
            assert np.allclose(s.P[a:b], want, rtol=1e-14, atol=0)


def test_symmetry_total_mass_and_monotone_sigma(oracle_lib):
    """P~ symmetric bit for bit; sum of qt = N_a (each row of NS_{.|i} sums
    to one); a larger perplexity never gives a smaller sigma_i; W is the
    per-entry quantisation of P~."""
    g = gen.rgg(3000, 0.04, seed=4)
    prev = None
    for U in (3.0, 12.0, 40.0, 150.0):
        s = oracle_lib.similarity_perplexity(g, 2, U)
        rows = np.repeat(np.arange(g.n), np.diff(s.row_ptr))
        key = {(int(r), int(c)): v for r, c, v in zip(rows, s.col, s.P)}
        for (r, c), v in list(key.items())[::37]:
            assert key[(c, r)] == v
        assert s.qt.sum() == pytest.approx(s.n_active, rel=1e-12)
        W = np.zeros(g.n, np.uint64)
        np.add.at(W, rows, np.floor(s.P * 2.0 ** 32).astype(np.uint64))
        assert np.array_equal(W, s.W)
        if prev is not None:
            assert np.all(s.t >= prev.t)
        prev = s


def test_brute_force_entropy_on_a_tiny_graph(oracle_lib):
    """A 7-node tree, k = 3: the calibrated t of its centre found by a dense
    scan of t (10^5 points) to within the scan's step."""
    u = np.array([0, 0, 0, 1, 2, 3])
    v = np.array([1, 2, 3, 4, 5, 6])
    g = gen.canonical_csr(7, u, v)
    U = 4.0
    s = oracle_lib.similarity_perplexity(g, 3, U)
    c = np.array([3, 3, 0], np.float64)  # the centre: 3 at hop 1, 3 at hop 2
    ts = np.linspace(1e-6, 1.0, 100001)
    e = ts[:, None] ** (np.arange(1, 4) ** 2)[None, :]
    Z = (c[None, :] * e).sum(1)
    p = e / Z[:, None]
    H = -(c[None, :] * p * np.log(np.maximum(p, 1e-300))).sum(1)
    t_scan = ts[np.argmin(np.abs(H - math.log(U)))]
    assert s.t[0] == pytest.approx(t_scan, abs=2e-5)


def test_layout_with_perplexity_runs(oracle_lib):
    """The end-to-end oracle layout takes the node-wise similarity."""
    g = gen.grid(10, 10)
    y, sim, _ = oracle_lib.layout(g, k=3, M=5, b=1, T=30, min_nodes=1 << 30, max_levels=1,
                                  perplexity=8.0, return_all=True)
    assert sim.perplexity == 8.0 and np.all(np.isfinite(y))
    with pytest.raises(ValueError):
        oracle_lib.similarity_perplexity(g, 2, 0.5)
