"""Pins of the oracle's random streams: the Philox4x64-10 bijection, the
initial layout and the negative-sample draw.  Marked "not gpu"."""
import math

import numpy as np
import pytest

from paper_2008_07799_amd import gen


def _numpy_philox(ctr, key):
    """numpy's independent Philox4x64-10: it increments the 256-bit counter
    before producing its first block."""
    c = sum(int(x) << (64 * i) for i, x in enumerate(ctr))
    k = int(key[0]) | (int(key[1]) << 64)
    g = np.random.Philox(counter=(c - 1) % (1 << 256), key=k)
    return g.random_raw(4).astype(np.uint64)


def test_philox_matches_numpy(oracle_lib):
    rng = np.random.default_rng(7)
    for _ in range(500):
        ctr = rng.integers(0, 2**64, size=4, dtype=np.uint64)
        key = rng.integers(0, 2**64, size=2, dtype=np.uint64)
        assert np.array_equal(oracle_lib.philox(ctr, key), _numpy_philox(ctr, key))
    # structured counters as the method uses them (small ints, zero high word)
    for a in range(50):
        ctr = np.array([a, 3, a % 4, 0], np.uint64)
        key = np.array([0, 3], np.uint64)
        assert np.array_equal(oracle_lib.philox(ctr, key), _numpy_philox(ctr, key))


def test_init_uniform_grid(oracle_lib):
    """Random layout of the coarsest graph (Sec. 3.2.3): every coordinate is
    2u-1 with u a 24-bit fraction of the Philox word for (node, level)."""
    y = oracle_lib.init(1000, seed=0, level=2)
    assert y.shape == (1000, 2)
    assert np.all(y >= -1.0) and np.all(y < 1.0)
    assert np.all((y * 2**23) == np.round(y * 2**23))
    for v in (0, 1, 517, 999):
        w = _numpy_philox([v, 2, 0, 0], [0, 1])
        ux = float(int(w[0]) >> 40) / 2**24
        uy = float(int(w[1]) >> 40) / 2**24
        assert y[v, 0] == 2 * ux - 1 and y[v, 1] == 2 * uy - 1
    assert abs(y.mean()) < 0.05 and abs(y.var() - 1 / 3) < 0.03


def _small_sim(oracle_lib, n=60, p=0.08, k=2, sub=0):
    g = gen.random_graph(n, p, seed=3, sub=sub)
    return g, oracle_lib.similarity(g, k)


def test_draw_is_inverse_cdf(oracle_lib):
    """draw(w) is the unique v with C_v <= floor(w S / 2^64) < C_{v+1}."""
    g, sim = _small_sim(oracle_lib)
    S = int(sim.C[-1])
    Cs = [int(c) for c in sim.C]
    rng = np.random.default_rng(0)
    words = [int(x) for x in rng.integers(0, 2**64, size=3000, dtype=np.uint64)]
    words += [0, 2**64 - 1]
    for w in words:
        r = (w * S) >> 64
        v = oracle_lib.draw(sim, w)
        assert Cs[v] <= r < Cs[v + 1]


def test_draw_never_returns_isolated(oracle_lib):
    g = gen.canonical_csr(10, np.array([0, 1, 5]), np.array([1, 2, 6]))
    sim = oracle_lib.similarity(g, 1)
    active = set(np.nonzero(np.diff(sim.row_ptr))[0].tolist())
    rng = np.random.default_rng(1)
    for w in rng.integers(0, 2**64, size=5000, dtype=np.uint64):
        assert oracle_lib.draw(sim, int(w)) in active


def test_negative_frequencies_chi2(oracle_lib):
    """Draws over (iteration, node, slot) follow the node weights W/S
    (Sec. 3.2.2: negatives by node weight sum_l NS_{j,l})."""
    from scipy.stats import chisquare

    g, sim = _small_sim(oracle_lib, n=40, p=0.15, k=1, sub=1)
    n = sim.n
    counts = np.zeros(n)
    draws = 0
    for it in range(200):
        for i in range(n):
            for m in range(10):
                counts[oracle_lib.draw(sim, oracle_lib.neg_word(0, it, i, m))] += 1
                draws += 1
    p = sim.W.astype(np.float64) / float(sim.C[-1])
    mask = p > 0
    assert counts[~mask].sum() == 0
    stat, pval = chisquare(counts[mask], draws * p[mask])
    assert pval > 1e-4


def test_neg_word_slots_share_one_block(oracle_lib):
    """Slots 4g..4g+3 of one (iteration, node) take the four words of one
    Philox block with counter (node, iteration, g, 0), key (seed, 3)."""
    w = _numpy_philox([17, 5, 1, 0], [9, 3])
    for s in range(4):
        assert oracle_lib.neg_word(9, 5, 17, 4 + s) == int(w[s])
