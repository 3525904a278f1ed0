"""Layout-quality evaluators of the oracle (TEST INFRASTRUCTURE ONLY).

* neighbourhood preservation NP (Sec. 4.1, Eq. NP): mean over nodes of the
  Jaccard index between NNG(v, k_eval) in the graph and the |NNG(v, k_eval)|
  nearest layout neighbours of y_v, with k_eval = 2.  Ties among layout
  distances are broken by node id.  Isolated nodes (empty NNG) are skipped.
  `np_per_node` computes it per node by brute force (every distance), the
  mean version with a k-d tree.
* objective_eval: the sampled objective with a fixed evaluation seed and
  M_eval negatives per node, rescaled to M negatives.
"""
from __future__ import annotations

import numpy as np

from . import drgo


def np_per_node(y, rp, col, nodes) -> np.ndarray:
    """NP_v (Sec. 4.1, Eq. NP) of each node in `nodes` by brute force: the
    squared layout distance to every other node in FP64 (dx*dx + dy*dy),
    N_L(v) = the m = |N_G(v)| smallest (distance, id) pairs, N_G(v) = row v
    of the pattern (rp, col); NP_v = |N_G & N_L| / |N_G | N_L|, -1 for m = 0."""
    y = np.asarray(y, dtype=np.float64)
    n = y.shape[0]
    ids = np.arange(n)
    out = np.zeros(len(nodes), np.float64)
    for t, v in enumerate(nodes):
        v = int(v)
        m = int(rp[v + 1] - rp[v])
        if m == 0:
            out[t] = -1.0
            continue
        dx = y[v, 0] - y[:, 0]
        dy = y[v, 1] - y[:, 1]
        d2 = dx * dx + dy * dy
        d2[v] = np.inf
        thr = np.partition(d2, m - 1)[m - 1]
        less = d2 < thr
        eq = np.nonzero(d2 == thr)[0]  # ascending ids
        take = m - int(less.sum())
        layout = np.concatenate([ids[less], eq[:take]])
        inter = np.intersect1d(layout, col[rp[v]:rp[v + 1]], assume_unique=True).size
        out[t] = inter / (2.0 * m - inter)
    return out


def neighbourhood_preservation(csr, y, k_eval: int = 2, sample: int | None = None,
                               seed: int = 12345, pattern=None) -> float:
    from scipy.spatial import cKDTree

    y = np.asarray(y, dtype=np.float64)
    if pattern is None:
        rp, col, _ = drgo.khop(csr, k_eval)
    else:
        rp, col = pattern
    n = int(csr.n)
    sizes = np.diff(rp)
    nodes = np.nonzero(sizes > 0)[0]
    if sample is not None and nodes.size > sample:
        rng = np.random.default_rng(seed)
        nodes = np.sort(rng.choice(nodes, size=sample, replace=False))
    tree = cKDTree(y)
    total = 0.0
    for v in nodes:
        kv = int(sizes[v])
        want = min(n, kv + 1 + 8)
        d, idx = tree.query(y[v], k=want)
        d = np.atleast_1d(d)
        idx = np.atleast_1d(idx)
        ok = (idx != v) & (idx < n)
        d, idx = d[ok], idx[ok]
        order = np.lexsort((idx, d))
        layout_nb = set(idx[order][:kv].tolist())
        graph_nb = set(col[rp[v]:rp[v + 1]].tolist())
        inter = len(layout_nb & graph_nb)
        union = len(layout_nb | graph_nb)
        total += inter / union
    return total / max(1, nodes.size)


def objective_eval(sim, y, M: int, b: int, gamma: float, M_eval: int = 50,
                   seed: int = 0x5EED, it: int = 0) -> float:
    return drgo.objective(sim, y, M=M_eval, b=b, gamma=gamma * M / M_eval, seed=seed, it=it)
