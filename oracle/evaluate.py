"""Layout-quality evaluators of the oracle (TEST INFRASTRUCTURE ONLY).

* neighbourhood preservation NP (Sec. 4.1, Eq. NP): mean over nodes of the
  Jaccard index between NNG(v, k_eval) in the graph and the |NNG(v, k_eval)|
  nearest layout neighbours of y_v, with k_eval = 2.  Ties among layout
  distances are broken by node id.  Isolated nodes (empty NNG) are skipped.
  `np_per_node` computes it per node by brute force (every distance), the
  mean version with a k-d tree.
* stress (Sec. 4.1): weights 1/SPD^2, best scale alpha in closed form;
  `stress_terms` gives the per-source sums a sampled estimate is made of.
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


def stress_terms(csr, y, sources) -> np.ndarray:
    """Per source s: (A, B, P) = (sum L/D, sum L^2/D^2, number of pairs) over
    the nodes j != s reachable from s, L = ||y_s - y_j|| (FP64), D = the
    shortest-path distance (Sec. 4.1, stress with weights 1/D^2)."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import shortest_path
    y = np.asarray(y, dtype=np.float64)
    A = sp.csr_matrix((np.ones(len(csr.col)), csr.col, csr.row_ptr), shape=(csr.n, csr.n))
    D = shortest_path(A, method="D", unweighted=True, directed=False,
                      indices=np.asarray(sources))
    out = np.zeros((len(sources), 3))
    for t, s in enumerate(sources):
        ok = np.isfinite(D[t]) & (D[t] > 0)
        L = np.sqrt(((y[ok] - y[s]) ** 2).sum(axis=1))
        r = L / D[t][ok]
        out[t] = (r.sum(), (r * r).sum(), ok.sum())
    return out


def stress(csr, y, sources=None) -> float:
    """Normalised stress min_alpha (1/|V|^2) sum w (alpha L - D)^2, w = 1/D^2
    (Sec. 4.1): (P - A^2/B) / |V|^2, over all sources or scaled up from a
    sample of them."""
    n = int(csr.n)
    src = np.arange(n) if sources is None else np.asarray(sources)
    t = stress_terms(csr, y, src).sum(axis=0)
    if t[1] <= 0:
        return 0.0
    return (n / len(src)) * (t[2] - t[0] * t[0] / t[1]) / (n * n)


def objective_eval(sim, y, M: int, b: int, gamma: float, M_eval: int = 50,
                   seed: int = 0x5EED, it: int = 0) -> float:
    return drgo.objective(sim, y, M=M_eval, b=b, gamma=gamma * M / M_eval, seed=seed, it=it)
