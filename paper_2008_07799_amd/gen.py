"""Seeded synthetic input graphs.

This module only makes inputs: undirected graphs in canonical CSR
form (symmetric, rows sorted ascending, no self-loops, no duplicate edges),
which is the input the layout method takes (Sec. 3.1, problem statement),
and edge lengths for weighted variants of them.
It holds none of the layout method's arithmetic, so both the GPU library's
tests and the CPU oracle's tests can draw their inputs from it.

Every generator is deterministic in its seed.  Random streams come from
numpy's Philox bit generator keyed by (seed, stream tag) so that two families
drawn with the same seed never share a stream.

Graph families stand in for the paper's dataset classes (Table 1), which are
not available here:
  * grid           -- 2-D lattices such as the 17x17 "grid17"
  * rgg            -- random geometric graphs (2-D finite-element-like meshes)
  * rmat           -- R-MAT power-law graphs (social / web graphs)
  * ba             -- Barabasi-Albert preferential attachment graphs
  * grid_deleted   -- grids with a fraction of edges removed
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

_TAG_RMAT = 11
_TAG_RGG = 12
_TAG_GRID_DEL = 13
_TAG_BA = 14
_TAG_BATCH = 15
_TAG_MISC = 16


def _rng(seed: int, tag: int, sub: int = 0) -> np.random.Generator:
    key = np.array([int(seed) & 0xFFFFFFFFFFFFFFFF,
                    ((int(tag) & 0xFFFFFFFF) << 32) | (int(sub) & 0xFFFFFFFF)],
                   dtype=np.uint64)
    return np.random.Generator(np.random.Philox(key=key))


@dataclass
class CSR:
    """Canonical undirected graph: int32 row_ptr[n+1], int32 col[nnz]."""
    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def n_edges(self) -> int:
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))


def canonical_csr(n: int, u: np.ndarray, v: np.ndarray, name: str = "") -> CSR:
    """Symmetrise an edge list, drop self-loops and duplicates, sort rows."""
    u = np.asarray(u, dtype=np.int64).ravel()
    v = np.asarray(v, dtype=np.int64).ravel()
    keep = u != v
    u, v = u[keep], v[keep]
    src = np.concatenate([u, v])
    dst = np.concatenate([v, u])
    key = np.unique(src * np.int64(n) + dst)
    src = key // n
    dst = key - src * n
    counts = np.bincount(src, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("graph too large for int32 CSR")
    return CSR(n, row_ptr.astype(np.int32), dst.astype(np.int32), name)


def grid(rows: int, cols: int) -> CSR:
    """rows x cols 4-neighbour lattice, node id = r*cols + c."""
    idx = np.arange(rows * cols, dtype=np.int64).reshape(rows, cols)
    u = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    v = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    return canonical_csr(rows * cols, u, v, f"grid{rows}x{cols}")


def grid_deleted(n: int, frac: float = 0.05, seed: int = 0, sub: int = 0) -> CSR:
    """First n nodes (row-major) of an r x ceil(n/r) grid, r = floor(sqrt(n)),
    with round(frac*|E|) edges removed, chosen by a seeded shuffle."""
    r = max(1, int(math.isqrt(n)))
    c = -(-n // r)
    idx = np.arange(r * c, dtype=np.int64).reshape(r, c)
    u = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    v = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    keep = (u < n) & (v < n)
    u, v = u[keep], v[keep]
    order = np.lexsort((v, u))
    u, v = u[order], v[order]
    n_del = int(round(frac * u.size))
    rng = _rng(seed, _TAG_GRID_DEL, sub)
    drop = rng.permutation(u.size)[:n_del]
    mask = np.ones(u.size, dtype=bool)
    mask[drop] = False
    return canonical_csr(n, u[mask], v[mask], f"griddel{n}")


def rgg(n: int, radius: float, seed: int = 0) -> CSR:
    """n points uniform in [0,1)^2; an edge joins every pair strictly closer
    than `radius` (no wrap-around)."""
    from scipy.spatial import cKDTree

    rng = _rng(seed, _TAG_RGG)
    pts = rng.random((n, 2))
    pairs = cKDTree(pts).query_pairs(radius, output_type="ndarray")
    if pairs.size:
        d2 = ((pts[pairs[:, 0]] - pts[pairs[:, 1]]) ** 2).sum(axis=1)
        pairs = pairs[d2 < radius * radius]
    return canonical_csr(n, pairs[:, 0], pairs[:, 1], f"rgg{n}")


def rmat(scale: int, edge_factor: int, a: float = 0.57, b: float = 0.19,
         c: float = 0.19, seed: int = 0, permute: bool = True) -> CSR:
    """R-MAT: 2^scale nodes, edge_factor*2^scale recursive quadrant draws
    with probabilities (a, b, c, d=1-a-b-c); ids shuffled by a seeded
    permutation so hubs do not sit at low ids; then symmetrised with
    self-loops and duplicates removed."""
    n = 1 << scale
    e = edge_factor * n
    rng = _rng(seed, _TAG_RMAT)
    u = np.zeros(e, dtype=np.int64)
    v = np.zeros(e, dtype=np.int64)
    t1, t2, t3 = a, a + b, a + b + c
    for _ in range(scale):
        r = rng.random(e)
        ub = r >= t2
        vb = ((r >= t1) & (r < t2)) | (r >= t3)
        u = (u << 1) | ub
        v = (v << 1) | vb
        del r, ub, vb
    if permute:
        perm = rng.permutation(n).astype(np.int64)
        u = perm[u]
        v = perm[v]
    return canonical_csr(n, u, v, f"rmat{scale}_{edge_factor}")


def ba(n: int, m: int = 3, seed: int = 0, sub: int = 0) -> CSR:
    """Barabasi-Albert: start from an (m+1)-clique; each new node attaches to
    m distinct existing nodes chosen with probability proportional to degree."""
    m0 = m + 1
    n = max(n, m0)
    rng = _rng(seed, _TAG_BA, sub)
    cu = [i for i in range(m0) for j in range(i + 1, m0)]
    cv = [j for i in range(m0) for j in range(i + 1, m0)]
    n_edges = len(cu) + (n - m0) * m
    # endpoint list: each edge contributes both endpoints; a uniform pick
    # from it is a degree-proportional pick
    rep = np.empty(2 * n_edges, dtype=np.int64)
    rep[: len(cu)] = cu
    rep[len(cu): 2 * len(cu)] = cv
    fill = 2 * len(cu)
    eu = np.empty(n_edges, dtype=np.int64)
    ev = np.empty(n_edges, dtype=np.int64)
    eu[: len(cu)] = cu
    ev[: len(cu)] = cv
    ne = len(cu)
    pool = rng.random(8 * m * (n - m0) + 64)
    pp = 0
    for t in range(m0, n):
        chosen = []
        while len(chosen) < m:
            if pp >= pool.size:
                pool = rng.random(pool.size)
                pp = 0
            x = int(rep[int(pool[pp] * fill)])
            pp += 1
            if x not in chosen:
                chosen.append(x)
        for x in chosen:
            eu[ne] = t
            ev[ne] = x
            ne += 1
            rep[fill] = t
            rep[fill + 1] = x
            fill += 2
    return canonical_csr(n, eu[:ne], ev[:ne], f"ba{n}")


def batch_sizes(G: int = 512, lo: int = 500, hi: int = 50_000, seed: int = 0) -> np.ndarray:
    """Node counts drawn log-uniform in [lo, hi]."""
    rng = _rng(seed, _TAG_BATCH)
    x = rng.random(G)
    return np.floor(np.exp(math.log(lo) + x * (math.log(hi) - math.log(lo)))).astype(np.int64)


def batch_graphs(G: int = 512, lo: int = 500, hi: int = 50_000, seed: int = 0):
    """Graph g is a grid with 5% of its edges deleted when g is even,
    otherwise a Barabasi-Albert graph with m=3."""
    sizes = batch_sizes(G, lo, hi, seed)
    out = []
    for g, n in enumerate(sizes):
        if g % 2 == 0:
            out.append(grid_deleted(int(n), 0.05, seed, sub=g))
        else:
            out.append(ba(int(n), 3, seed, sub=g))
    return out


def random_graph(n: int, p: float, seed: int = 0, sub: int = 0) -> CSR:
    """Erdos-Renyi G(n, p), for small test graphs."""
    rng = _rng(seed, _TAG_MISC, sub)
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(iu.size) < p
    return canonical_csr(n, iu[keep], ju[keep], f"er{n}")


_TAG_LENGTHS = 17


def edge_lengths(g: CSR, seed: int = 0, lo: float = 0.2, hi: float = 3.0) -> np.ndarray:
    """Edge lengths for a weighted variant of g: one float64 per CSR entry,
    uniform in [lo, hi), equal for (u, v) and (v, u)."""
    rng = _rng(seed, _TAG_LENGTHS)
    rows = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
    a = np.minimum(rows, g.col.astype(np.int64))
    b = np.maximum(rows, g.col.astype(np.int64))
    uniq, inv = np.unique(a * g.n + b, return_inverse=True)
    return rng.uniform(lo, hi, size=len(uniq))[inv]


def named(config: str, seed: int = 0) -> CSR:
    """The evaluation inputs by name."""
    if config == "grid32":
        return grid(32, 32)
    if config == "grid17":
        return grid(17, 17)
    if config == "rgg100k":
        return rgg(100_000, 0.006, seed)
    if config == "rmat20":
        return rmat(20, 16, seed=seed)
    if config == "rmat18":
        return rmat(18, 8, seed=seed)
    if config.startswith("rmat"):
        # rmat<scale>_<edge_factor>
        s, f = config[4:].split("_")
        return rmat(int(s), int(f), seed=seed)
    raise KeyError(config)
