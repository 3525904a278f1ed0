"""Python side of the CPU oracle (TEST INFRASTRUCTURE ONLY).

Loads libdrgo.so (plain FP64 C, built from drgo.c by oracle/build.py) and
composes its steps into the full multilevel layout in the paper's order
(Sec. 3.2): sparse distance matrix -> node similarity -> coarsening ->
random layout of the coarsest graph -> optimisation with gradients forwarded
to the level nodes -> refinement by copying coarse positions, level by level.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this module.  It shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "libdrgo.so")

_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    src = os.path.join(_HERE, "drgo.c")
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(src):
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", _LIB, src, "-lm"], cwd=_HERE)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    build()
    L = C.CDLL(_LIB)
    L.drgo_philox.argtypes = [_u64p, _u64p, _u64p]
    L.drgo_khop_count.argtypes = [C.c_int32, _i32p, _i32p, C.c_int32, _i64p]
    L.drgo_khop_count.restype = C.c_int64
    L.drgo_khop_fill.argtypes = [C.c_int32, _i32p, _i32p, C.c_int32, _i64p, _i32p, _u8p]
    L.drgo_similarity.argtypes = [C.c_int32, C.c_int32, C.c_double, _i64p, _i32p, _u8p,
                                  _f64p, _f64p, _f64p, _f64p, _f64p, _u64p, _u64p]
    L.drgo_similarity_rows.argtypes = [C.c_int32, _i32p, _i32p, C.c_int32, C.c_double,
                                       C.c_int32, _i32p, _i64p, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    L.drgo_similarity_rows.restype = C.c_int64
    L.drgo_similarity_perplexity.argtypes = [C.c_int32, C.c_int32, C.c_double, _i64p, _i32p,
                                             _u8p, _f64p, _f64p, _f64p, _f64p, _f64p, _f64p,
                                             _u64p, _u64p]
    L.drgo_similarity_perplexity.restype = C.c_int32
    L.drgo_hop_bounded_dist.argtypes = [C.c_int32, _i32p, _i32p, _f64p, C.c_int32, _i64p,
                                        _i32p, _f64p]
    L.drgo_similarity_weighted.argtypes = [C.c_int32, C.c_double, _i64p, _i32p, _f64p, _f64p,
                                           _f64p, _f64p, _f64p, _f64p, _u64p, _u64p]
    L.drgo_exp_neg.argtypes = [C.c_double]
    L.drgo_exp_neg.restype = C.c_double
    L.drgo_ln.argtypes = [C.c_double]
    L.drgo_ln.restype = C.c_double
    L.drgo_draw.argtypes = [_u64p, C.c_int32, C.c_uint64]
    L.drgo_draw.restype = C.c_int32
    L.drgo_neg_word.argtypes = [C.c_uint64, C.c_uint64, C.c_int32, C.c_int32]
    L.drgo_neg_word.restype = C.c_uint64
    L.drgo_coarsen_level.argtypes = [C.c_int32, _i32p, _i32p, C.c_uint64, C.c_int32, _i32p]
    L.drgo_coarsen_level.restype = C.c_int32
    L.drgo_contract.argtypes = [C.c_int32, _i32p, _i32p, _i32p, C.c_int32, _i32p, _i32p]
    L.drgo_contract.restype = C.c_int64
    L.drgo_init.argtypes = [C.c_int32, C.c_uint64, C.c_int32, _f64p, C.c_int32]
    cmap_t = C.c_void_p
    step_args = [C.c_int32, _i64p, _i32p, _f64p, _f64p, _u64p, cmap_t, _f64p,
                 C.c_int32, C.c_double, C.c_double, C.c_double, C.c_uint64, C.c_uint64, _f64p,
                 C.c_int32]
    L.drgo_step_direction.argtypes = step_args
    it_args = [C.c_int32, _i64p, _i32p, _f64p, _f64p, _u64p, cmap_t, C.c_int32, _f64p,
               C.c_int32, C.c_double, C.c_double, C.c_double, C.c_double, C.c_uint64, C.c_uint64,
               C.c_int32]
    L.drgo_iter_sync.argtypes = it_args
    L.drgo_iter_seq.argtypes = it_args
    obj_args = [C.c_int32, _i64p, _i32p, _f64p, _f64p, _u64p, _f64p, C.c_int32, C.c_double,
                C.c_double, C.c_uint64, C.c_uint64]
    L.drgo_objective.argtypes = obj_args + [C.c_int32]
    L.drgo_objective.restype = C.c_double
    L.drgo_objective_grad.argtypes = obj_args + [_f64p, C.c_int32]
    ex_args = [C.c_int32, _i64p, _i32p, _f64p, _f64p, _u64p, _f64p, C.c_int32, C.c_double,
               C.c_double]
    L.drgo_objective_exact.argtypes = ex_args + [C.c_int32]
    L.drgo_objective_exact.restype = C.c_double
    L.drgo_objective_exact_grad.argtypes = ex_args + [_f64p, C.c_int32]
    L.drgo_step_expected.argtypes = ex_args + [_f64p, C.c_int32]
    _lib = L
    return L


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


# ---------------------------------------------------------------- primitives
def philox(ctr, key) -> np.ndarray:
    out = np.zeros(4, np.uint64)
    lib().drgo_philox(_c(ctr, np.uint64), _c(key, np.uint64), out)
    return out


@dataclass
class Sim:
    """Sparse similarity P~ (CSR over all n nodes) plus sampling table."""
    n: int
    k: int
    sigma: float
    row_ptr: np.ndarray  # int64[n+1]
    col: np.ndarray      # int32[nnz]
    hop: np.ndarray      # uint8[nnz]
    e: np.ndarray        # float64[k]
    Z: np.ndarray
    invZ: np.ndarray
    P: np.ndarray        # float64[nnz]
    qt: np.ndarray       # float64[n]
    W: np.ndarray        # uint64[n]
    C: np.ndarray        # uint64[n+1]
    perplexity: float = 0.0  # > 0: node-wise sigma_i calibrated to it
    t: np.ndarray = None     # float64[n]: exp(-1/(2 sigma_i^2)) per node
    A: np.ndarray = None     # float64[n, k]: NS_{j|i} of hop d in A[i, d-1]
    gd: np.ndarray = None    # float64[nnz]: weighted graph distance per entry
    E: np.ndarray = None     # float64[nnz]: exp(-gd^2 / (2 sigma^2))

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def n_active(self) -> int:
        return int(np.count_nonzero(np.diff(self.row_ptr)))


def khop(csr, k: int):
    """Rows of NNG(v, k) with hop counts, ascending column order."""
    L = lib()
    n = int(csr.n)
    rp = _c(csr.row_ptr, np.int32)
    col = _c(csr.col, np.int32)
    out_rp = np.zeros(n + 1, np.int64)
    nnz = L.drgo_khop_count(n, rp, col, int(k), out_rp)
    out_col = np.zeros(max(nnz, 1), np.int32)
    out_hop = np.zeros(max(nnz, 1), np.uint8)
    L.drgo_khop_fill(n, rp, col, int(k), out_rp, out_col, out_hop)
    return out_rp, out_col[:nnz], out_hop[:nnz]


def similarity(csr, k: int, sigma: float = 1.0) -> Sim:
    rp, col, hop = khop(csr, k)
    return similarity_from_pattern(int(csr.n), k, sigma, rp, col, hop)


def similarity_from_pattern(n, k, sigma, rp, col, hop) -> Sim:
    nnz = int(rp[-1])
    e = np.zeros(k, np.float64)
    Z = np.zeros(n, np.float64)
    invZ = np.zeros(n, np.float64)
    P = np.zeros(max(nnz, 1), np.float64)
    qt = np.zeros(n, np.float64)
    W = np.zeros(n, np.uint64)
    Cc = np.zeros(n + 1, np.uint64)
    colc = _c(col if nnz else np.zeros(1, np.int32), np.int32)
    hopc = _c(hop if nnz else np.ones(1, np.uint8), np.uint8)
    lib().drgo_similarity(n, k, float(sigma), _c(rp, np.int64), colc, hopc,
                          e, Z, invZ, P, qt, W, Cc)
    return Sim(n, k, float(sigma), _c(rp, np.int64), colc[:nnz], hopc[:nnz], e, Z, invZ,
               P[:nnz], qt, W, Cc)


def similarity_perplexity(csr, k: int, perplexity: float) -> Sim:
    """P~ with one sigma_i per node (Eq. NS), each chosen so that NS_{.|i}
    has the given perplexity (t-SNE's calibration); see
    drgo_similarity_perplexity."""
    rp, col, hop = khop(csr, k)
    return similarity_perplexity_from_pattern(int(csr.n), k, perplexity, rp, col, hop)


def similarity_perplexity_from_pattern(n, k, perplexity, rp, col, hop) -> Sim:
    nnz = int(rp[-1])
    t = np.zeros(n, np.float64)
    A = np.zeros(n * k, np.float64)
    Z = np.zeros(n, np.float64)
    invZ = np.zeros(n, np.float64)
    P = np.zeros(max(nnz, 1), np.float64)
    qt = np.zeros(n, np.float64)
    W = np.zeros(n, np.uint64)
    Cc = np.zeros(n + 1, np.uint64)
    colc = _c(col if nnz else np.zeros(1, np.int32), np.int32)
    hopc = _c(hop if nnz else np.ones(1, np.uint8), np.uint8)
    rc = lib().drgo_similarity_perplexity(n, k, float(perplexity), _c(rp, np.int64), colc, hopc,
                                          t, A, Z, invZ, P, qt, W, Cc)
    if rc != 0:
        raise ValueError("k must be in 1..8 and perplexity >= 1")
    return Sim(n, k, 0.0, _c(rp, np.int64), colc[:nnz], hopc[:nnz], np.zeros(k), Z, invZ,
               P[:nnz], qt, W, Cc, float(perplexity), t, A.reshape(n, k))


def similarity_weighted(csr, lengths, k: int, sigma: float = 1.0) -> Sim:
    """P~ of a graph with positive symmetric edge lengths (one per CSR
    entry): GD_ij = the shortest path of at most k edges, the pattern the
    hop-defined NNG(i, k); see drgo_hop_bounded_dist."""
    rp, col, hop = khop(csr, k)
    n = int(csr.n)
    nnz = int(rp[-1])
    colc = _c(col if nnz else np.zeros(1, np.int32), np.int32)
    gd = np.zeros(max(nnz, 1), np.float64)
    lib().drgo_hop_bounded_dist(n, _c(csr.row_ptr, np.int32), _c(csr.col, np.int32),
                                _c(lengths, np.float64), int(k), _c(rp, np.int64), colc, gd)
    E = np.zeros(max(nnz, 1), np.float64)
    Z = np.zeros(n, np.float64)
    invZ = np.zeros(n, np.float64)
    P = np.zeros(max(nnz, 1), np.float64)
    qt = np.zeros(n, np.float64)
    W = np.zeros(n, np.uint64)
    Cc = np.zeros(n + 1, np.uint64)
    lib().drgo_similarity_weighted(n, float(sigma), _c(rp, np.int64), colc, gd, E, Z, invZ, P,
                                   qt, W, Cc)
    hopc = _c(hop if nnz else np.ones(1, np.uint8), np.uint8)
    return Sim(n, k, float(sigma), _c(rp, np.int64), colc[:nnz], hopc[:nnz], np.zeros(k), Z,
               invZ, P[:nnz], qt, W, Cc, gd=gd[:nnz], E=E[:nnz])


def node_sigma(sim: Sim) -> np.ndarray:
    """sigma_i = sqrt(-1 / (2 ln t_i)) of a node-wise similarity (inf where
    t_i = 1, the uniform distribution; 0 for isolated nodes)."""
    out = np.zeros(sim.n, np.float64)
    act = np.diff(sim.row_ptr) > 0
    with np.errstate(divide="ignore"):
        lt = np.log(sim.t[act])
        out[act] = np.where(lt < 0, np.sqrt(-0.5 / np.where(lt < 0, lt, -1.0)), np.inf)
    return out


def similarity_rows(csr, k: int, sources, sigma: float = 1.0) -> dict:
    """P~ restricted to the rows `sources` (Sec. 3.2.1, as `similarity`), for
    graphs too large to take whole: per row its columns (ascending), hops,
    values, and 1/Z, qt, W of the row."""
    L = lib()
    n = int(csr.n)
    rp = _c(csr.row_ptr, np.int32)
    col = _c(csr.col, np.int32)
    src = _c(sources, np.int32)
    out_rp = np.zeros(len(src) + 1, np.int64)
    nnz = L.drgo_similarity_rows(n, rp, col, int(k), float(sigma), len(src), src, out_rp,
                                 None, None, None, None, None, None)
    if nnz < 0:
        raise ValueError("k out of range")
    out_col = np.zeros(max(nnz, 1), np.int32)
    out_hop = np.zeros(max(nnz, 1), np.uint8)
    out_P = np.zeros(max(nnz, 1), np.float64)
    invZ = np.zeros(len(src), np.float64)
    qt = np.zeros(len(src), np.float64)
    W = np.zeros(len(src), np.uint64)
    ptr = lambda a: a.ctypes.data_as(C.c_void_p)  # noqa: E731
    L.drgo_similarity_rows(n, rp, col, int(k), float(sigma), len(src), src, out_rp, ptr(out_col),
                           ptr(out_hop), ptr(out_P), ptr(invZ), ptr(qt), ptr(W))
    return {"row_ptr": out_rp, "col": out_col[:nnz], "hop": out_hop[:nnz], "P": out_P[:nnz],
            "invZ": invZ, "qt": qt, "W": W}


def draw(sim: Sim, w: int) -> int:
    return int(lib().drgo_draw(sim.C, sim.n, C.c_uint64(int(w))))


def neg_word(seed: int, it: int, i: int, m: int) -> int:
    return int(lib().drgo_neg_word(seed, it, i, m))


def coarsen_level(csr, seed: int, level: int):
    n = int(csr.n)
    m = np.zeros(max(n, 1), np.int32)
    nc = lib().drgo_coarsen_level(n, _c(csr.row_ptr, np.int32), _c(csr.col, np.int32),
                                  int(seed), int(level), m)
    return m[:n], int(nc)


def contract(csr, cmap, nc):
    from types import SimpleNamespace
    rp = np.zeros(nc + 1, np.int32)
    oc = np.zeros(max(int(csr.row_ptr[-1]), 1), np.int32)
    nnz = lib().drgo_contract(int(csr.n), _c(csr.row_ptr, np.int32), _c(csr.col, np.int32),
                              _c(cmap, np.int32), int(nc), rp, oc)
    return SimpleNamespace(n=int(nc), row_ptr=rp, col=oc[:nnz].copy())


def n_active_csr(csr) -> int:
    return int(np.count_nonzero(np.diff(np.asarray(csr.row_ptr, np.int64))))


@dataclass
class Hier:
    """G^0..G^L: one-level maps maps[l]: V^l -> V^{l+1} and composed maps
    cmaps[l]: V^0 -> V^l (cmaps[0] is the identity)."""
    graphs: list
    maps: list = field(default_factory=list)
    cmaps: list = field(default_factory=list)

    @property
    def levels(self) -> int:
        return len(self.graphs)

    @property
    def sizes(self):
        return [int(g.n) for g in self.graphs]


def hierarchy(csr, seed: int = 0, rho: float = 0.8, min_nodes: int = 1000,
              max_levels: int = 64) -> Hier:
    """Coarsen until |V^{l+1}| > rho |V^l| (counting non-isolated nodes; the
    level that fails the test is discarded), until fewer than min_nodes
    non-isolated nodes remain, or until max_levels levels exist (Sec. 3.2.3)."""
    graphs = [csr]
    maps = []
    cm = [np.arange(csr.n, dtype=np.int32)]
    while len(graphs) < max_levels:
        g = graphs[-1]
        na = n_active_csr(g)
        if na == 0 or na < min_nodes:
            break
        m, nc = coarsen_level(g, seed, len(graphs) - 1)
        gc = contract(g, m, nc)
        if n_active_csr(gc) > rho * na:
            break
        graphs.append(gc)
        maps.append(m)
        cm.append(m[cm[-1]])
    return Hier(graphs, maps, cm)


def init(nl: int, seed: int, level: int, dim: int = 2) -> np.ndarray:
    """Coarsest-level layout, [nl, dim] (dim 2 or 3, Sec. 3.1)."""
    y = np.zeros(dim * max(nl, 1), np.float64)
    lib().drgo_init(int(nl), int(seed), int(level), y, int(dim))
    return y[: dim * nl].reshape(nl, dim)


def _cm_ptr(cmap):
    if cmap is None:
        return None, None
    a = _c(cmap, np.int32)
    return a, a.ctypes.data_as(C.c_void_p)


def _b(b) -> float:
    """The proximity shape b as the oracle takes it: a whole or half number."""
    v = float(b)
    if v * 2 != int(v * 2) or not (1.0 <= v <= 3.0):
        raise ValueError("b must be 1, 1.5, 2, 2.5 or 3")
    return v


def _dim(y) -> int:
    d = int(np.shape(y)[1])
    if d not in (2, 3):
        raise ValueError("coordinates must be [n, 2] or [n, 3]")
    return d


def step_direction(sim: Sim, y, cmap=None, M=5, b=1, gamma=0.1, clip=math.inf, seed=0, it=0):
    keep, p = _cm_ptr(cmap)
    d = _dim(y)
    g = np.zeros(d * sim.n, np.float64)
    yy = _c(y, np.float64).ravel()
    lib().drgo_step_direction(sim.n, sim.row_ptr, _pcol(sim), _pP(sim), sim.qt, sim.C, p, yy,
                              int(M), _b(b), float(gamma), float(clip), int(seed), int(it), g, d)
    return g.reshape(sim.n, d)


def _pcol(sim):
    return sim.col if sim.nnz else np.zeros(1, np.int32)


def _pP(sim):
    return sim.P if sim.nnz else np.zeros(1, np.float64)


def iter_sync(sim: Sim, y, cmap=None, M=5, b=1, gamma=0.1, eta=1.0, clip=4.0, seed=0, it=0,
              seq=False):
    """One iteration in place on y (level coordinates [nl, 2])."""
    keep, p = _cm_ptr(cmap)
    nl = y.shape[0]
    d = _dim(y)
    yy = np.ascontiguousarray(y, dtype=np.float64).reshape(-1)
    fn = lib().drgo_iter_seq if seq else lib().drgo_iter_sync
    fn(sim.n, sim.row_ptr, _pcol(sim), _pP(sim), sim.qt, sim.C, p, nl, yy, int(M), _b(b),
       float(gamma), float(eta), float(clip), int(seed), int(it), d)
    y[...] = yy.reshape(nl, d)
    return y


def objective(sim, y, M=5, b=1, gamma=0.1, seed=0, it=0) -> float:
    return float(lib().drgo_objective(sim.n, sim.row_ptr, _pcol(sim), _pP(sim), sim.qt, sim.C,
                                      _c(y, np.float64).ravel(), int(M), _b(b), float(gamma),
                                      int(seed), int(it), _dim(y)))


def objective_grad(sim, y, M=5, b=1, gamma=0.1, seed=0, it=0) -> np.ndarray:
    d = _dim(y)
    g = np.zeros(d * sim.n, np.float64)
    lib().drgo_objective_grad(sim.n, sim.row_ptr, _pcol(sim), _pP(sim), sim.qt, sim.C,
                              _c(y, np.float64).ravel(), int(M), _b(b), float(gamma),
                              int(seed), int(it), g, d)
    return g.reshape(sim.n, d)


def objective_exact(sim, y, M=5, b=1, gamma=0.1) -> float:
    return float(lib().drgo_objective_exact(sim.n, sim.row_ptr, _pcol(sim), _pP(sim), sim.qt,
                                            sim.C, _c(y, np.float64).ravel(), int(M), _b(b),
                                            float(gamma), _dim(y)))


def objective_exact_grad(sim, y, M=5, b=1, gamma=0.1) -> np.ndarray:
    d = _dim(y)
    g = np.zeros(d * sim.n, np.float64)
    lib().drgo_objective_exact_grad(sim.n, sim.row_ptr, _pcol(sim), _pP(sim), sim.qt, sim.C,
                                    _c(y, np.float64).ravel(), int(M), _b(b), float(gamma), g, d)
    return g.reshape(sim.n, d)


def step_expected(sim, y, M=5, b=1, gamma=0.1) -> np.ndarray:
    d = _dim(y)
    g = np.zeros(d * sim.n, np.float64)
    lib().drgo_step_expected(sim.n, sim.row_ptr, _pcol(sim), _pP(sim), sim.qt, sim.C,
                             _c(y, np.float64).ravel(), int(M), _b(b), float(gamma), g, d)
    return g.reshape(sim.n, d)


# ------------------------------------------------------------- full layout
def schedule(T: int, levels: int, gamma: float = 0.1, gamma_coarsest: float = 0.01):
    """Per level (coarsest first): (level, T_l, gamma_l).  T is the total
    iteration count split evenly over levels, the finest level taking the
    remainder; the coarsest level uses the smaller repulsion weight when
    there is more than one level (Sec. 4.2, weight of negative samples)."""
    out = []
    base = T // levels
    for l in range(levels - 1, -1, -1):
        Tl = base + (T - base * levels if l == 0 else 0)
        g = gamma_coarsest if (l == levels - 1 and levels > 1) else gamma
        out.append((l, Tl, g))
    return out


def eta_at(eta0: float, t: int, Tl: int) -> float:
    return eta0 * (1.0 - t / Tl)


def layout(csr, k=1, sigma=1.0, M=5, b=1, gamma=0.1, gamma_coarsest=0.01, T=400, eta0=1.0,
           clip=4.0, rho=0.8, min_nodes=1000, max_levels=64, seed=0, mode="sync",
           sim: Sim | None = None, hier: Hier | None = None, return_all=False, dim=2,
           perplexity=0.0, lengths=None):
    """Full multilevel layout; returns Y^0 [n, dim] (float64).  perplexity >
    0 takes node-wise sigma_i calibrated to it instead of sigma; lengths
    (one per CSR entry) takes the weighted similarity."""
    if sim is None:
        if lengths is not None:
            sim = similarity_weighted(csr, lengths, k, sigma)
        elif perplexity > 0:
            sim = similarity_perplexity(csr, k, perplexity)
        else:
            sim = similarity(csr, k, sigma)
    if hier is None:
        hier = hierarchy(csr, seed, rho, min_nodes, max_levels)
    Lc = hier.levels
    y = init(hier.sizes[-1], seed, Lc - 1, dim)
    gi = 0
    for (l, Tl, g) in schedule(T, Lc, gamma, gamma_coarsest):
        cmap = None if l == 0 else hier.cmaps[l]
        for t in range(Tl):
            iter_sync(sim, y, cmap, M, b, g, eta_at(eta0, t, Tl), clip, seed, gi,
                      seq=(mode == "seq"))
            gi += 1
        if l > 0:
            y = y[hier.maps[l - 1]].copy()
    if return_all:
        return y, sim, hier
    return y
