"""Python binding of libdrgraph.so (argument marshalling only).

Functions carry the names of the C entry points in include/drgraph.h.  Device
arrays are torch tensors on the GPU; every step of the layout runs in the
library's HIP kernels.  Importing works without a GPU; calling a function
that needs the library raises if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libdrgraph.so")

DRG_OK = 0
DRG_E_INVALID = -1
DRG_E_GRAPH = -2
DRG_E_OOM = -3
DRG_E_DEVICE = -4
DRG_E_UNSUPPORTED = -5
DRG_VALIDATE = 1
DRG_MODE_SYNC = 0
DRG_MODE_ASYNC = 1
DRG_SWEEP_ROW = 0
DRG_SWEEP_WINDOW = 1
DRG_SWEEP_BLOCKED = 2
DRG_SWEEP_ROW_ASYNC = 3
DRG_SWEEP_BLOCKED_ASYNC = 4


class DrgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"drgraph status {status}: {msg}")
        self.status = status


class Csr(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int32), ("row_ptr", C.c_void_p),
                ("col", C.c_void_p)]


class StepParams(C.Structure):
    _fields_ = [("M", C.c_int32), ("b", C.c_int32), ("gamma", C.c_float), ("eta", C.c_float),
                ("clip", C.c_float), ("level", C.c_int32), ("mode", C.c_int32),
                ("dim", C.c_int32), ("seed", C.c_uint64), ("iter", C.c_uint64),
                ("b_half", C.c_int32), ("_pad", C.c_int32)]


class ObjParams(C.Structure):
    _fields_ = [("M", C.c_int32), ("b", C.c_int32), ("gamma", C.c_double), ("seed", C.c_uint64),
                ("iter", C.c_uint64), ("dim", C.c_int32), ("b_half", C.c_int32)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


class LayoutParams(C.Structure):
    _fields_ = [("k", C.c_int32), ("M", C.c_int32), ("b", C.c_int32), ("T", C.c_int32),
                ("sigma", C.c_double), ("gamma", C.c_float), ("gamma_coarsest", C.c_float),
                ("eta0", C.c_float), ("clip", C.c_float), ("rho", C.c_double),
                ("min_nodes", C.c_int32), ("max_levels", C.c_int32), ("mode", C.c_int32),
                ("dim", C.c_int32), ("seed", C.c_uint64), ("b_half", C.c_int32),
                ("_pad", C.c_int32), ("perplexity", C.c_double)]


def _shape(b):
    """(whole part, half flag) of the shape parameter b: 1, 1.5, 2, 2.5 or 3."""
    twice = float(b) * 2.0
    if twice != int(twice) or not 2 <= twice <= 6:
        raise ValueError(f"b must be 1, 1.5, 2, 2.5 or 3, not {b}")
    return int(twice) // 2, int(twice) % 2


_lib = None
_P = C.c_void_p


def lib():
    """The loaded library; raises when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libdrgraph.so not built ({LIB_PATH}); run "
                           "python -m paper_2008_07799_amd.build")
    # torch ships its own HIP runtime; loading it first makes the library bind
    # to that same runtime (one runtime per process, shared streams and
    # pointers) instead of bringing in a second one, which then finds no device
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    st = C.c_int32
    sig = {
        "drg_last_error": ([], C.c_char_p),
        "drg_version": ([], C.c_char_p),
        "drg_layout_params_default": ([C.POINTER(LayoutParams)], st),
        "drg_ctx_create": ([C.c_int32, _P, C.POINTER(Allocator), C.POINTER(_P)], st),
        "drg_ctx_destroy": ([_P], None),
        "drg_ctx_synchronize": ([_P], st),
        "drg_ctx_set_profiling": ([_P, C.c_int32], st),
        "drg_ctx_kernel_stats": ([_P, C.POINTER(C.c_int64), C.POINTER(C.c_double)], st),
        "drg_ctx_last_sweep": ([_P, C.POINTER(C.c_int32)], st),
        "drg_build_similarity_perplexity": ([_P, C.POINTER(Csr), C.c_int32, C.c_double,
                                             C.c_uint32, C.POINTER(_P)], st),
        "drg_sim_node_sigma": ([_P, _P], st),
        "drg_build_similarity_weighted": ([_P, C.POINTER(Csr), _P, C.c_int32, C.c_double,
                                           C.c_uint32, C.POINTER(_P)], st),
        "drg_build_similarity": ([_P, C.POINTER(Csr), C.c_int32, C.c_double, C.c_uint32,
                                  C.POINTER(_P)], st),
        "drg_sim_info": ([_P, C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                          C.POINTER(C.c_int32), C.POINTER(C.c_int32)], st),
        "drg_sim_export": ([_P] + [_P] * 8, st),
        "drg_sim_export_rows": ([_P, C.c_int32, _P, C.c_int64] + [_P] * 7, st),
        "drg_neighbourhood_preservation": ([_P, _P, _P, C.c_int32, _P, _P], st),
        "drg_stress_sampled": ([_P, C.POINTER(Csr), _P, C.c_int32, _P, _P,
                                C.POINTER(C.c_double)], st),
        "drg_sim_destroy": ([_P], None),
        "drg_coarsen": ([_P, C.POINTER(Csr), C.c_uint64, C.c_double, C.c_int32, C.c_int32,
                         C.POINTER(_P)], st),
        "drg_hier_info": ([_P, C.POINTER(C.c_int32), _P], st),
        "drg_hier_export": ([_P, C.c_int32, _P, _P, _P, _P, C.POINTER(C.c_int64)], st),
        "drg_hier_export_map": ([_P, C.c_int32, _P], st),
        "drg_hier_destroy": ([_P], None),
        "drg_init_layout": ([_P, C.c_int32, C.c_uint64, C.c_int32, _P], st),
        "drg_prolong": ([_P, _P, C.c_int32, _P, _P], st),
        "drg_layout_step": ([_P, _P, _P, C.POINTER(StepParams), _P], st),
        "drg_init_layout_f64": ([_P, C.c_int32, C.c_uint64, C.c_int32, _P], st),
        "drg_init_layout_3d": ([_P, C.c_int32, C.c_uint64, C.c_int32, _P], st),
        "drg_init_layout_3d_f64": ([_P, C.c_int32, C.c_uint64, C.c_int32, _P], st),
        "drg_prolong_3d": ([_P, _P, C.c_int32, _P, _P], st),
        "drg_prolong_3d_f64": ([_P, _P, C.c_int32, _P, _P], st),
        "drg_prolong_f64": ([_P, _P, C.c_int32, _P, _P], st),
        "drg_layout_step_f64": ([_P, _P, _P, C.POINTER(StepParams), _P], st),
        "drg_layout_run": ([_P, _P, _P, C.POINTER(LayoutParams), _P], st),
        "drg_layout_run_until": ([_P, _P, _P, C.POINTER(LayoutParams), C.c_int32, C.c_int32,
                                  _P], st),
        "drg_layout_resume": ([_P, _P, _P, C.POINTER(LayoutParams), C.c_int32, C.c_int32, _P,
                               _P], st),
        "drg_objective_fwd": ([_P, _P, C.POINTER(ObjParams), _P, _P, _P], st),
        "drg_objective_bwd": ([_P, _P, C.POINTER(ObjParams), _P, _P, _P], st),
        "drg_objective_fwd_noalloc": ([_P, _P, C.POINTER(ObjParams), _P, _P], st),
        "drg_objective_fwd_f64": ([_P, _P, C.POINTER(ObjParams), _P, _P, _P], st),
        "drg_objective_bwd_f64": ([_P, _P, C.POINTER(ObjParams), _P, _P, _P], st),
        "drg_sample_negatives": ([_P, _P, C.c_int32, C.c_uint64, C.c_uint64, _P], st),
        "drg_sim_coo": ([_P, _P, _P, _P, _P], st),
        "drg_layout": ([_P, C.POINTER(Csr), C.POINTER(LayoutParams), _P], st),
        "drg_batch_create": ([_P, C.POINTER(Csr), C.c_int32, C.POINTER(LayoutParams),
                              C.POINTER(_P)], st),
        "drg_batch_info": ([_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                            C.POINTER(C.c_int32), _P, _P], st),
        "drg_batch_run": ([_P, _P, _P], st),
        "drg_batch_tuning": ([_P, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32), _P, _P,
                              _P], st),
        "drg_batch_destroy": ([_P], None),
        "drg_layout_batched": ([_P, C.POINTER(Csr), C.c_int32, C.POINTER(LayoutParams), _P], st),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(status: int):
    if status != DRG_OK:
        raise DrgError(status, lib().drg_last_error().decode(errors="replace"))


def _dev(t, dtype, name, shape=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return C.c_void_p(t.data_ptr())


def _np_ptr(a):
    return C.c_void_p(a.ctypes.data) if a is not None else None


# ------------------------------------------------------------------ context
class Context:
    """A library context on `device`; `allocator` (optional) is a drgraph
    Allocator structure whose callbacks provide all device memory of the
    objects built through this context (it must outlive them)."""

    def __init__(self, device: int = 0, stream=None, allocator: Allocator | None = None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.device = device
        self.stream = stream
        self.allocator = allocator
        h = C.c_void_p()
        _check(lib().drg_ctx_create(device, C.c_void_p(stream.cuda_stream),
                                    C.byref(allocator) if allocator is not None else None,
                                    C.byref(h)))
        self._free = lib().drg_ctx_destroy  # kept: module globals are gone at exit
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self._free(self.h)
            self.h = None

    __del__ = close

    def synchronize(self):
        _check(lib().drg_ctx_synchronize(self.h))

    def set_profiling(self, on: bool):
        _check(lib().drg_ctx_set_profiling(self.h, 1 if on else 0))

    def kernel_stats(self):
        n = C.c_int64()
        ms = C.c_double()
        _check(lib().drg_ctx_kernel_stats(self.h, C.byref(n), C.byref(ms)))
        return int(n.value), float(ms.value)

    def last_sweep(self) -> int:
        """DRG_SWEEP_* form launched by the latest layout step (-1: none yet)."""
        f = C.c_int32()
        _check(lib().drg_ctx_last_sweep(self.h, C.byref(f)))
        return int(f.value)


def _csr(row_ptr, col) -> Csr:
    import torch
    n = row_ptr.numel() - 1
    nnz = col.numel()
    return Csr(n, nnz, _dev(row_ptr, torch.int32, "row_ptr").value,
               _dev(col, torch.int32, "col").value if nnz else None)


def to_device(csr, device="cuda"):
    """gen.CSR -> (row_ptr, col) int32 tensors on the GPU."""
    import torch
    rp = torch.from_numpy(np.ascontiguousarray(csr.row_ptr, np.int32)).to(device)
    col = torch.from_numpy(np.ascontiguousarray(csr.col, np.int32)).to(device)
    return rp, col


# ------------------------------------------------------------------ similarity
class Similarity:
    def __init__(self, h):
        self._free = lib().drg_sim_destroy
        self.h = h
        n = C.c_int32()
        nnz = C.c_int64()
        na = C.c_int32()
        k = C.c_int32()
        blk = C.c_int32()
        _check(lib().drg_sim_info(h, C.byref(n), C.byref(nnz), C.byref(na), C.byref(k),
                                  C.byref(blk)))
        self.n, self.nnz, self.n_active, self.k = n.value, nnz.value, na.value, k.value
        self.blocked = bool(blk.value)

    def close(self):
        if getattr(self, "h", None):
            self._free(self.h)
            self.h = None

    __del__ = close

    def node_sigma(self) -> np.ndarray:
        """sigma_i per node (host float64): the global sigma, or the
        calibrated one of a node-wise similarity (inf where uniform); 0 for
        isolated nodes."""
        out = np.zeros(self.n, np.float64)
        _check(lib().drg_sim_node_sigma(self.h, _np_ptr(out)))
        return out

    def export(self, values: bool = True, pattern: bool = True) -> dict:
        """The whole similarity as host numpy arrays; pattern=False leaves out
        the per-entry arrays (columns, hops, values) and copies the per-node
        ones only."""
        n, nnz, k = self.n, self.nnz, self.k
        m = max(nnz, 1) if pattern else 0
        out = {"row_ptr": np.zeros(n + 1, np.int64),
               "col": np.zeros(m, np.int32) if pattern else None,
               "hop": np.zeros(m, np.uint8) if pattern else None, "qt": np.zeros(n, np.float64),
               "W": np.zeros(n, np.uint64), "e": np.zeros(max(k, 1), np.float64),
               "invZ": np.zeros(n, np.float64)}
        out["P"] = np.zeros(m, np.float64) if values and pattern else None
        _check(lib().drg_sim_export(self.h, _np_ptr(out["row_ptr"]), _np_ptr(out["col"]),
                                    _np_ptr(out["hop"]), _np_ptr(out["P"]), _np_ptr(out["qt"]),
                                    _np_ptr(out["W"]), _np_ptr(out["e"]),
                                    _np_ptr(out["invZ"])))
        if pattern:
            out["col"] = out["col"][:nnz]
            out["hop"] = out["hop"][:nnz]
            if values:
                out["P"] = out["P"][:nnz]
        out["e"] = out["e"][:k]
        return out

    def export_rows(self, rows, values: bool = True) -> dict:
        """Rows `rows` only (host numpy): per-row lengths, then the rows'
        columns, hops and (with values) FP64 P~ one after another; qt, W, invZ of
        the rows."""
        r = np.ascontiguousarray(rows, np.int32)
        m = len(r)
        lens = np.zeros(max(m, 1), np.int64)
        _check(lib().drg_sim_export_rows(self.h, m, _np_ptr(r), 0, _np_ptr(lens), None, None,
                                         None, None, None, None))
        tot = int(lens[:m].sum())
        out = {"row_len": lens[:m], "col": np.zeros(max(tot, 1), np.int32),
               "hop": np.zeros(max(tot, 1), np.uint8),
               "P": np.zeros(max(tot, 1), np.float64) if values else None,
               "qt": np.zeros(max(m, 1), np.float64), "W": np.zeros(max(m, 1), np.uint64),
               "invZ": np.zeros(max(m, 1), np.float64)}
        _check(lib().drg_sim_export_rows(self.h, m, _np_ptr(r), tot, _np_ptr(lens),
                                         _np_ptr(out["col"]), _np_ptr(out["hop"]), _np_ptr(out["P"]),
                                         _np_ptr(out["qt"]), _np_ptr(out["W"]),
                                         _np_ptr(out["invZ"])))
        out["col"] = out["col"][:tot]
        out["hop"] = out["hop"][:tot]
        if values:
            out["P"] = out["P"][:tot]
        for key in ("qt", "W", "invZ"):
            out[key] = out[key][:m]
        return out


def drg_build_similarity(ctx: Context, row_ptr, col, k: int, sigma: float = 1.0,
                         validate: bool = False) -> Similarity:
    g = _csr(row_ptr, col)
    h = C.c_void_p()
    _check(lib().drg_build_similarity(ctx.h, C.byref(g), int(k), float(sigma),
                                      DRG_VALIDATE if validate else 0, C.byref(h)))
    return Similarity(h)


def drg_build_similarity_perplexity(ctx: Context, row_ptr, col, k: int, perplexity: float,
                                    validate: bool = False) -> Similarity:
    """P~ with one sigma_i per node calibrated to `perplexity` (Eq. NS)."""
    g = _csr(row_ptr, col)
    h = C.c_void_p()
    _check(lib().drg_build_similarity_perplexity(ctx.h, C.byref(g), int(k), float(perplexity),
                                                 DRG_VALIDATE if validate else 0, C.byref(h)))
    return Similarity(h)


def drg_build_similarity_weighted(ctx: Context, row_ptr, col, lengths, k: int,
                                  sigma: float = 1.0) -> Similarity:
    """P~ of a weighted graph: lengths = one positive length per CSR entry
    (float64 device tensor, symmetric); GD = shortest path of at most k
    edges (Eq. NS with weighted graph distances)."""
    import torch
    g = _csr(row_ptr, col)
    lp = _dev(lengths, torch.float64, "lengths", (int(col.numel()),))
    h = C.c_void_p()
    _check(lib().drg_build_similarity_weighted(ctx.h, C.byref(g), lp, int(k), float(sigma), 0,
                                               C.byref(h)))
    return Similarity(h)


def drg_neighbourhood_preservation(ctx: Context, sim: Similarity, y, nodes):
    """NP of `nodes` (Sec. 4.1, Eq. NP) for the layout y [n, 2] (FP32, device),
    with graph neighbourhoods = the rows of `sim`: a float64 device tensor,
    -1 where a node has no neighbourhood."""
    import torch
    yp = _dev(y, torch.float32, "y", (sim.n, 2))
    np_ = _dev(nodes, torch.int32, "nodes")
    out = torch.empty(nodes.numel(), dtype=torch.float64, device=y.device)
    _check(lib().drg_neighbourhood_preservation(ctx.h, sim.h, yp, int(nodes.numel()), np_,
                                                C.c_void_p(out.data_ptr())))
    ctx.synchronize()
    return out


def drg_stress_sampled(ctx: Context, row_ptr, col, y, sources):
    """Per-source stress sums (A, B, P) (Sec. 4.1; see drgraph.h) as a
    [count, 3] float64 device tensor, and the library's sampled stress
    estimate."""
    import torch
    g = _csr(row_ptr, col)
    yp = _dev(y, torch.float32, "y", (g.n, 2))
    sp = _dev(sources, torch.int32, "sources")
    out = torch.empty((sources.numel(), 3), dtype=torch.float64, device=y.device)
    est = C.c_double()
    _check(lib().drg_stress_sampled(ctx.h, C.byref(g), yp, int(sources.numel()), sp,
                                    C.c_void_p(out.data_ptr()), C.byref(est)))
    return out, float(est.value)


# ------------------------------------------------------------------ hierarchy
class Hierarchy:
    def __init__(self, h):
        self._free = lib().drg_hier_destroy
        self.h = h
        lv = C.c_int32()
        _check(lib().drg_hier_info(h, C.byref(lv), None))
        self.levels = lv.value
        sizes = np.zeros(self.levels, np.int32)
        _check(lib().drg_hier_info(h, C.byref(lv), _np_ptr(sizes)))
        self.sizes = [int(x) for x in sizes]

    def close(self):
        if getattr(self, "h", None):
            self._free(self.h)
            self.h = None

    __del__ = close

    def export(self, level: int, n0: int) -> dict:
        nf = self.sizes[level - 1]
        nl = self.sizes[level]
        nnz = C.c_int64()
        _check(lib().drg_hier_export(self.h, level, None, None, None, None, C.byref(nnz)))
        out = {"map": np.zeros(nf, np.int32), "cmap": np.zeros(n0, np.int32),
               "row_ptr": np.zeros(nl + 1, np.int32), "col": np.zeros(max(nnz.value, 1), np.int32)}
        _check(lib().drg_hier_export(self.h, level, _np_ptr(out["map"]), _np_ptr(out["cmap"]),
                                     _np_ptr(out["row_ptr"]), _np_ptr(out["col"]), C.byref(nnz)))
        out["col"] = out["col"][: nnz.value]
        return out

    def export_map(self, level: int, n0: int) -> np.ndarray:
        """Finest node -> node of `level` (host int32 [n0])."""
        out = np.zeros(n0, np.int32)
        _check(lib().drg_hier_export_map(self.h, level, _np_ptr(out)))
        return out


def drg_coarsen(ctx: Context, row_ptr, col, seed: int = 0, rho: float = 0.8,
                min_nodes: int = 1000, max_levels: int = 64) -> Hierarchy:
    g = _csr(row_ptr, col)
    h = C.c_void_p()
    _check(lib().drg_coarsen(ctx.h, C.byref(g), int(seed), float(rho), int(min_nodes),
                             int(max_levels), C.byref(h)))
    return Hierarchy(h)


# ------------------------------------------------------------------ layout
def _coords(y, name, shape):
    """float32 -> the product entry point, float64 -> its FP64 instance."""
    import torch
    if isinstance(y, torch.Tensor) and y.dtype == torch.float64:
        return _dev(y, torch.float64, name, shape), True
    return _dev(y, torch.float32, name, shape), False


def _dim(y) -> int:
    """Coordinate dimension of a [n, 2] or [n, 3] tensor (Sec. 3.1)."""
    d = int(y.shape[1]) if y.dim() == 2 else 0
    if d not in (2, 3):
        raise ValueError("coordinates must be [n, 2] or [n, 3]")
    return d


def drg_init_layout(ctx: Context, n: int, seed: int, level: int, y):
    """Random layout of a level into y [n, 2] or [n, 3]."""
    d = _dim(y)
    ptr, f64 = _coords(y, "y", (n, d))
    if d == 3:
        fn = lib().drg_init_layout_3d_f64 if f64 else lib().drg_init_layout_3d
    else:
        fn = lib().drg_init_layout_f64 if f64 else lib().drg_init_layout
    _check(fn(ctx.h, int(n), int(seed), int(level), ptr))


def drg_prolong(ctx: Context, hier: Hierarchy, level: int, y_level, y_finer):
    d = _dim(y_level)
    a, f64 = _coords(y_level, "y_level", (hier.sizes[level], d))
    b, f64b = _coords(y_finer, "y_finer", (hier.sizes[level - 1], d))
    if f64 != f64b:
        raise TypeError("y_level and y_finer must have the same dtype")
    if d == 3:
        fn = lib().drg_prolong_3d_f64 if f64 else lib().drg_prolong_3d
    else:
        fn = lib().drg_prolong_f64 if f64 else lib().drg_prolong
    _check(fn(ctx.h, hier.h, int(level), a, b))


def drg_layout_step(ctx: Context, sim: Similarity, hier, y, *, M=5, b=1, gamma=0.1, eta=1.0,
                    clip=4.0, level=0, mode=DRG_MODE_SYNC, seed=0, iter=0):
    nl = sim.n if level == 0 else hier.sizes[level]
    d = _dim(y)
    bw, bh = _shape(b)
    p = StepParams(int(M), bw, float(gamma), float(eta), float(clip), int(level), int(mode),
                   d, int(seed), int(iter), bh)
    ptr, f64 = _coords(y, "y", (nl, d))
    fn = lib().drg_layout_step_f64 if f64 else lib().drg_layout_step
    _check(fn(ctx.h, sim.h, hier.h if hier is not None else None, C.byref(p), ptr))


def layout_params(**kw) -> LayoutParams:
    """Defaults with keyword overrides; b may be 1, 1.5, 2, 2.5 or 3."""
    p = LayoutParams()
    _check(lib().drg_layout_params_default(C.byref(p)))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        if k == "b":
            p.b, p.b_half = _shape(v)
        else:
            setattr(p, k, v)
    return p


def _pdim(params: LayoutParams) -> int:
    return 3 if params.dim == 3 else 2


def drg_layout_run(ctx: Context, sim: Similarity, hier: Hierarchy, params: LayoutParams, y_out):
    """The whole schedule; y_out [n, 2] (or [n, 3] with params.dim = 3)."""
    import torch
    _check(lib().drg_layout_run(ctx.h, sim.h, hier.h, C.byref(params),
                                _dev(y_out, torch.float32, "y_out", (sim.n, _pdim(params)))))


def drg_layout_run_until(ctx: Context, sim: Similarity, hier: Hierarchy, params: LayoutParams,
                         level: int, t: int, y_level):
    """Runs the schedule until t iterations of `level` are done; writes that
    level's coordinates into y_level [n_level, dim] (float32, device)."""
    import torch
    _check(lib().drg_layout_run_until(ctx.h, sim.h, hier.h, C.byref(params), int(level), int(t),
                                      _dev(y_level, torch.float32, "y_level",
                                           (hier.sizes[level], _pdim(params)))))


def drg_layout_resume(ctx: Context, sim: Similarity, hier: Hierarchy, params: LayoutParams,
                      level: int, t: int, y_level, y_out):
    """Continues the schedule from (level, t, y_level) to the end; finest
    coordinates into y_out [n, dim]."""
    import torch
    d = _pdim(params)
    _check(lib().drg_layout_resume(ctx.h, sim.h, hier.h, C.byref(params), int(level), int(t),
                                   _dev(y_level, torch.float32, "y_level",
                                        (hier.sizes[level], d)),
                                   _dev(y_out, torch.float32, "y_out", (sim.n, d))))


def drg_layout(ctx: Context, row_ptr, col, params: LayoutParams, y_out):
    """End to end; y_out [n, 2] (or [n, 3] with params.dim = 3)."""
    import torch
    g = _csr(row_ptr, col)
    _check(lib().drg_layout(ctx.h, C.byref(g), C.byref(params),
                            _dev(y_out, torch.float32, "y_out", (g.n, _pdim(params)))))


# ------------------------------------------------------------------ batches
def _batch_args(graphs, params):
    """graphs: list of (row_ptr, col) device int32 tensors; params: one
    LayoutParams for all or a list of them."""
    if isinstance(params, LayoutParams):
        params = [params] * len(graphs)
    if len(params) != len(graphs) or not graphs:
        raise ValueError("need one LayoutParams per graph and at least one graph")
    ga = (Csr * len(graphs))(*[_csr(rp, col) for rp, col in graphs])
    pa = (LayoutParams * len(graphs))(*params)
    return ga, pa


class Batch:
    """A recorded batched run (drg_batch_create); run() replays it."""

    def __init__(self, ctx: Context, graphs, params):
        ga, pa = _batch_args(graphs, params)
        self.count = len(graphs)
        h = C.c_void_p()
        _check(lib().drg_batch_create(ctx.h, ga, self.count, pa, C.byref(h)))
        self._free = lib().drg_batch_destroy
        self.h = h
        n = C.c_int64()
        nnz = C.c_int64()
        T = C.c_int32()
        nodes = np.zeros(self.count, np.int32)
        levels = np.zeros(self.count, np.int32)
        _check(lib().drg_batch_info(h, C.byref(n), C.byref(nnz), C.byref(T), _np_ptr(nodes),
                                    _np_ptr(levels)))
        self.n_total, self.nnz, self.T = n.value, nnz.value, T.value
        self.nodes = [int(x) for x in nodes]
        self.levels = [int(x) for x in levels]
        self.base = np.concatenate([[0], np.cumsum(nodes, dtype=np.int64)])

    def tuning(self) -> dict:
        """Sweep forms timed at creation: list of (rows per group or 0 for the
        row form, LDS chunk, ms) and the index in use."""
        n = C.c_int32()
        ch = C.c_int32()
        _check(lib().drg_batch_tuning(self.h, 0, C.byref(n), C.byref(ch), None, None, None))
        rpl = np.zeros(max(n.value, 1), np.int32)
        chunk = np.zeros(max(n.value, 1), np.int32)
        ms = np.zeros(max(n.value, 1), np.float32)
        _check(lib().drg_batch_tuning(self.h, n.value, C.byref(n), C.byref(ch), _np_ptr(rpl),
                                      _np_ptr(chunk), _np_ptr(ms)))
        return {"candidates": [(int(rpl[i]), int(chunk[i]), float(ms[i])) for i in range(n.value)],
                "chosen": ch.value}

    def run(self, ctx: Context, y_out):
        import torch
        _check(lib().drg_batch_run(ctx.h, self.h,
                                   _dev(y_out, torch.float32, "y_out", (self.n_total, 2))))

    def close(self):
        if getattr(self, "h", None):
            self._free(self.h)
            self.h = None

    __del__ = close


def drg_batch_create(ctx: Context, graphs, params) -> Batch:
    return Batch(ctx, graphs, params)


def drg_layout_batched(ctx: Context, graphs, params, y_out):
    import torch
    ga, pa = _batch_args(graphs, params)
    n = sum(int(rp.numel()) - 1 for rp, _ in graphs)
    _check(lib().drg_layout_batched(ctx.h, ga, len(graphs), pa,
                                    _dev(y_out, torch.float32, "y_out", (n, 2))))


# ------------------------------------------------------------------ objective
def _obj_params(M, b, gamma, seed, iter, d) -> ObjParams:
    bw, bh = _shape(b)
    return ObjParams(int(M), bw, float(gamma), int(seed), int(iter), d, bh)


def drg_objective_fwd(ctx: Context, sim: Similarity, y, *, M=5, b=1, gamma=0.1, seed=0, iter=0,
                      rows=False):
    """The sampled objective L^ at y ([n,2], float32 or float64).  Returns a
    0-d tensor, or with rows=True the per-row values [n]."""
    import torch
    d = _dim(y)
    ptr, f64 = _coords(y, "y", (sim.n, d))
    p = _obj_params(M, b, gamma, seed, iter, d)
    out = torch.empty((sim.n,) if rows else (), dtype=y.dtype, device=y.device)
    fn = lib().drg_objective_fwd_f64 if f64 else lib().drg_objective_fwd
    optr = C.c_void_p(out.data_ptr())
    _check(fn(ctx.h, sim.h, C.byref(p), ptr, None if rows else optr, optr if rows else None))
    return out


def drg_objective_fwd_noalloc(ctx: Context, sim: Similarity, y, loss, *, M=5, b=1, gamma=0.1,
                              seed=0, iter=0):
    """The FP32 loss of drg_objective_fwd written into the caller's 0-d float32
    device tensor `loss`, with no allocation in the library (static scratch,
    at most 2^20 nodes); enqueued only: synchronise before reading it."""
    import torch
    d = _dim(y)
    yp = _dev(y, torch.float32, "y", (sim.n, d))
    lp = _dev(loss, torch.float32, "loss", ())
    p = _obj_params(M, b, gamma, seed, iter, d)
    _check(lib().drg_objective_fwd_noalloc(ctx.h, sim.h, C.byref(p), yp, lp))


def drg_objective_bwd(ctx: Context, sim: Similarity, y, dloss=None, *, M=5, b=1, gamma=0.1,
                      seed=0, iter=0):
    """dloss * dL^/dy as a tensor like y; dloss is a 0-d device tensor or None."""
    import torch
    d = _dim(y)
    ptr, f64 = _coords(y, "y", (sim.n, d))
    p = _obj_params(M, b, gamma, seed, iter, d)
    dy = torch.empty_like(y)
    dl = None
    if dloss is not None:
        dloss = dloss.to(dtype=y.dtype).contiguous()
        dl = C.c_void_p(dloss.data_ptr())
    fn = lib().drg_objective_bwd_f64 if f64 else lib().drg_objective_bwd
    _check(fn(ctx.h, sim.h, C.byref(p), ptr, dl, C.c_void_p(dy.data_ptr())))
    return dy


def drg_sample_negatives(ctx: Context, sim: Similarity, M: int, seed: int, iter: int):
    import torch
    out = torch.empty((sim.n, M), dtype=torch.int32, device="cuda")
    _check(lib().drg_sample_negatives(ctx.h, sim.h, int(M), int(seed), int(iter),
                                      C.c_void_p(out.data_ptr())))
    return out


def drg_sim_coo(ctx: Context, sim: Similarity):
    """(rows, cols, P) device tensors of P~ in CSR order (FP32 values)."""
    import torch
    rows = torch.empty(sim.nnz, dtype=torch.int32, device="cuda")
    cols = torch.empty(sim.nnz, dtype=torch.int32, device="cuda")
    P = torch.empty(sim.nnz, dtype=torch.float32, device="cuda")
    _check(lib().drg_sim_coo(ctx.h, sim.h, C.c_void_p(rows.data_ptr()),
                             C.c_void_p(cols.data_ptr()), C.c_void_p(P.data_ptr())))
    return rows, cols, P


def _objective_function():
    import torch

    class DRGObjective(torch.autograd.Function):
        """L^(y) with the library's forward and hand-written backward.  Only y
        (and the scalar parameters) are saved; the backward draws the
        negatives again from their counters."""

        @staticmethod
        def forward(fctx, y, ctx, sim, M, b, gamma, seed, it):
            fctx.save_for_backward(y)
            fctx.args = (ctx, sim, M, b, gamma, seed, it)
            return drg_objective_fwd(ctx, sim, y.contiguous(), M=M, b=b, gamma=gamma, seed=seed,
                                     iter=it)

        @staticmethod
        def backward(fctx, gloss):
            (y,) = fctx.saved_tensors
            ctx, sim, M, b, gamma, seed, it = fctx.args
            dy = drg_objective_bwd(ctx, sim, y.contiguous(), gloss, M=M, b=b, gamma=gamma,
                                   seed=seed, iter=it)
            return dy, None, None, None, None, None, None, None

    return DRGObjective


_DRGObjective = None


def objective(y, ctx: Context, sim: Similarity, *, M=5, b=1, gamma=0.1, seed=0, iter=0):
    """Differentiable L^(y) (torch.autograd.Function over the library)."""
    global _DRGObjective
    if _DRGObjective is None:
        _DRGObjective = _objective_function()
    _shape(b)
    return _DRGObjective.apply(y, ctx, sim, int(M), float(b), float(gamma), int(seed), int(iter))
