"""Benchmark of the DRGraph layout hot path on one MI355X.

One step = one complete layout of the workload through the C-ABI library,
with the input graph already resident in device memory: k-hop sparse
distance matrix and similarity, negative-sampling table, multilevel
coarsening, random initial layout, every iteration of the schedule at every
level, and the refinements between levels.

Metric: pair-updates/s = (T iterations x pairs per iteration) / time to
layout, pairs per iteration = nnz(P~) + M * N_a (every stored pair is swept
once and every non-isolated node draws M negatives, at every level).

Prints one JSON line.  Extra objects:
  roofline     -- the dominant kernel against the roof that binds it, with its
                  launch duration measured with HIP events on the library's
                  stream over the timed region.  The column-blocked sweep is
                  bound by vector-ALU issue ("alu"): achieved = the 15 VALU
                  lane-instructions a stored pair needs x pairs per launch /
                  launch time, against 256 CUs x 64 lanes x 2.4 GHz.  Row-form
                  sweeps are reported against HBM with the algorithmic bytes
                  16 nnz + 16 M N_a + 28 N per launch.  `traffic` (HBM bytes per
                  launch), `hbm_measured`, `valu_issue` and `l2_hit_rate` come
                  from committed rocprofv3 counter summaries and are null
                  unless those were taken on the current sources; `convention`
                  keeps the algorithmic-bytes figure of the blocked sweep,
                  which counts 16 bytes per pair that LDS and recomputation
                  serve and is therefore not a fraction of any roof;
  cpu_baseline -- the FP64 oracle, single-threaded, timed on a bounded sample
                  of the same workload family, with the time-to-layout of the
                  workload extrapolated from it (labelled as such).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # R-MAT power-law graph: 2^20 nodes, 16*2^20 generated edges, k=2, M=5,
    # 500 iterations, multilevel until < 1000 nodes
    "rmat20_k2": dict(graph="rmat20", k=2, M=5, b=1, T=500, min_nodes=1000, max_levels=64),
    # the same family at the paper's own neighbourhood order
    "rmat20_k1": dict(graph="rmat20", k=1, M=5, b=1, T=500, min_nodes=1000, max_levels=64),
    # random geometric graph, 100k nodes, radius 0.006, 3 levels
    "rgg100k_k3": dict(graph="rgg100k", k=3, M=10, b=2, T=500, min_nodes=1, max_levels=3),
    # 32x32 grid, single level
    "grid32_k3": dict(graph="grid32", k=3, M=5, b=3, T=300, min_nodes=1 << 30, max_levels=1),
    # R-MAT 2^18, average degree 16, k=2
    "rmat18_k2": dict(graph="rmat18", k=2, M=5, b=1, T=500, min_nodes=1000, max_levels=64),
}


# sources that make up each profiled kernel (the counter summaries hold
# their hash; a summary taken on other sources is not used)
KERNEL_SOURCES = {
    "k_sweep_blocked": ("blocked.hip", "drg_blocked.hpp", "drg_common.hpp", "drg_forces.hpp"),
    "k_sweep": ("layout.hip", "drg_common.hpp", "drg_forces.hpp"),
    "k_b_sweep_win": ("batch.hip", "drg_blocked.hpp", "drg_common.hpp", "drg_forces.hpp"),
    "k_b_sweep": ("batch.hip", "drg_blocked.hpp", "drg_common.hpp", "drg_forces.hpp"),
}


def _kernel_source_hash(kernel: str) -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(kernel, ()):
        with open(os.path.join(ROOT, "paper_2008_07799_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic(workload: str, kernel: str):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if
    they were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != _kernel_source_hash(kernel):
        return None
    return rec.get("bytes_per_launch")


def _l2_hit_rate(workload: str, kernel: str):
    """L2 hit rate of the kernel (TCC_HIT / (TCC_HIT + TCC_MISS)) from a
    committed rocprofv3 counter summary, if taken on the current source."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_l2.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != _kernel_source_hash(kernel):
        return None
    return rec.get("l2_hit_rate")


# Lane-operation issue peak without packed FP32: 256 CUs x 4 SIMDs x 16 lanes
# x 2.4 GHz (one wave64 VALU instruction per CU per cycle).
VALU_LANE_PEAK = 256 * 64 * 2.4e9

# VALU lane-instructions one stored pair needs in the column-blocked sweep
# (b = 1, clip unable to bind): column extract, LDS address, two differences,
# 1 + d^2 as two FMAs, reciprocal, hop bit, hop-weight select, 1/Z_i + 1/Z_j,
# weight, weight x reciprocal, two FMAs into the partials, row-end test.
ALU_OPS_PER_PAIR = 15


def _valu_issue(workload: str, kernel: str, avg_ms: float):
    """VALU issue rate of the launch: wave64 VALU instructions per dispatch
    from a committed rocprofv3 SQ counter summary (if taken on the current
    kernel source) x 64 lanes / the launch time measured in this run."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_valu.json")
    if not os.path.exists(path) or avg_ms <= 0:
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != _kernel_source_hash(kernel):
        return None
    lane_ops = rec["counters_per_dispatch"]["SQ_INSTS_VALU"] * 64
    achieved = lane_ops / (avg_ms / 1000.0)
    return {"achieved": achieved, "peak": VALU_LANE_PEAK, "unit": "lane-ops/s",
            "frac": achieved / VALU_LANE_PEAK,
            "lane_slots_per_pair": rec["valu_lane_slots_per_pair"],
            "counter_issue_per_cu_cycle": rec["valu_insts_per_cu_cycle"]}


def roofline(workload, kernel, avg_ms, launches, nnz, n_active, n, M, b, copy_gbs) -> dict:
    """The dominant kernel against its roof (see the module docstring)."""
    t = avg_ms / 1000.0
    alg_bytes = 16.0 * nnz + 16.0 * M * n_active + 28.0 * n
    traffic = _traffic(workload, kernel)
    hbm_measured = None
    if traffic and t > 0:
        hbm_measured = {"achieved": traffic / t / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": traffic / t / 1e9 / HBM_PEAK_GBS}
    common = {"kernel": kernel, "launches": launches, "avg_launch_ms": avg_ms,
              "traffic": traffic, "hbm_measured": hbm_measured,
              "valu_issue": _valu_issue(workload, kernel, avg_ms),
              "l2_hit_rate": _l2_hit_rate(workload, kernel),
              "measured_copy_GBs": copy_gbs}
    if kernel.startswith("k_sweep_blocked") and b == 1 and t > 0:
        ops = ALU_OPS_PER_PAIR * float(nnz)
        achieved = ops / t / 1e12
        peak = VALU_LANE_PEAK / 1e12
        conv = alg_bytes / t / 1e9
        return {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Tlane-op/s",
                "frac": achieved / peak, "algorithmic_lane_ops_per_pair": ALU_OPS_PER_PAIR,
                "pairs_per_launch": nnz, **common,
                "convention": {"algorithmic_bytes_per_launch": alg_bytes, "GBs": conv,
                               "frac_of_8TBs": conv / HBM_PEAK_GBS,
                               "note": "16 B per pair by convention; the sweep reads 2 B "
                                       "entries and LDS-staged records, so this is not a "
                                       "fraction of any roof"}}
    achieved = alg_bytes / t / 1e9 if t > 0 else 0.0
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": alg_bytes, **common}


def _copy_bandwidth(mib: int = 4096) -> float:
    """Bandwidth of a plain device-to-device copy (bytes read + written per
    second, GB/s), HIP events around 8 copies of a `mib` MiB buffer."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(8):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    gbs = 8 * 2 * n * 4 / (e0.elapsed_time(e1) / 1000.0) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def host_cpu() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg: dict, workload_pairs: float = 0.0, workload_nnz: float = 0.0) -> dict:
    """The oracle (FP64, one thread) on a bounded sample: an R-MAT of the same
    generator at scale 14 (edge factor 16) with the workload's k, M and b;
    similarity built once, then synchronous iterations at level 0 timed.
    The workload's time-to-layout is extrapolated from the sample's rates
    (similarity entries per second, pair-updates per second)."""
    from oracle import drgo
    from paper_2008_07799_amd import gen

    if cfg["graph"].startswith("rmat"):
        g = gen.rmat(14, 16, seed=0)
        sample = "R-MAT scale 14, edge factor 16"
    elif cfg["graph"] == "rgg100k":
        g = gen.rgg(20000, 0.0134, seed=0)
        sample = "RGG 20k nodes"
    else:
        g = gen.grid(32, 32)
        sample = "32x32 grid"
    drgo.build()
    t0 = time.perf_counter()
    sim = drgo.similarity(g, cfg["k"])
    t_sim = time.perf_counter() - t0
    y = drgo.init(g.n, 0, 0)
    pairs = sim.nnz + cfg["M"] * sim.n_active
    iters = 0
    t0 = time.perf_counter()
    while True:
        drgo.iter_sync(sim, y, None, cfg["M"], cfg["b"], 0.1, 1.0, 4.0, 0, iters)
        iters += 1
        el = time.perf_counter() - t0
        if el > 8.0 or iters >= 200:
            break
    rate = pairs * iters / el
    out = {"value": rate, "unit": "pair-updates/s", "cores": 1, "kind": "oracle",
           "host_cpu": host_cpu(), "host_threads": os.cpu_count(),
           "sample": f"{sample} (n={g.n}, nnz(P)={sim.nnz}), k={cfg['k']}, M={cfg['M']}, "
                     f"b={cfg['b']}: {iters} synchronous iterations at level 0 in "
                     f"{el:.2f} s after a {t_sim:.2f} s similarity build"}
    if workload_pairs > 0:
        t_it = cfg["T"] * workload_pairs / rate
        t_s = workload_nnz * t_sim / max(sim.nnz, 1)
        out["extrapolated_time_to_layout_s"] = {
            "value": t_it + t_s, "iterations_s": t_it, "similarity_s": t_s,
            "note": "EXTRAPOLATED from the sample's rates to the workload's pair count "
                    "and pattern size; not measured"}
    return out


def cpu_plan(parts: str = "abcdef") -> dict:
    """The oracle timed on the host (FP64, one thread) over the workloads:
    the 32x32 grid and the 100k-node RGG in full; R-MAT 2^20 at k = 1 in full;
    R-MAT 2^16 at k = 2 (similarity and 10 level-0 iterations) with the
    2^20-node k = 2 layout extrapolated from its rates; 16 graphs of the
    512-graph batch spanning its size range, with the whole batch
    extrapolated by pair count; the autograd workload's forward and gradient
    on R-MAT 2^18.  Extrapolated figures are labelled."""
    from oracle import drgo
    from paper_2008_07799_amd import gen

    drgo.build()
    out = {"kind": "oracle", "cores": 1, "host_cpu": host_cpu(), "host_threads": os.cpu_count()}

    def log(*a):
        print("[cpu-plan]", *a, file=sys.stderr, flush=True)

    def done(key):
        # each workload's figures as soon as they are measured
        print(json.dumps({"cpu_plan_part": key, **out[key]}), flush=True)

    def similarity(g, k, tag):
        """drgo.similarity in its three steps (count, fill, normalise), each
        reported as it ends."""
        L = drgo.lib()
        rp32 = np.ascontiguousarray(g.row_ptr, np.int32)
        col32 = np.ascontiguousarray(g.col, np.int32)
        out_rp = np.zeros(g.n + 1, np.int64)
        nnz = L.drgo_khop_count(g.n, rp32, col32, int(k), out_rp)
        log(tag, f"pattern counted: {nnz} entries")
        out_col = np.zeros(max(nnz, 1), np.int32)
        out_hop = np.zeros(max(nnz, 1), np.uint8)
        L.drgo_khop_fill(g.n, rp32, col32, int(k), out_rp, out_col, out_hop)
        log(tag, "pattern filled")
        sim = drgo.similarity_from_pattern(g.n, k, 1.0, out_rp, out_col[:nnz], out_hop[:nnz])
        log(tag, "similarity normalised")
        return sim

    def full_layout(g, k, M, b, T, min_nodes, max_levels, seed=0, tag=""):
        t0 = time.perf_counter()
        sim = similarity(g, k, tag)
        t_sim = time.perf_counter() - t0
        hier = drgo.hierarchy(g, seed, 0.8, min_nodes, max_levels)
        t_h = time.perf_counter() - t0 - t_sim
        Lc = hier.levels
        y = drgo.init(hier.sizes[-1], seed, Lc - 1)
        gi, last = 0, time.perf_counter()
        t1 = time.perf_counter()
        for (l, Tl, gam) in drgo.schedule(T, Lc, 0.1, 0.01):
            cm = None if l == 0 else hier.cmaps[l]
            for t in range(Tl):
                drgo.iter_sync(sim, y, cm, M, b, gam, drgo.eta_at(1.0, t, Tl), 4.0, seed, gi)
                gi += 1
                if time.perf_counter() - last > 20:
                    last = time.perf_counter()
                    log(tag, f"iteration {gi}/{T}")
            if l > 0:
                y = y[hier.maps[l - 1]].copy()
        t_it = time.perf_counter() - t1
        pairs = sim.nnz + M * sim.n_active
        return {"time_to_layout_s": time.perf_counter() - t0, "similarity_s": t_sim,
                "hierarchy_s": t_h, "iterations_s": t_it, "levels": hier.sizes, "nnz_P": sim.nnz,
                "pair_updates_per_s": T * pairs / t_it}

    if "a" in parts:
        log("grid32")
        out["grid32_k3"] = full_layout(gen.grid(32, 32), 3, 5, 3, 300, 1 << 30, 1, tag="grid32")
        done("grid32_k3")
    if "b" in parts:
        log("rgg100k")
        out["rgg100k_k3"] = full_layout(gen.named("rgg100k"), 3, 10, 2, 500, 1, 3, tag="rgg100k")
        done("rgg100k_k3")
    if "c" in parts:
        log("rmat20 k=1")
        g20 = gen.named("rmat20")
        out["rmat20_k1"] = full_layout(g20, 1, 5, 1, 500, 1000, 64, tag="rmat20 k=1")
        del g20
        done("rmat20_k1")
    if "d" in parts:
        rmat16_part(out, log, similarity)
        done("rmat16_k2_sample")
    if "e" in parts:
        batch_part(out, log, full_layout)
        done("batch512_k3_subset")
    if "f" in parts:
        autograd_part(out, log, similarity)
        done("autograd_rmat18_k2")
    return out


def rmat16_part(out, log, similarity):
    from oracle import drgo
    from paper_2008_07799_amd import gen
    log("rmat16 k=2 sample")
    g16 = gen.rmat(16, 16, seed=0)
    t0 = time.perf_counter()
    sim = similarity(g16, 2, "rmat16")
    t_sim = time.perf_counter() - t0
    y = drgo.init(g16.n, 0, 0)
    t0 = time.perf_counter()
    for it in range(10):
        drgo.iter_sync(sim, y, None, 5, 1, 0.1, 1.0, 4.0, 0, it)
        log("rmat16 iteration", it)
    t_it = time.perf_counter() - t0
    pairs16 = sim.nnz + 5 * sim.n_active
    rate = 10 * pairs16 / t_it
    # R-MAT 2^20, k = 2: pattern entries and active nodes as the library counts
    # them (its rows match the oracle rows-only similarity on sampled rows)
    nnz20, na20 = 23762699968, 646140
    out["rmat16_k2_sample"] = {
        "nnz_P": sim.nnz, "similarity_s": t_sim, "iterations": 10, "iterations_s": t_it,
        "pair_updates_per_s": rate, "similarity_entries_per_s": sim.nnz / t_sim,
        "extrapolated_rmat20_k2_time_to_layout_s": {
            "value": 500 * (nnz20 + 5 * na20) / rate + nnz20 / (sim.nnz / t_sim),
            "note": "EXTRAPOLATED from the 2^16 sample's rates to nnz 2.376e10, 500 "
                    "iterations; the oracle cannot hold that pattern (about 310 GB)"}}
    del sim


def batch_part(out, log, full_layout):
    from oracle import drgo
    from paper_2008_07799_amd import gen
    log("batch subset")
    graphs = gen.batch_graphs(512)
    order = np.argsort([g.n for g in graphs], kind="stable")
    pick = [int(order[i]) for i in range(0, 512, 32)]
    t_sub, work_sub = 0.0, 0.0
    for c in pick:
        g = graphs[c]
        b = 3 if c % 2 == 0 else 1
        r = full_layout(g, 3, 5, b, 300, 1000, 64, seed=c, tag=f"batch graph {c}")
        log(f"batch graph {c} (n={g.n}) done")
        t_sub += r["time_to_layout_s"]
        work_sub += 300 * (r["nnz_P"] + 5 * int(np.count_nonzero(np.diff(g.row_ptr))))
    work_all = 0.0
    for g in graphs:
        rp = np.zeros(g.n + 1, np.int64)
        nnz = drgo.lib().drgo_khop_count(g.n, np.ascontiguousarray(g.row_ptr, np.int32),
                                         np.ascontiguousarray(g.col, np.int32), 3, rp)
        work_all += 300 * (nnz + 5 * int(np.count_nonzero(np.diff(g.row_ptr))))
    out["batch512_k3_subset"] = {
        "graphs": pick, "subset_time_to_layout_s": t_sub,
        "extrapolated_batch_time_to_layout_s": {
            "value": t_sub * work_all / work_sub,
            "note": "EXTRAPOLATED from the 16-graph subset by pair count (T x (nnz + M N_a))"}}
    del graphs


def autograd_part(out, log, similarity):
    from oracle import drgo
    from paper_2008_07799_amd import gen
    log("autograd rmat18 forward + gradient")
    g18 = gen.named("rmat18")
    t0 = time.perf_counter()
    sim = similarity(g18, 2, "rmat18")
    t_sim = time.perf_counter() - t0
    y = np.random.default_rng(0).uniform(-5, 5, size=(g18.n, 2))
    t0 = time.perf_counter()
    drgo.objective(sim, y, 5, 1, 0.1, 0, 0)
    t_f = time.perf_counter() - t0
    log("rmat18 forward done")
    t0 = time.perf_counter()
    drgo.objective_grad(sim, y, 5, 1, 0.1, 0, 0)
    t_g = time.perf_counter() - t0
    out["autograd_rmat18_k2"] = {"nnz_P": sim.nnz, "similarity_s": t_sim, "forward_s": t_f,
                                 "gradient_s": t_g}


def bench_autograd(args):
    """The differentiable form on R-MAT 2^18 (edge factor 8), k=2, M=5, b=1:
    one step = L^ forward (library) + anchor MSE on 1% of the nodes, backward
    (hand-written, library), SGD update of Y.  Compared with the same loss
    written in eager PyTorch on the same P~ (device COO) and negatives."""
    import torch
    from paper_2008_07799_amd import drgraph as d
    from paper_2008_07799_amd import gen

    M, b, gamma, lam, lr = 5, 1, 0.1, 1.0, 0.5
    print("[bench] generating rmat18", file=sys.stderr, flush=True)
    g = gen.rmat(18, 8, seed=0)
    torch.cuda.set_device(0)
    rp, col = d.to_device(g)
    ctx = d.Context(0)
    sim = d.drg_build_similarity(ctx, rp, col, 2)
    n, na = g.n, sim.n_active
    rng = np.random.default_rng(0)
    anchors = torch.from_numpy(rng.choice(n, size=n // 100, replace=False)).cuda()
    targets = torch.from_numpy(rng.uniform(-1, 1, size=(anchors.numel(), 2)).astype(np.float32)).cuda()
    y0 = torch.from_numpy(rng.uniform(-5, 5, size=(n, 2)).astype(np.float32)).cuda()

    def anchor_term(y):
        return lam * ((y[anchors] - targets) ** 2).sum(dim=1).mean()

    def ours_loss(y, it):
        return -d.objective(y, ctx, sim, M=M, b=b, gamma=gamma, seed=0, iter=it) / na + anchor_term(y)

    rows, cols, P = d.drg_sim_coo(ctx, sim)
    rows, cols = rows.long(), cols.long()
    qt = torch.from_numpy(sim.export(values=False)["qt"].astype(np.float32)).cuda()
    ar = torch.arange(n, device="cuda")

    def eager_loss(y, it):
        neg = d.drg_sample_negatives(ctx, sim, M, 0, it).long()
        dd = y[rows] - y[cols]
        d2 = (dd * dd).sum(dim=1)
        att = (P * -torch.log1p(d2 ** b)).sum()
        valid = (neg >= 0) & (neg != ar[:, None])
        vv = neg.clamp(min=0)
        dn = y[:, None, :] - y[vv]
        d2n = (dn * dn).sum(dim=-1)
        ok = valid & (d2n > 0)
        d2s = torch.where(ok, d2n, torch.ones_like(d2n))
        term = torch.where(ok, b * torch.log(d2s) - torch.log1p(d2s ** b), torch.zeros_like(d2s))
        rep = gamma * (qt[:, None] * term).sum()
        return -(att + rep) / na + anchor_term(y)

    def run(loss_fn, steps, warm):
        y = y0.clone().requires_grad_(True)
        for s in range(warm + steps):
            if s == warm:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
            y.grad = None
            loss = loss_fn(y, s)
            loss.backward()
            with torch.no_grad():
                y -= lr * y.grad
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1000.0 / steps, y.detach()

    # accuracy at the same point, both against the FP64 instance of the
    # library's objective (which matches the FP64 oracle to 1e-10)
    y64 = y0.double()
    l64 = float(-d.drg_objective_fwd(ctx, sim, y64, M=M, b=b, gamma=gamma, seed=0, iter=0) / na
                + lam * ((y64[anchors] - targets.double()) ** 2).sum(dim=1).mean())
    g64 = -d.drg_objective_bwd(ctx, sim, y64, M=M, b=b, gamma=gamma, seed=0, iter=0) / na
    g64[anchors] += 2.0 * lam * (y64[anchors] - targets.double()) / anchors.numel()
    acc = {}
    for name, fn in (("ours", ours_loss), ("eager", eager_loss)):
        ya = y0.clone().requires_grad_(True)
        la = fn(ya, 0)
        la.backward()
        acc[name] = {"loss_rel_err_vs_fp64": abs(float(la.detach()) - l64) / abs(l64),
                     "grad_rel_err_vs_fp64": float((ya.grad.double() - g64).abs().max()
                                                   / g64.abs().max())}
        del ya, la
    torch.cuda.empty_cache()
    print("[bench] ours", file=sys.stderr, flush=True)
    ms_ours, _ = run(ours_loss, args.steps, max(1, args.warmup))
    ms_eager = None
    if not args.no_compare:
        torch.cuda.empty_cache()
        print("[bench] eager", file=sys.stderr, flush=True)
        ms_eager, _ = run(eager_loss, args.steps, max(1, args.warmup))
    pairs = sim.nnz + M * na
    rec = {
        "metric": "pair-updates/s + time-to-layout, 1M-node R-MAT; batched/autograd vs plain",
        "value": pairs / (ms_ours / 1000.0), "unit": "pair-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": max(1, args.warmup), "ms_per_step": ms_ours,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "autograd_rmat18_k2", "graph": "rmat18", "n": n, "k": 2, "M": M,
                   "b": b, "nnz_P": sim.nnz, "n_active": na, "anchors": int(anchors.numel()),
                   "step": "forward + backward + SGD update"},
        "vs_eager_pytorch": {"eager_ms_per_step": ms_eager,
                             "speedup": ms_eager / ms_ours if ms_eager else None,
                             "accuracy": acc},
    }
    print(json.dumps(rec), flush=True)


def bench_batch(args):
    """The batched form: 512 graphs, log-uniform 500..50,000 nodes, grids
    minus 5% of their edges (even index, b=3) and Barabasi-Albert m=3 (odd
    index, b=1), k=3, M=5, 300 iterations over each graph's own levels.
    One step = drg_batch_create (similarity of all graphs, hierarchies,
    schedules, recorded run) + one replay.  Compared with the plain path: a
    loop of drg_layout calls, one per graph, whose outputs are bit-identical."""
    import torch
    from paper_2008_07799_amd import drgraph as d
    from paper_2008_07799_amd import gen

    M, T, k = 5, 300, 3
    print("[bench] generating 512 graphs", file=sys.stderr, flush=True)
    graphs = gen.batch_graphs(512)
    torch.cuda.set_device(0)
    ctx = d.Context(0)
    devs = [d.to_device(g) for g in graphs]
    params = [d.layout_params(k=k, M=M, b=3 if c % 2 == 0 else 1, T=T, min_nodes=1000,
                              seed=c) for c in range(len(graphs))]
    n_total = sum(g.n for g in graphs)
    y = torch.zeros((n_total, 2), dtype=torch.float32, device="cuda")

    def step():
        t = time.perf_counter()
        b = d.drg_batch_create(ctx, devs, params)
        t_create = time.perf_counter() - t
        print(f"[bench]   batch created: {b.n_total} nodes, nnz={b.nnz}, "
              f"levels {min(b.levels)}..{max(b.levels)} ({t_create:.2f} s)",
              file=sys.stderr, flush=True)
        b.run(ctx, y)
        print(f"[bench]   batch run done ({time.perf_counter() - t:.2f} s), sweep tuning "
              f"{b.tuning()}", file=sys.stderr, flush=True)
        return b, t_create

    for w in range(args.warmup):
        print(f"[bench] warmup step {w}", file=sys.stderr, flush=True)
        step()[0].close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        print(f"[bench] timed step {s}", file=sys.stderr, flush=True)
        if s:
            b.close()
        b, t_create = step()
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1000.0 / args.steps
    # replays of the recorded run alone (HIP events on the library's stream)
    ctx.set_profiling(True)
    for _ in range(2):
        b.run(ctx, y)
    launches, run_ms = ctx.kernel_stats()
    ctx.set_profiling(False)
    run_ms /= max(1, launches)
    tuning = b.tuning()
    yb = y.cpu().numpy()
    # per-graph active rows, for the pair count
    nnz_total = b.nnz
    n_active = 0
    for g in graphs:
        n_active += int(np.count_nonzero(np.diff(g.row_ptr) > 0))
    pairs = nnz_total + M * n_active  # k >= 1: a node is active iff it has an edge
    b.close()
    compare = None
    if not args.no_compare:
        # the plain path: one drg_layout per graph
        print("[bench] plain per-graph loop", file=sys.stderr, flush=True)
        yp = torch.zeros_like(y)
        base = np.concatenate([[0], np.cumsum([g.n for g in graphs])])
        torch.cuda.synchronize()
        tp = time.perf_counter()
        for c, (rp, col) in enumerate(devs):
            d.drg_layout(ctx, rp, col, params[c], yp[base[c]:base[c + 1]])
        torch.cuda.synchronize()
        plain_ms = (time.perf_counter() - tp) * 1000.0
        compare = {"plain_ms": plain_ms, "speedup": plain_ms / ms_per_step,
                   "bit_identical": bool(np.array_equal(yp.cpu().numpy(), yb))}
    alg_bytes = 16.0 * nnz_total + 16.0 * M * n_active + 28.0 * n_total
    it_ms = run_ms / T
    # one iteration of the recorded run (every graph at its level: stage, the
    # row-form sweep of the smaller graphs, the column-blocked sweep and
    # finish of the large ones, apply), from HIP events around the replays
    kernel = "iteration (k_b_stage + k_b_sweep/k_b_sweep_win + k_b_sweep_blocked + k_b_finish + k_b_apply)"
    # 99% of the stored pairs belong to the column-blocked BA graphs (b = 1):
    # the iteration is priced at the blocked sweep's 15 lane-instructions per pair
    achieved = ALU_OPS_PER_PAIR * float(nnz_total) / (it_ms / 1000.0) / 1e12
    peak = VALU_LANE_PEAK / 1e12
    conv = alg_bytes / (it_ms / 1000.0) / 1e9
    rec = {
        "metric": "pair-updates/s + time-to-layout, 1M-node R-MAT; batched/autograd vs plain",
        "value": T * pairs / (ms_per_step / 1000.0), "unit": "pair-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batch512_k3", "graphs": len(graphs), "n_total": n_total,
                   "nnz_P": nnz_total, "n_active": n_active, "k": k, "M": M, "T": T,
                   "b": "3 (grids), 1 (BA)", "time_to_layout_s": ms_per_step / 1000.0,
                   "create_s": t_create, "replay_ms": run_ms, "avg_iteration_ms": it_ms,
                   "sweep_tuning": tuning,
                   "replay_pair_updates_per_s": T * pairs / (run_ms / 1000.0)},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Tlane-op/s",
                     "frac": achieved / peak, "traffic": None, "kernel": kernel,
                     "avg_launch_ms": it_ms,
                     "algorithmic_lane_ops_per_pair": ALU_OPS_PER_PAIR,
                     "convention": {"algorithmic_bytes_per_launch": alg_bytes, "GBs": conv,
                                    "frac_of_8TBs": conv / HBM_PEAK_GBS,
                                    "note": "16 B per pair by convention; not a fraction "
                                            "of any roof (LDS-staged records, 2 B entries)"}},
        "vs_plain_per_graph_loop": compare,
    }
    print(json.dumps(rec), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat20_k2",
                    choices=sorted(WORKLOADS) + ["autograd_rmat18_k2", "batch512_k3"])
    ap.add_argument("--mode", default="sync", choices=["sync", "async"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the comparison runs (per-graph loop, eager PyTorch)")
    ap.add_argument("--source-hash", default="", metavar="KERNEL",
                    help="only print the source hash of a profiled kernel")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized device buffer 8 times (counter calibration)")
    ap.add_argument("--cpu-plan", default="", metavar="PARTS",
                    help="only time the CPU oracle over the workloads: a grid32, b rgg100k, "
                         "c rmat20 k=1, d rmat16 k=2 sample, e batch subset, f autograd "
                         "(e.g. abcdef; about 20 minutes in all)")
    args = ap.parse_args()
    if args.cpu_plan:
        print(json.dumps(cpu_plan(args.cpu_plan)), flush=True)
        return
    if args.source_hash:
        print(_kernel_source_hash(args.source_hash))
        return
    if args.copy_probe:
        import torch
        n = args.copy_probe * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(8):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_per_launch": n * 4, "launches": 8}), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the library and this benchmark run on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    if args.workload == "autograd_rmat18_k2":
        bench_autograd(args)
        return
    if args.workload == "batch512_k3":
        bench_batch(args)
        return

    import torch
    from paper_2008_07799_amd import drgraph as d
    from paper_2008_07799_amd import gen

    cfg = WORKLOADS[args.workload]
    mode = d.DRG_MODE_SYNC if args.mode == "sync" else d.DRG_MODE_ASYNC
    print(f"[bench] generating {cfg['graph']}", file=sys.stderr, flush=True)
    g = gen.named(cfg["graph"], seed=0)
    torch.cuda.set_device(0)
    rp, col = d.to_device(g)
    ctx = d.Context(0)
    params = d.layout_params(k=cfg["k"], M=cfg["M"], b=cfg["b"], T=cfg["T"],
                             min_nodes=cfg["min_nodes"], max_levels=cfg["max_levels"],
                             seed=0, mode=mode)
    y = torch.zeros((g.n, 2), dtype=torch.float32, device="cuda")

    phase_s = {"similarity": 0.0, "hierarchy": 0.0, "layout": 0.0}
    kept = {}

    def step(keep=False):
        t = time.perf_counter()
        sim = d.drg_build_similarity(ctx, rp, col, cfg["k"])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        print(f"[bench]   similarity nnz={sim.nnz} ({t1 - t:.2f} s)", file=sys.stderr, flush=True)
        hier = d.drg_coarsen(ctx, rp, col, seed=0, rho=0.8, min_nodes=cfg["min_nodes"],
                             max_levels=cfg["max_levels"])
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        print(f"[bench]   hierarchy {hier.sizes} ({t2 - t:.2f} s)", file=sys.stderr, flush=True)
        d.drg_layout_run(ctx, sim, hier, params, y)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        print(f"[bench]   layout done ({t3 - t:.2f} s)", file=sys.stderr, flush=True)
        phase_s["similarity"] += t1 - t
        phase_s["hierarchy"] += t2 - t1
        phase_s["layout"] += t3 - t2
        info = (sim.nnz, sim.n_active, hier.sizes, sim.blocked)
        if keep:
            kept["sim"] = sim
        else:
            sim.close()
        hier.close()
        return info

    for w in range(args.warmup):
        print(f"[bench] warmup step {w}", file=sys.stderr, flush=True)
        step()
    for key in phase_s:
        phase_s[key] = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        print(f"[bench] timed step {s}", file=sys.stderr, flush=True)
        nnz, n_active, sizes, blocked = step(keep=(s == args.steps - 1))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    # the sweep kernel's launches timed with HIP events on the library's
    # stream, in one more (untimed) layout: the timed steps run without the
    # events, which keep a small run from being recorded into one graph
    print("[bench] kernel timing step", file=sys.stderr, flush=True)
    ctx.set_profiling(True)
    prof_phase = dict(phase_s)
    step()
    phase_s.update(prof_phase)
    launches, sweep_ms = ctx.kernel_stats()
    ctx.set_profiling(False)

    # layout quality of the result (outside the timed region): NP (Sec. 4.1)
    # of 1000 sampled non-isolated nodes, graph neighbourhoods = the rows of
    # the workload's own similarity (k_eval = k)
    sim = kept.pop("sim")
    deg = np.diff(g.row_ptr)
    sample = np.random.default_rng(0).choice(np.nonzero(deg > 0)[0], size=1000, replace=False)
    t_np = time.perf_counter()
    np_vals = d.drg_neighbourhood_preservation(
        ctx, sim, y, torch.from_numpy(np.sort(sample).astype(np.int32)).cuda()).cpu().numpy()
    t_np = time.perf_counter() - t_np
    sim.close()
    # and the sampled stress (Sec. 4.1): whole-graph searches from 64 sources
    t_st = time.perf_counter()
    src = np.sort(np.random.default_rng(1).choice(np.nonzero(deg > 0)[0], size=64,
                                                  replace=False)).astype(np.int32)
    _, stress_est = d.drg_stress_sampled(ctx, rp, col, y, torch.from_numpy(src).cuda())
    t_st = time.perf_counter() - t_st
    M, T, n = cfg["M"], cfg["T"], g.n
    pairs = nnz + M * n_active
    value = T * pairs / (ms_per_step / 1000.0)
    avg_ms = sweep_ms / max(1, launches)
    alg_bytes = 16.0 * nnz + 16.0 * M * n_active + 28.0 * n
    form = ctx.last_sweep()
    kernel = {d.DRG_SWEEP_BLOCKED: "k_sweep_blocked",
              d.DRG_SWEEP_BLOCKED_ASYNC: "k_sweep_blocked+k_finish_inplace (async stages)",
              d.DRG_SWEEP_ROW_ASYNC: "k_sweep_async",
              d.DRG_SWEEP_WINDOW: "k_sweep_win"}.get(form, "k_sweep")
    ran_mode = "async" if form in (d.DRG_SWEEP_BLOCKED_ASYNC, d.DRG_SWEEP_ROW_ASYNC) else "sync"
    copy_gbs = _copy_bandwidth()
    roof = roofline(args.workload, kernel, avg_ms, launches, nnz, n_active, n, M, cfg["b"],
                    copy_gbs)
    rec = {
        "metric": "pair-updates/s + time-to-layout, 1M-node R-MAT; batched/autograd vs plain",
        "value": value,
        "unit": "pair-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "graph": cfg["graph"], "n": n,
                   "undirected_edges": g.nnz // 2, "k": cfg["k"], "M": M, "b": cfg["b"],
                   "T": T, "levels": sizes, "nnz_P": nnz, "n_active": n_active,
                   "mode": ran_mode, "time_to_layout_s": ms_per_step / 1000.0,
                   "layout_only_s": phase_s["layout"] / args.steps,
                   "np_sampled": {"value": float(np_vals[np_vals >= 0].mean()), "nodes": 1000,
                                  "k_eval": cfg["k"], "seconds": t_np},
                   "stress_sampled": {"value": stress_est, "sources": 64, "seconds": t_st},
                   "phases_s": {k: v / args.steps for k, v in phase_s.items()},
                   "iteration_sweep_pair_updates_per_s": pairs / (avg_ms / 1000.0)},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline(cfg, pairs, nnz)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
