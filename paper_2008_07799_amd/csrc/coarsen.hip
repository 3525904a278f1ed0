// coarsen.hip -- multilevel coarsening (Sec. 3.2.3, Fig. 3).
//
// The paper repeatedly picks a random unassigned node and groups it with its
// unassigned first-order neighbours.  With a Philox priority per node and
// nodes visited in descending (priority, -id) order, a node starts a group
// exactly when no higher-priority neighbour started one (the greedy maximal
// independent set), and every other node joins the highest-priority group
// centre among its neighbours.  That answer is reached here by rounds of
// local decisions over all nodes in parallel: a node becomes a centre once all
// its higher-priority neighbours are decided non-centres, and a member once
// any of them is a centre.  Coarse ids are the centres ranked by node id.
// The coarse graph keeps one edge between two groups joined by a fine edge;
// it is built like a BFS row: the fine neighbours of all members, mapped to
// their group, are collected in a bitmap and emitted in ascending order.
#include <memory>

#include "drg_bitmap.hpp"
#include "drg_internal.hpp"

namespace drg {

__global__ void k_prio(int32_t n, uint64_t seed, int32_t level, uint64_t* __restrict__ pri) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    pri[v] = philox4x64((uint64_t)(uint32_t)v, (uint64_t)(uint32_t)level, 0, 0, seed, TAG_COARSEN)
                 .w[0];
}

__device__ __forceinline__ bool outranks(uint64_t pu, int32_t u, uint64_t pv, int32_t v) {
    return pu > pv || (pu == pv && u < v);
}

// state: 0 undecided, 1 centre, 2 member.  Decisions are final, so reading a
// neighbour's state while it is being written only delays a decision.
__global__ void k_mis_round(int32_t n, const int32_t* __restrict__ rp,
                            const int32_t* __restrict__ col, const uint64_t* __restrict__ pri,
                            int32_t* state, int32_t* __restrict__ undecided) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    volatile int32_t* vs = state;
    if (vs[v] != 0) return;
    const uint64_t pv = pri[v];
    bool wait = false;
    for (int32_t x = rp[v]; x < rp[v + 1]; ++x) {
        const int32_t u = col[x];
        if (!outranks(pri[u], u, pv, (int32_t)v)) continue;
        const int32_t su = vs[u];
        if (su == 1) {
            vs[v] = 2;
            return;
        }
        if (su == 0) wait = true;
    }
    if (!wait)
        vs[v] = 1;
    else
        *undecided = 1;
}

__global__ void k_owner(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                        const uint64_t* __restrict__ pri, const int32_t* __restrict__ state,
                        int32_t* __restrict__ owner, int32_t* __restrict__ is_centre) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    if (state[v] == 1) {
        owner[v] = (int32_t)v;
        is_centre[v] = 1;
        return;
    }
    int32_t best = -1;
    uint64_t pb = 0;
    for (int32_t x = rp[v]; x < rp[v + 1]; ++x) {
        const int32_t u = col[x];
        if (state[u] != 1) continue;
        const uint64_t pu = pri[u];
        if (best < 0 || outranks(pu, u, pb, best)) {
            best = u;
            pb = pu;
        }
    }
    owner[v] = best;
    is_centre[v] = 0;
}

__global__ void k_map(int32_t n, const int32_t* __restrict__ owner, const int32_t* __restrict__ rank,
                      int32_t* __restrict__ map) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) map[v] = rank[owner[v]];
}

__global__ void k_iota_keys(int32_t n, const int32_t* __restrict__ map, uint32_t* __restrict__ keys,
                            int32_t* __restrict__ vals) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    keys[v] = (uint32_t)map[v];
    vals[v] = (int32_t)v;
}

// seg[c] = first position of a key >= c in the sorted keys, c = 0..nc
__global__ void k_seg_bounds(int32_t n, int32_t nc, const uint32_t* __restrict__ keys,
                             int32_t* __restrict__ seg) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c > nc) return;
    int32_t lo = 0, hi = n;
    while (lo < hi) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        if ((int64_t)keys[mid] < c)
            lo = mid + 1;
        else
            hi = mid;
    }
    seg[c] = lo;
}

__global__ void k_compose(int32_t n0, const int32_t* __restrict__ prev,
                          const int32_t* __restrict__ map, int32_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n0) out[i] = map[prev[i]];
}

constexpr int CT_BLOCK = 256;
constexpr int CT_WPT = 8;

struct ContractArgs {
    int32_t nc, nwords;
    const int32_t* rp;
    const int32_t* col;
    const int32_t* map;
    const int32_t* perm;   // fine nodes grouped by coarse node
    const int32_t* seg;    // [nc+1]
    int32_t* cnt;          // count pass: [nc]
    const int32_t* crp;    // fill pass: [nc+1]
    int32_t* ccol;         // fill pass
    uint32_t* gbm;
    int32_t* work;
};

template <bool FILL, bool LDS_BM, int G>
__global__ __launch_bounds__(CT_BLOCK) void k_contract(ContractArgs a) {
    extern __shared__ uint32_t s_bm[];
    __shared__ int32_t s_c;
    __shared__ int32_t s_red[CT_BLOCK / WAVE];
    uint32_t* bm = LDS_BM ? s_bm : a.gbm + (size_t)blockIdx.x * (size_t)a.nwords;
    const int tid = threadIdx.x;
    for (int w = tid; w < a.nwords; w += CT_BLOCK) bm[w] = 0;
    __syncthreads();
    for (;;) {
        if (tid == 0) s_c = atomicAdd(a.work, 1);
        __syncthreads();
        const int32_t c = s_c;
        if (c >= a.nc) break;
        const int32_t mb = a.seg[c], me = a.seg[c + 1];
        for (int32_t fi = tid / G; fi < me - mb; fi += CT_BLOCK / G) {
            const int32_t u = a.perm[mb + fi];
            for (int32_t x = a.rp[u] + (tid % G); x < a.rp[u + 1]; x += G) {
                const int32_t t = a.map[a.col[x]];
                if (t != c) atomicOr(&bm[t >> 5], 1u << (t & 31));
            }
        }
        __syncthreads();
        if constexpr (!FILL) {
            const int total = bitmap_count_clear<CT_BLOCK>(bm, a.nwords, s_red);
            if (tid == 0) a.cnt[c] = total;
        } else {
            int32_t* out = a.ccol;
            bitmap_emit_clear<CT_BLOCK, CT_WPT>(bm, a.nwords, -1, (int64_t)a.crp[c], s_red,
                                               [&](int64_t o, uint32_t v) { out[o] = (int32_t)v; });
        }
        __syncthreads();
    }
}

template <bool FILL, bool LDS_BM>
static void launch_contract(drg_ctx* ctx, const ContractArgs& a, int G, int grid, size_t lds) {
#define DRG_CT_CASE(GG)                                                                         \
    case GG: {                                                                                  \
        auto fn = k_contract<FILL, LDS_BM, GG>;                                                 \
        if (LDS_BM)                                                                             \
            DRG_HIP(hipFuncSetAttribute((const void*)fn,                                        \
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)); \
        hipLaunchKernelGGL(fn, dim3(grid), dim3(CT_BLOCK), LDS_BM ? lds : 0, ctx->stream, a);   \
        break;                                                                                  \
    }
    switch (G) {
        DRG_CT_CASE(4)
        DRG_CT_CASE(16)
        default:
        DRG_CT_CASE(64)
    }
#undef DRG_CT_CASE
    DRG_LAUNCH_CHECK();
}

static int key_bits_for(int64_t nc) {
    int b = 1;
    while (b < 32 && ((int64_t)1 << b) < nc) ++b;
    return b;
}

// Groups the n nodes by key map[] (ascending node id inside each group).
static void group_by(drg_ctx* ctx, int32_t n, int32_t nc, const int32_t* map, int32_t* perm,
                     int32_t* seg) {
    hipStream_t st = ctx->stream;
    DevBuf<uint32_t> keys(n);
    hipLaunchKernelGGL(k_iota_keys, dim3(ceil_div(n, 256)), dim3(256), 0, st, n, map, keys.get(),
                       perm);
    DRG_LAUNCH_CHECK();
    radix_sort_pairs(keys.get(), perm, n, key_bits_for(nc), st);
    hipLaunchKernelGGL(k_seg_bounds, dim3(ceil_div((int64_t)nc + 1, 256)), dim3(256), 0, st, n, nc,
                       keys.get(), seg);
    DRG_LAUNCH_CHECK();
    DRG_HIP(hipStreamSynchronize(st));
}

// One level: map (n -> nc) and the contracted graph.
static void coarsen_one(drg_ctx* ctx, int32_t n, const int32_t* rp, const int32_t* col,
                        int64_t nnz, uint64_t seed, int32_t level, drg_level& out) {
    hipStream_t st = ctx->stream;
    DevBuf<uint64_t> pri(n);
    DevBuf<int32_t> state(n), owner(n), is_centre(n), rank((int64_t)n + 1), flag(1);
    hipLaunchKernelGGL(k_prio, dim3(ceil_div(n, 256)), dim3(256), 0, st, n, seed, level,
                       pri.get());
    DRG_LAUNCH_CHECK();
    DRG_HIP(hipMemsetAsync(state.get(), 0, sizeof(int32_t) * n, st));
    for (int round = 0;; ++round) {
        if (round > 100000) throw Error(DRG_E_DEVICE, "coarsening did not converge");
        DRG_HIP(hipMemsetAsync(flag.get(), 0, sizeof(int32_t), st));
        hipLaunchKernelGGL(k_mis_round, dim3(ceil_div(n, 256)), dim3(256), 0, st, n, rp, col,
                           pri.get(), state.get(), flag.get());
        DRG_LAUNCH_CHECK();
        int32_t h = 0;
        DRG_HIP(hipMemcpyAsync(&h, flag.get(), sizeof(int32_t), hipMemcpyDeviceToHost, st));
        DRG_HIP(hipStreamSynchronize(st));
        if (!h) break;
    }
    hipLaunchKernelGGL(k_owner, dim3(ceil_div(n, 256)), dim3(256), 0, st, n, rp, col, pri.get(),
                       state.get(), owner.get(), is_centre.get());
    DRG_LAUNCH_CHECK();
    exclusive_scan<int32_t>(is_centre.get(), rank.get(), n, st);
    int32_t nc = 0;
    DRG_HIP(hipMemcpyAsync(&nc, rank.get() + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    DRG_HIP(hipStreamSynchronize(st));
    out.n = nc;
    out.map.alloc(n);
    hipLaunchKernelGGL(k_map, dim3(ceil_div(n, 256)), dim3(256), 0, st, n, owner.get(),
                       rank.get(), out.map.get());
    DRG_LAUNCH_CHECK();
    // members of each coarse node, then the contracted adjacency
    DevBuf<int32_t> perm(n), seg((int64_t)nc + 1), cnt(nc);
    group_by(ctx, n, nc, out.map.get(), perm.get(), seg.get());
    const int nwords = (nc + 31) / 32;
    const size_t lds = (size_t)nwords * 4;
    const bool in_lds = lds + 256 <= (size_t)ctx->max_lds;
    int per_cu = in_lds ? std::max(1, (int)(ctx->max_lds / (lds + 256))) : 4;
    per_cu = std::min(per_cu, 8);
    const int grid = std::max(1, std::min<int>(ctx->num_cu * per_cu, nc));
    DevBuf<uint32_t> gbm;
    if (!in_lds) gbm.alloc((int64_t)grid * nwords);
    DevBuf<int32_t> work(1);
    const double mean_deg = n > 0 ? (double)nnz / n : 1.0;
    const int G = mean_deg <= 6 ? 4 : (mean_deg <= 24 ? 16 : 64);
    ContractArgs a{};
    a.nc = nc;
    a.nwords = nwords;
    a.rp = rp;
    a.col = col;
    a.map = out.map.get();
    a.perm = perm.get();
    a.seg = seg.get();
    a.cnt = cnt.get();
    a.gbm = gbm.get();
    a.work = work.get();
    DRG_HIP(hipMemsetAsync(work.get(), 0, sizeof(int32_t), st));
    if (in_lds)
        launch_contract<false, true>(ctx, a, G, grid, lds);
    else
        launch_contract<false, false>(ctx, a, G, grid, 0);
    out.rp.alloc((int64_t)nc + 1);
    exclusive_scan<int32_t>(cnt.get(), out.rp.get(), nc, st);
    int32_t cnnz = 0;
    DRG_HIP(hipMemcpyAsync(&cnnz, out.rp.get() + nc, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    DRG_HIP(hipStreamSynchronize(st));
    out.nnz = cnnz;
    out.col.alloc(cnnz);
    a.crp = out.rp.get();
    a.ccol = out.col.get();
    DRG_HIP(hipMemsetAsync(work.get(), 0, sizeof(int32_t), st));
    if (in_lds)
        launch_contract<true, true>(ctx, a, G, grid, lds);
    else
        launch_contract<true, false>(ctx, a, G, grid, 0);
    DRG_HIP(hipStreamSynchronize(st));
    out.n_active = (int32_t)count_nonempty_rows<int32_t>(out.rp.get(), nc, st);
}

void validate_csr_impl(drg_ctx* ctx, const drg_csr* g, bool full);

drg_hier* build_hierarchy(drg_ctx* ctx, const drg_csr* g, uint64_t seed, double rho,
                          int min_nodes, int max_levels) {
    if (!g) throw Error(DRG_E_INVALID, "graph is NULL");
    if (!(rho > 0.0 && rho <= 1.0)) throw Error(DRG_E_INVALID, "rho must be in (0, 1]");
    if (max_levels < 1) throw Error(DRG_E_INVALID, "max_levels must be >= 1");
    if (min_nodes < 0) throw Error(DRG_E_INVALID, "min_nodes must be >= 0");
    if (g->n <= 0 || g->n >= (1 << 30)) throw Error(DRG_E_INVALID, "n must be in 1..2^30-1");
    if (g->nnz < 0 || !g->row_ptr || (g->nnz > 0 && !g->col))
        throw Error(DRG_E_INVALID, "bad CSR pointers or nnz");
    validate_csr_impl(ctx, g, false);
    hipStream_t st = ctx->stream;
    auto h = std::make_unique<drg_hier>();
    h->device = ctx->device;
    h->n0 = g->n;
    h->lv.emplace_back();
    h->lv[0].n = g->n;
    h->lv[0].nnz = g->nnz;
    h->lv[0].n_active = (int32_t)count_nonempty_rows<int32_t>(g->row_ptr, g->n, st);
    while ((int)h->lv.size() < max_levels) {
        drg_level& cur = h->lv.back();
        const int32_t na = cur.n_active;
        if (na == 0 || na < min_nodes) break;
        const int32_t l = (int32_t)h->lv.size() - 1;
        const int32_t* rp = l == 0 ? g->row_ptr : cur.rp.get();
        const int32_t* col = l == 0 ? g->col : cur.col.get();
        drg_level nxt;
        coarsen_one(ctx, cur.n, rp, col, cur.nnz, seed, l, nxt);
        if ((double)nxt.n_active > rho * (double)na) break;
        nxt.cmap.alloc(h->n0);
        if (l == 0) {
            DRG_HIP(hipMemcpyAsync(nxt.cmap.get(), nxt.map.get(), sizeof(int32_t) * h->n0,
                                   hipMemcpyDeviceToDevice, st));
        } else {
            hipLaunchKernelGGL(k_compose, dim3(ceil_div(h->n0, 256)), dim3(256), 0, st, h->n0,
                               cur.cmap.get(), nxt.map.get(), nxt.cmap.get());
            DRG_LAUNCH_CHECK();
        }
        nxt.perm.alloc(h->n0);
        nxt.seg.alloc((int64_t)nxt.n + 1);
        group_by(ctx, h->n0, nxt.n, nxt.cmap.get(), nxt.perm.get(), nxt.seg.get());
        h->lv.push_back(std::move(nxt));
    }
    DRG_HIP(hipStreamSynchronize(st));
    return h.release();
}

}  // namespace drg
