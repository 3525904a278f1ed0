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
// The coarse graph keeps one edge between two groups joined by a fine edge:
// every fine edge becomes the pair (group of u, group of v), the pairs are
// sorted and the first of each run of equal pairs is kept, so every coarse
// row comes out ascending and free of duplicates.
#include <memory>

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

// the better of two owner candidates (b = -1: none)
__device__ __forceinline__ void owner_better(uint64_t& pb, int32_t& b, uint64_t pu, int32_t u) {
    if (u >= 0 && (b < 0 || outranks(pu, u, pb, b))) {
        b = u;
        pb = pu;
    }
}

// Every non-centre joins the highest-priority centre among its neighbours
// (-1 if none).  One lane per node; a node with more than OWNER_SEQ
// neighbours (an R-MAT hub) is scanned by the whole wave, lane l taking
// neighbours l, l+64, ..., then a butterfly of the candidates: the order of
// a maximum does not change it.
constexpr int OWNER_SEQ = 64;

__global__ __launch_bounds__(256) void k_owner(int32_t n, const int32_t* __restrict__ rp,
                                               const int32_t* __restrict__ col,
                                               const uint64_t* __restrict__ pri,
                                               const int32_t* __restrict__ state,
                                               int32_t* __restrict__ owner,
                                               int32_t* __restrict__ is_centre) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = v < n;
    if (__ballot(valid) == 0) return;  // the whole wave leaves
    const int lane = __lane_id();
    const int32_t rs = valid ? rp[v] : 0, re = valid ? rp[v + 1] : 0;
    const bool centre = valid && state[v] == 1;
    const bool big = valid && !centre && re - rs > OWNER_SEQ;
    int32_t best = -1;
    uint64_t pb = 0;
    if (valid && !centre && !big) {
        for (int32_t x = rs; x < re; ++x) {
            const int32_t u = col[x];
            if (state[u] == 1) owner_better(pb, best, pri[u], u);
        }
    }
    uint64_t m = __ballot(big);
    while (m) {
        const int src = __ffsll((unsigned long long)m) - 1;
        m &= m - 1;
        const int32_t b0 = __builtin_amdgcn_readlane(rs, src);
        const int32_t b1 = __builtin_amdgcn_readlane(re, src);
        int32_t wb = -1;
        uint64_t wp = 0;
        for (int32_t x = b0 + lane; x < b1; x += WAVE) {
            const int32_t u = col[x];
            if (state[u] == 1) owner_better(wp, wb, pri[u], u);
        }
        for (int off = WAVE / 2; off > 0; off >>= 1) {
            const uint32_t lo = __shfl_xor((uint32_t)wp, off);
            const uint32_t hi = __shfl_xor((uint32_t)(wp >> 32), off);
            const int32_t ob = __shfl_xor(wb, off);
            owner_better(wp, wb, ((uint64_t)hi << 32) | lo, ob);
        }
        if (lane == src) {
            best = wb;
            pb = wp;
        }
    }
    if (!valid) return;
    owner[v] = centre ? (int32_t)v : best;
    is_centre[v] = centre ? 1 : 0;
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

// (group of u, group of v) of every fine edge, one wave per fine row; a pair
// inside one group gets c = nc, which sorts after every kept pair
__global__ __launch_bounds__(256) void k_edge_pairs(int32_t n, int32_t nc,
                                                    const int32_t* __restrict__ rp,
                                                    const int32_t* __restrict__ col,
                                                    const int32_t* __restrict__ map,
                                                    uint32_t* __restrict__ t_out,
                                                    int32_t* __restrict__ c_out) {
    const int lane = __lane_id();
    const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const int64_t nw = (int64_t)gridDim.x * blockDim.x / WAVE;
    for (int64_t u = w0; u < n; u += nw) {
        const int32_t c = map[u];
        for (int32_t x = rp[u] + lane; x < rp[u + 1]; x += WAVE) {
            const int32_t t = map[col[x]];
            const bool self = t == c;
            t_out[x] = self ? 0u : (uint32_t)t;
            c_out[x] = self ? nc : c;
        }
    }
}

// head[x] = 1 for the first of each run of equal (c, t) pairs with c < nc
__global__ void k_pair_heads(int64_t m, int32_t nc, const uint32_t* __restrict__ c,
                             const int32_t* __restrict__ t, int32_t* __restrict__ head) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= m) return;
    head[x] = (c[x] < (uint32_t)nc && (x == 0 || c[x] != c[x - 1] || t[x] != t[x - 1])) ? 1 : 0;
}

__global__ void k_pair_emit(int64_t m, const uint32_t* __restrict__ c,
                            const int32_t* __restrict__ t, const int32_t* __restrict__ head,
                            const int32_t* __restrict__ pos, uint32_t* __restrict__ ck,
                            int32_t* __restrict__ ccol) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= m || !head[x]) return;
    ck[pos[x]] = c[x];
    ccol[pos[x]] = t[x];
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

// A union of graphs being coarsened together: node v belongs to graph
// gid[v], whose nodes start at gbase[gid[v]] (device arrays indexed by graph).
struct UnionLevel {
    const int32_t* gid = nullptr;
    const int32_t* gbase = nullptr;
    const uint64_t* gseed = nullptr;
    std::vector<int32_t> members;   // graphs of the union, ascending
    std::vector<int32_t> hbase;     // [count] node base of each member (host)
    std::vector<int32_t> hn;        // [count] node count of each member (host)
    // out
    std::vector<int32_t> cbase, cn; // [count] coarse base and size of each member
    DevBuf<int32_t> cgid;           // [nc] graph of each coarse node
};

__global__ void k_prio_union(int32_t n, const int32_t* __restrict__ gid,
                             const int32_t* __restrict__ gbase, const uint64_t* __restrict__ gseed,
                             int32_t level, uint64_t* __restrict__ pri) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t c = gid[v];
    pri[v] = philox4x64((uint64_t)(uint32_t)((int32_t)v - gbase[c]), (uint64_t)(uint32_t)level, 0,
                        0, gseed[c], TAG_COARSEN)
                 .w[0];
}

// graph of every coarse node: all members of a group belong to one graph,
// so every member writes the same value
__global__ void k_coarse_gid(int32_t n, const int32_t* __restrict__ map,
                             const int32_t* __restrict__ gid, int32_t* __restrict__ cgid) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) cgid[map[v]] = gid[v];
}

__global__ void k_gather_i32(int32_t m, const int32_t* __restrict__ at,
                             const int32_t* __restrict__ src, int32_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) out[i] = src[at[i]];
}

template <typename T>
static void to_dev(DevBuf<T>& d, const std::vector<T>& h, hipStream_t st) {
    d.alloc((int64_t)h.size());
    if (!h.empty())
        DRG_HIP(hipMemcpyAsync(d.get(), h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice, st));
}

// One level: map (n -> nc) and the contracted graph.  With u, the graphs of
// a union are coarsened at once: priorities are keyed by each graph's own
// node ids and seed, coarse ids of a graph are contiguous (its centres in id
// order), and map values and coarse columns are union coarse ids.
static void coarsen_one(drg_ctx* ctx, int32_t n, const int32_t* rp, const int32_t* col,
                        int64_t nnz, uint64_t seed, int32_t level, drg_level& out,
                        UnionLevel* u = nullptr) {
    hipStream_t st = ctx->stream;
    DevBuf<uint64_t> pri(n);
    DevBuf<int32_t> state(n), owner(n), is_centre(n), rank((int64_t)n + 1), flag(1);
    if (u)
        hipLaunchKernelGGL(k_prio_union, dim3(ceil_div(n, 256)), dim3(256), 0, st, n, u->gid,
                           u->gbase, u->gseed, level, pri.get());
    else
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
    if (u) {
        // coarse base of every member graph = rank of its first node
        const int32_t m = (int32_t)u->members.size();
        std::vector<int32_t> at(2 * m);
        for (int32_t i = 0; i < m; ++i) {
            const int32_t c = u->members[i];
            at[2 * i] = u->hbase[c];
            at[2 * i + 1] = u->hbase[c] + u->hn[c];
        }
        DevBuf<int32_t> dat, dv(2 * m);
        to_dev(dat, at, st);
        hipLaunchKernelGGL(k_gather_i32, dim3(ceil_div(2 * m, 256)), dim3(256), 0, st, 2 * m,
                           dat.get(), rank.get(), dv.get());
        DRG_LAUNCH_CHECK();
        std::vector<int32_t> hv(2 * m);
        DRG_HIP(hipMemcpyAsync(hv.data(), dv.get(), sizeof(int32_t) * 2 * m,
                               hipMemcpyDeviceToHost, st));
        DRG_HIP(hipStreamSynchronize(st));
        const int32_t count = (int32_t)u->hbase.size();
        u->cbase.assign(count, -1);
        u->cn.assign(count, 0);
        for (int32_t i = 0; i < m; ++i) {
            const int32_t c = u->members[i];
            u->cbase[c] = hv[2 * i];
            u->cn[c] = hv[2 * i + 1] - hv[2 * i];
        }
        u->cgid.alloc(nc);
        hipLaunchKernelGGL(k_coarse_gid, dim3(ceil_div(n, 256)), dim3(256), 0, st, n,
                           out.map.get(), u->gid, u->cgid.get());
        DRG_LAUNCH_CHECK();
    }
    // the contracted adjacency: (c, t) pairs of all fine edges, sorted by t
    // then (stably) by c, the first of each run kept
    out.rp.alloc((int64_t)nc + 1);
    DevBuf<uint32_t> tk(std::max<int64_t>(nnz, 1));
    DevBuf<int32_t> cv(std::max<int64_t>(nnz, 1));
    if (nnz > 0) {
        const int grid = (int)std::max<int64_t>(
            1, std::min<int64_t>(ceil_div((int64_t)n * WAVE, 256), (int64_t)ctx->num_cu * 32));
        hipLaunchKernelGGL(k_edge_pairs, dim3(grid), dim3(256), 0, st, n, nc, rp, col,
                           out.map.get(), tk.get(), cv.get());
        DRG_LAUNCH_CHECK();
        radix_sort_pairs(tk.get(), cv.get(), nnz, key_bits_for(nc), st);
        // now sort by c: keys and values swap roles
        uint32_t* ck = reinterpret_cast<uint32_t*>(cv.get());
        int32_t* tv = reinterpret_cast<int32_t*>(tk.get());
        radix_sort_pairs(ck, tv, nnz, key_bits_for((int64_t)nc + 1), st);
        DevBuf<int32_t> head(nnz), pos(nnz + 1);
        hipLaunchKernelGGL(k_pair_heads, dim3(ceil_div(nnz, 256)), dim3(256), 0, st, nnz, nc, ck,
                           tv, head.get());
        DRG_LAUNCH_CHECK();
        exclusive_scan<int32_t>(head.get(), pos.get(), nnz, st);
        int32_t cnnz = 0;
        DRG_HIP(hipMemcpyAsync(&cnnz, pos.get() + nnz, sizeof(int32_t), hipMemcpyDeviceToHost,
                               st));
        DRG_HIP(hipStreamSynchronize(st));
        out.nnz = cnnz;
        out.col.alloc(std::max(cnnz, 1));
        DevBuf<uint32_t> crow(std::max(cnnz, 1));
        hipLaunchKernelGGL(k_pair_emit, dim3(ceil_div(nnz, 256)), dim3(256), 0, st, nnz, ck, tv,
                           head.get(), pos.get(), crow.get(), out.col.get());
        DRG_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_seg_bounds, dim3(ceil_div((int64_t)nc + 1, 256)), dim3(256), 0, st,
                           cnnz, nc, crow.get(), out.rp.get());
        DRG_LAUNCH_CHECK();
    } else {
        out.nnz = 0;
        out.col.alloc(1);
        DRG_HIP(hipMemsetAsync(out.rp.get(), 0, sizeof(int32_t) * ((int64_t)nc + 1), st));
    }
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

// ------------------------------------------------------------------ unions
// Keeps the graphs with nb[c] >= 0: node v of graph c becomes nb[c] + (v -
// ob[c]), its row moves by ne[c] - oe[c] and its columns by nb[c] - ob[c].
__global__ void k_compact(int32_t n, const int32_t* __restrict__ gid,
                          const int32_t* __restrict__ ob, const int32_t* __restrict__ nb,
                          const int32_t* __restrict__ oe, const int32_t* __restrict__ ne,
                          const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                          int32_t* __restrict__ nrp, int32_t* __restrict__ ncol,
                          int32_t* __restrict__ ngid) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t c = gid[v];
    if (nb[c] < 0) return;
    const int32_t nv = nb[c] + ((int32_t)v - ob[c]);
    const int32_t eoff = ne[c] - oe[c], voff = nb[c] - ob[c];
    nrp[nv] = rp[v] + eoff;
    ngid[nv] = c;
    for (int32_t x = rp[v]; x < rp[v + 1]; ++x) ncol[x + eoff] = col[x] + voff;
}

// map pool entry of every node of a kept graph: its coarse id, graph-local.
__global__ void k_store_map(int32_t n, const int32_t* __restrict__ gid,
                            const int32_t* __restrict__ vb, const int32_t* __restrict__ cb,
                            const int64_t* __restrict__ mo, const int32_t* __restrict__ map,
                            int32_t* __restrict__ pool) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t c = gid[v];
    if (mo[c] < 0) return;
    pool[mo[c] + ((int32_t)v - vb[c])] = map[v] - cb[c];
}

// cmap_l(j) = map_l(cmap_{l-1}(j)) for the finest nodes of kept graphs, and
// the sort key (graph's first level-l union id + cmap) of every finest node.
__global__ void k_compose_union(int32_t n0, const int32_t* __restrict__ gid0,
                                const int32_t* __restrict__ base0,
                                const int64_t* __restrict__ prev_co,
                                const int32_t* __restrict__ prev_cmap,
                                const int64_t* __restrict__ mo, const int32_t* __restrict__ mpool,
                                const int64_t* __restrict__ co, const int32_t* __restrict__ kb,
                                int32_t* __restrict__ cpool, uint32_t* __restrict__ keys,
                                int32_t* __restrict__ vals) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n0) return;
    const int32_t c = gid0[j];
    vals[j] = (int32_t)j;
    if (co[c] < 0) {
        keys[j] = 0xFFFFFFFFu;
        return;
    }
    const int32_t loc = (int32_t)j - base0[c];
    const int32_t prev = prev_cmap ? prev_cmap[prev_co[c] + loc] : loc;
    const int32_t cm = mpool[mo[c] + prev];
    cpool[co[c] + loc] = cm;
    keys[j] = (uint32_t)(kb[c] + cm);
}

// perm pool: the sorted finest members, graph-local.
__global__ void k_store_perm(int32_t m, const int32_t* __restrict__ vals,
                             const int32_t* __restrict__ gid0, const int32_t* __restrict__ base0,
                             int32_t* __restrict__ ppool) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= m) return;
    const int32_t j = vals[x];
    ppool[x] = j - base0[gid0[j]];
}

// seg pool: member offsets of every level node of a kept graph, relative to
// the graph's first member; the entry after a graph's last node is n_0.
__global__ void k_store_seg(int32_t nl, int32_t m, const int32_t* __restrict__ kgraph,
                            const int32_t* __restrict__ kbk, int32_t nk,
                            const uint32_t* __restrict__ keys, const int64_t* __restrict__ co,
                            const int64_t* __restrict__ so, const int32_t* __restrict__ n0,
                            int32_t* __restrict__ spool) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= nl) return;
    // kept graph owning level-node u: last i with kbk[i] <= u
    int32_t lo = 0, hi = nk - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if ((int64_t)kbk[mid] <= u)
            lo = mid;
        else
            hi = mid - 1;
    }
    const int32_t c = kgraph[lo];
    const int32_t a = (int32_t)u - kbk[lo];
    int32_t l = 0, h = m;  // first sorted key >= u
    while (l < h) {
        const int32_t mid = l + ((h - l) >> 1);
        if ((int64_t)keys[mid] < u)
            l = mid + 1;
        else
            h = mid;
    }
    spool[so[c] + a] = l - (int32_t)co[c];
    const bool last = (lo + 1 < nk) ? (u + 1 == kbk[lo + 1]) : (u + 1 == nl);
    if (last) spool[so[c] + a + 1] = n0[c];
}

// Level-synchronous: level l of every graph that still coarsens is built in
// one pass over the union of their level l-1 graphs.  A graph stops exactly
// where build_hierarchy stops it (max_levels, min_nodes, no active node, or
// too little reduction); graphs leave the union as they stop.
void build_hierarchy_union(drg_ctx* ctx, const drg_csr* g, const int32_t* gid,
                           const std::vector<int32_t>& base, const drg_layout_params* params,
                           UnionHier& out) {
    hipStream_t st = ctx->stream;
    const int32_t count = (int32_t)base.size() - 1;
    const int32_t N0 = g->n;
    out.lv.clear();
    out.lv.emplace_back();
    out.n.assign(count, {});
    for (int32_t c = 0; c < count; ++c) out.n[c].push_back(base[c + 1] - base[c]);
    std::vector<uint64_t> seeds(count);
    for (int32_t c = 0; c < count; ++c) seeds[c] = params[c].seed;
    DevBuf<uint64_t> dseed;
    DevBuf<int32_t> dbase0, dn0;
    to_dev(dseed, seeds, st);
    to_dev(dbase0, base, st);
    {
        std::vector<int32_t> n0(count);
        for (int32_t c = 0; c < count; ++c) n0[c] = out.n[c][0];
        to_dev(dn0, n0, st);
    }
    // current union (level l-1)
    int32_t cn = N0;
    int64_t cnnz = g->nnz;
    const int32_t* crp = g->row_ptr;
    const int32_t* ccol = g->col;
    const int32_t* cgid = gid;
    DevBuf<int32_t> own_rp, own_col, own_gid;
    std::vector<int32_t> vb(base.begin(), base.end() - 1), vn(count), ve(count), vm(count);
    std::vector<int32_t> na(count, 0);
    {
        std::vector<int32_t> rpb(count + 1);
        for (int32_t c = 0; c <= count; ++c)
            DRG_HIP(hipMemcpyAsync(&rpb[c], g->row_ptr + base[c], sizeof(int32_t),
                                   hipMemcpyDeviceToHost, st));
        DevBuf<int32_t> cnt(count);
        count_nonempty_by_group<int32_t>(g->row_ptr, gid, N0, cnt.get(), count, st);
        DRG_HIP(hipMemcpyAsync(na.data(), cnt.get(), sizeof(int32_t) * count,
                               hipMemcpyDeviceToHost, st));
        DRG_HIP(hipStreamSynchronize(st));
        for (int32_t c = 0; c < count; ++c) {
            vn[c] = out.n[c][0];
            ve[c] = rpb[c];
            vm[c] = rpb[c + 1] - rpb[c];
        }
    }
    std::vector<char> member(count, 1);
    for (int32_t l = 1;; ++l) {
        // graphs that try one more level
        std::vector<int32_t> E;
        for (int32_t c = 0; c < count; ++c)
            if (member[c] && l < params[c].max_levels && na[c] > 0 && na[c] >= params[c].min_nodes)
                E.push_back(c);
        if (E.empty()) break;
        // drop the others from the union
        auto compact = [&](const std::vector<char>& keep) {
            std::vector<int32_t> nb(count, -1), ne(count, -1), ob(count, 0), oe(count, 0);
            int32_t tn = 0, te = 0;
            for (int32_t c = 0; c < count; ++c) {
                ob[c] = member[c] ? vb[c] : 0;
                oe[c] = member[c] ? ve[c] : 0;
                if (member[c] && keep[c]) {
                    nb[c] = tn;
                    ne[c] = te;
                    tn += vn[c];
                    te += vm[c];
                }
            }
            DevBuf<int32_t> dob, dnb, doe, dne, nrp((int64_t)tn + 1), ncol(te), ngid(tn);
            to_dev(dob, ob, st);
            to_dev(dnb, nb, st);
            to_dev(doe, oe, st);
            to_dev(dne, ne, st);
            hipLaunchKernelGGL(k_compact, dim3(ceil_div(cn, 256)), dim3(256), 0, st, cn, cgid,
                               dob.get(), dnb.get(), doe.get(), dne.get(), crp, ccol, nrp.get(),
                               ncol.get(), ngid.get());
            DRG_LAUNCH_CHECK();
            DRG_HIP(hipMemcpyAsync(nrp.get() + tn, &te, sizeof(int32_t), hipMemcpyHostToDevice,
                                   st));
            DRG_HIP(hipStreamSynchronize(st));
            own_rp = std::move(nrp);
            own_col = std::move(ncol);
            own_gid = std::move(ngid);
            crp = own_rp.get();
            ccol = own_col.get();
            cgid = own_gid.get();
            cn = tn;
            cnnz = te;
            for (int32_t c = 0; c < count; ++c) {
                if (!(member[c] && keep[c])) member[c] = 0;
                if (member[c]) {
                    vb[c] = nb[c];
                    ve[c] = ne[c];
                }
            }
        };
        if ((int32_t)E.size() != (int32_t)std::count(member.begin(), member.end(), 1)) {
            std::vector<char> keep(count, 0);
            for (int32_t c : E) keep[c] = 1;
            compact(keep);
        }
        // coarsen the union of E
        UnionLevel u;
        DevBuf<int32_t> dvb;
        to_dev(dvb, vb, st);
        u.gid = cgid;
        u.gbase = dvb.get();
        u.gseed = dseed.get();
        u.members = E;
        u.hbase = vb;
        u.hn = vn;
        drg_level nxt;
        coarsen_one(ctx, cn, crp, ccol, cnnz, 0, l - 1, nxt, &u);
        // active nodes of every coarse graph; keep the ones that shrank enough
        std::vector<int32_t> nna(count, 0);
        {
            DevBuf<int32_t> cnt(count);
            count_nonempty_by_group<int32_t>(nxt.rp.get(), u.cgid.get(), nxt.n, cnt.get(), count,
                                             st);
            DRG_HIP(hipMemcpyAsync(nna.data(), cnt.get(), sizeof(int32_t) * count,
                                   hipMemcpyDeviceToHost, st));
        }
        std::vector<int32_t> cedge(count, 0), cerow(count, 0);
        {
            // coarse edge range of every graph: rows cbase .. cbase + cn
            for (int32_t c : E) {
                DRG_HIP(hipMemcpyAsync(&cerow[c], nxt.rp.get() + u.cbase[c], sizeof(int32_t),
                                       hipMemcpyDeviceToHost, st));
                DRG_HIP(hipMemcpyAsync(&cedge[c], nxt.rp.get() + u.cbase[c] + u.cn[c],
                                       sizeof(int32_t), hipMemcpyDeviceToHost, st));
            }
            DRG_HIP(hipStreamSynchronize(st));
        }
        std::vector<int32_t> K;
        std::vector<char> keep(count, 0);
        for (int32_t c : E)
            if (!((double)nna[c] > params[c].rho * (double)na[c])) {
                K.push_back(c);
                keep[c] = 1;
            }
        if (K.empty()) break;
        // level l pools of the kept graphs
        UnionHier::Pool P;
        P.mo.assign(count, -1);
        P.co.assign(count, -1);
        P.so.assign(count, -1);
        std::vector<int32_t> kb(count, 0), kgraph, kbk;
        int64_t tm = 0, tc = 0, ts = 0;
        int32_t tl = 0;
        for (int32_t c : K) {
            P.mo[c] = tm;
            P.co[c] = tc;
            P.so[c] = ts;
            kb[c] = tl;
            kgraph.push_back(c);
            kbk.push_back(tl);
            tm += vn[c];
            tc += out.n[c][0];
            ts += u.cn[c] + 1;
            tl += u.cn[c];
        }
        P.map.alloc(tm);
        P.cmap.alloc(tc);
        P.perm.alloc(tc);
        P.seg.alloc(ts);
        DevBuf<int64_t> dmo, dco, dso, dpco;
        DevBuf<int32_t> dcb, dkb, dkg, dkbk;
        to_dev(dmo, P.mo, st);
        to_dev(dco, P.co, st);
        to_dev(dso, P.so, st);
        to_dev(dcb, u.cbase, st);
        to_dev(dkb, kb, st);
        to_dev(dkg, kgraph, st);
        to_dev(dkbk, kbk, st);
        hipLaunchKernelGGL(k_store_map, dim3(ceil_div(cn, 256)), dim3(256), 0, st, cn, cgid,
                           dvb.get(), dcb.get(), dmo.get(), nxt.map.get(), P.map.get());
        DRG_LAUNCH_CHECK();
        const UnionHier::Pool* prev = l >= 2 ? &out.lv[l - 1] : nullptr;
        if (prev) to_dev(dpco, prev->co, st);
        DevBuf<uint32_t> keys(N0);
        DevBuf<int32_t> vals(N0);
        hipLaunchKernelGGL(k_compose_union, dim3(ceil_div(N0, 256)), dim3(256), 0, st, N0, gid,
                           dbase0.get(), prev ? dpco.get() : nullptr,
                           prev ? prev->cmap.get() : nullptr, dmo.get(), P.map.get(), dco.get(),
                           dkb.get(), P.cmap.get(), keys.get(), vals.get());
        DRG_LAUNCH_CHECK();
        const bool all = (int64_t)tc == (int64_t)N0;
        radix_sort_pairs(keys.get(), vals.get(), N0, all ? key_bits_for(tl) : 32, st);
        hipLaunchKernelGGL(k_store_perm, dim3(ceil_div(tc, 256)), dim3(256), 0, st, (int32_t)tc,
                           vals.get(), gid, dbase0.get(), P.perm.get());
        DRG_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_store_seg, dim3(ceil_div(tl, 256)), dim3(256), 0, st, tl,
                           (int32_t)tc, dkg.get(), dkbk.get(), (int32_t)K.size(), keys.get(),
                           dco.get(), dso.get(), dn0.get(), P.seg.get());
        DRG_LAUNCH_CHECK();
        DRG_HIP(hipStreamSynchronize(st));
        for (int32_t c : K) out.n[c].push_back(u.cn[c]);
        out.lv.push_back(std::move(P));
        // the kept coarse graphs become the next union
        own_rp = std::move(nxt.rp);
        own_col = std::move(nxt.col);
        own_gid = std::move(u.cgid);
        crp = own_rp.get();
        ccol = own_col.get();
        cgid = own_gid.get();
        cn = nxt.n;
        cnnz = nxt.nnz;
        for (int32_t c = 0; c < count; ++c) {
            member[c] = 0;
        }
        for (int32_t c : E) {
            member[c] = 1;
            vb[c] = u.cbase[c];
            vn[c] = u.cn[c];
            ve[c] = cerow[c];
            vm[c] = cedge[c] - cerow[c];
            na[c] = nna[c];
        }
        if (K.size() != E.size()) compact(keep);
    }
}

}  // namespace drg
