// batch.hip -- many independent graphs laid out together, every graph on
// its own multilevel schedule (Sec. 3.2.3), synchronous iteration (Sec. 3.2.2).
//
// The graphs are joined into one union graph: graph c owns the node ids
// base[c] .. base[c+1]-1.  The sparse similarity of the union is built in one
// pass (a source's search stays inside its own graph, so its row is the row of
// the single-graph build shifted by base[c]); the negatives of a node are drawn
// from its own graph's sampling table.  Each graph keeps its own hierarchy,
// iteration count, learning-rate schedule and parameters.
//
// Iteration t is three launches that each cover every graph, whatever level
// the graph is at: stage (records of every finest node from its graph's
// current level), sweep (waves own row ranges of one graph; a graph keeps the
// lanes per row its single-graph sweep uses) and apply (one thread per node of
// each graph's current level).  Prolongations run between iterations where a
// graph moves to a finer level.  The whole run -- initial layout, T
// iterations, prolongations -- is recorded once into a hipGraph and replayed
// by every run.  Every node goes through the same per-node arithmetic as in
// the single-graph path, so graph c of a batch reproduces its single-graph
// layout bit for bit.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <map>
#include <memory>
#include <string>
#include <type_traits>

#include "drg_blocked.hpp"
#include "drg_forces.hpp"
#include "drg_internal.hpp"

namespace drg {

struct BGraph {              // constants of graph c
    int32_t base, n;         // finest nodes are union ids base .. base+n-1
    int32_t G, b, M, L;      // lanes per row, exponent, negatives (0 if S = 0), levels
    int32_t gbits, guide_off, lv_off, blk;  // blk: swept on its column-blocked copy
    uint64_t S, Cbase;       // sampling total and C[base]
    uint64_t seed;
    float clip;
    int32_t noclip;          // the attraction clip cannot bind (attract_clip_free)
};

struct BLevel {              // graph c at level l
    int32_t n;               // nodes of the level
    int32_t pbase;           // union id of the graph's finest node 0
    int64_t yoff;            // first coordinate of the level in the batch buffer
    const int32_t* cmap;     // [n0] finest node -> level node (level >= 1)
    const int32_t* seg;      // [n+1] member offsets into perm (level >= 1)
    const int32_t* perm;     // [n0] finest members, ascending inside a node
    const int32_t* map;      // [n_{l-1}] finer node -> node of this level (level >= 1)
};

struct SweepForm {           // rpl = 0: row form; else windowed with rpl rows per group
    int rpl = 0, ch = 0;
};

struct BSched {              // graph c at iteration t
    int32_t level;           // -1: the graph has finished
    float eta, gamma;
    int32_t pad;
};

// largest c in [0, count) with off[c] <= x (off ascending, off[0] = 0)
__device__ __forceinline__ int32_t find_owner(const int32_t* __restrict__ off, int32_t count,
                                              int64_t x) {
    int32_t lo = 0, hi = count - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if ((int64_t)off[mid] <= x)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// ------------------------------------------------------------------ union graph
struct UGraph {
    const int32_t* rp;
    const int32_t* col;
    int32_t base, n;
    int32_t ebase, nnz;
};

__global__ void k_union_nodes(int32_t N, int32_t count, const int32_t* __restrict__ nbase,
                              const UGraph* __restrict__ ug, int32_t* __restrict__ urp,
                              int32_t* __restrict__ node_base, int32_t* __restrict__ gid) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    const int32_t c = find_owner(nbase, count, j);
    const UGraph u = ug[c];
    const int32_t v = (int32_t)j - u.base;
    urp[j] = u.ebase + u.rp[v];
    node_base[j] = u.base;
    gid[j] = c;
    if (v == u.n - 1 && c == count - 1) urp[N] = u.ebase + u.rp[u.n];
}

__global__ void k_union_edges(int32_t E, int32_t count, const int32_t* __restrict__ ebase,
                              const UGraph* __restrict__ ug, int32_t* __restrict__ ucol) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= E) return;
    const int32_t c = find_owner(ebase, count, x);
    const UGraph u = ug[c];
    ucol[x] = u.col[x - u.ebase] + u.base;
}

// Row offsets of every graph lie inside its own edge range, ascending, and
// start and end where its nnz says.
__global__ void k_check_union_rows(int32_t N, const int32_t* __restrict__ gid,
                                   const UGraph* __restrict__ ug, const int32_t* __restrict__ urp,
                                   int* __restrict__ bad) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    const UGraph u = ug[gid[j]];
    const int32_t a = urp[j], e = urp[j + 1];
    bool ok = a >= u.ebase && e <= u.ebase + u.nnz && e >= a;
    if (j == u.base) ok = ok && a == u.ebase;
    if (j == (int64_t)u.base + u.n - 1) ok = ok && e == u.ebase + u.nnz;
    if (!ok) atomicOr(bad, 1);
}

__global__ void k_check_union_cols(int32_t N, const int32_t* __restrict__ gid,
                                   const UGraph* __restrict__ ug, const int32_t* __restrict__ urp,
                                   const int32_t* __restrict__ ucol, int* __restrict__ bad) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    const UGraph u = ug[gid[j]];
    for (int32_t x = urp[j]; x < urp[j + 1]; ++x) {
        const int32_t v = ucol[x];
        if (v < u.base || v >= u.base + u.n) {
            atomicOr(bad, 2);
            return;
        }
    }
}

// ------------------------------------------------------------------ sampling guides
// Per graph: guide[b] = draw result of the smallest word of bucket b, and
// guide[2^gbits] that of the largest word (as the single-graph table).
__global__ void k_b_guide(int32_t total, int32_t count, const int32_t* __restrict__ goff,
                          const BGraph* __restrict__ gt, const uint64_t* __restrict__ C,
                          int32_t* __restrict__ guide) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= total) return;
    const int32_t c = find_owner(goff, count, x);
    const BGraph g = gt[c];
    const int64_t b = x - goff[c];
    const int64_t nb = (int64_t)1 << g.gbits;
    if (g.S == 0) {
        guide[x] = 0;
        return;
    }
    const uint64_t r = b < nb ? __umul64hi((uint64_t)b << (64 - g.gbits), g.S) : g.S - 1;
    const uint64_t* Cg = C + g.base;
    int32_t lo = 0, hi = g.n - 1;
    while (lo < hi) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        if (Cg[mid + 1] - g.Cbase > r)
            hi = mid;
        else
            lo = mid + 1;
    }
    guide[x] = lo;
}

// Negative draw inside graph g: the local v with C_g[v+1] > floor(w S_g / 2^64).
__device__ __forceinline__ int32_t draw_in_graph(uint64_t w, const uint64_t* __restrict__ C,
                                                 const int32_t* __restrict__ guide,
                                                 const BGraph& g) {
    const uint64_t r = __umul64hi(w, g.S);
    const uint32_t bkt = (uint32_t)(w >> (64 - g.gbits));
    const int32_t* gd = guide + g.guide_off;
    const uint64_t* Cg = C + g.base;
    int32_t lo = gd[bkt], hi = gd[bkt + 1];
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (Cg[mid + 1] - g.Cbase > r)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

// ------------------------------------------------------------------ iteration kernels
__global__ void k_b_init(int32_t total, int32_t count, const int32_t* __restrict__ off,
                         const BGraph* __restrict__ gt, const BLevel* __restrict__ lt,
                         float2* __restrict__ y) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= total) return;
    const int32_t c = find_owner(off, count, x);
    const BGraph g = gt[c];
    const int32_t v = (int32_t)(x - off[c]);
    y[lt[g.lv_off + g.L - 1].yoff + v] = init_point<float>(v, g.L - 1, g.seed);
}

__global__ void k_b_stage(int32_t N, int32_t count, int32_t t, const int32_t* __restrict__ gid,
                          const BGraph* __restrict__ gt, const BLevel* __restrict__ lt,
                          const BSched* __restrict__ sched, const float* __restrict__ invZ,
                          const float* __restrict__ invZlo, const float2* __restrict__ y,
                          float4* __restrict__ rec) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    const int32_t c = gid[j];
    const int32_t l = sched[(int64_t)t * count + c].level;
    if (l < 0) return;
    const BGraph g = gt[c];
    const BLevel d = lt[g.lv_off + l];
    const int32_t v = (int32_t)j - g.base;
    const float2 p = y[d.yoff + (l == 0 ? v : d.cmap[v])];
    rec[j] = mk4<float>(p.x, p.y, invZ[j], invZlo[j]);
}

struct BSweepArgs {
    int32_t count, t;
    const int32_t* woff;      // [count+1] waves of each graph
    const BGraph* gt;
    const BSched* sched;
    const int64_t* prp;
    const uint32_t* colhop;
    const float4* rec;
    const float* qt;
    const uint64_t* C;
    const int32_t* guide;
    float2* g;
    HalfE<double> eh;
};

template <int B, bool CLIP>
__device__ __forceinline__ float2 b_row(const BSweepArgs& a, const BGraph& g, int64_t i,
                                        int32_t v, int lane, float gamma) {
    return sweep_row<float, B, CLIP>(a.rec[i], a.prp[i], a.prp[i + 1], lane, g.G, a.colhop,
                               a.rec, a.eh,
                               g.clip, false, g.M, g.seed, (uint64_t)a.t, v,
                               [&](uint64_t w) {
                                   return g.base + draw_in_graph(w, a.C, a.guide, g);
                               },
                               (double)gamma * (double)a.qt[i]);
}

// Graph c owns waves woff[c] .. woff[c+1]-1; each handles 64/G consecutive
// rows.  A block runs 4 consecutive waves; the blocks of one XCD take a
// contiguous range of waves, so each XCD works through few graphs at a time.
__global__ __launch_bounds__(256) void k_b_sweep(BSweepArgs a) {
    const int32_t total = a.woff[a.count];
    const int32_t gw = __builtin_amdgcn_readfirstlane(
        xcd_block((int32_t)blockIdx.x, (int32_t)gridDim.x) * 4 + (int32_t)(threadIdx.x / WAVE));
    if (gw >= total) return;
    const int32_t c = find_owner(a.woff, a.count, gw);
    const BSched sc = a.sched[(int64_t)a.t * a.count + c];
    if (sc.level < 0) return;
    const BGraph g = a.gt[c];
    const int lane = __lane_id() % g.G;
    const int32_t v = (gw - a.woff[c]) * (WAVE / g.G) + (int32_t)(__lane_id() / g.G);
    if (v >= g.n) return;
    const int64_t i = (int64_t)g.base + v;
    float2 gi = make_float2(0.0f, 0.0f);
    if (a.prp[i] < a.prp[i + 1]) {
        if (g.noclip) {
            if (g.b == 1)
                gi = b_row<1, false>(a, g, i, v, lane, sc.gamma);
            else if (g.b == 2)
                gi = b_row<2, false>(a, g, i, v, lane, sc.gamma);
            else
                gi = b_row<3, false>(a, g, i, v, lane, sc.gamma);
        } else {
            if (g.b == 1)
                gi = b_row<1, true>(a, g, i, v, lane, sc.gamma);
            else if (g.b == 2)
                gi = b_row<2, true>(a, g, i, v, lane, sc.gamma);
            else
                gi = b_row<3, true>(a, g, i, v, lane, sc.gamma);
        }
    }
    if (lane == 0) a.g[i] = gi;
}

// Windowed form (bit-identical to k_b_sweep): one workgroup per item.
struct BWinArgs {
    int32_t count, t, CH;
    const WinItem* items;
    const BGraph* gt;
    const BSched* sched;
    const int64_t* prp;
    const uint32_t* colhop;
    const float4* rec;
    const float* qt;
    const uint64_t* C;
    const int32_t* guide;
    float2* g;
    HalfE<double> eh;
};

template <int RPL>
__global__ __launch_bounds__(WIN_BLOCK) void k_b_sweep_win(BWinArgs a) {
    extern __shared__ float4 s_rec[];
    const WinItem it = a.items[xcd_block((int32_t)blockIdx.x, (int32_t)gridDim.x)];
    const BSched sc = a.sched[(int64_t)a.t * a.count + it.graph];
    if (sc.level < 0) return;  // the whole workgroup leaves
    const BGraph g = a.gt[it.graph];
    if (g.blk) return;  // swept by k_b_sweep_blocked
    auto draw = [&](uint64_t w) { return g.base + draw_in_graph(w, a.C, a.guide, g); };
    auto key = [&](int64_t i) { return (int32_t)(i - g.base); };
    auto item = [&](auto b_c, auto clip_c) {
        window_item<decltype(b_c)::value, decltype(clip_c)::value, RPL, WIN_BLOCK>(
            it, g.G, s_rec, a.CH, a.prp, a.colhop, a.rec, a.qt, a.eh, g.clip, false, g.M, g.seed,
            (uint64_t)a.t, sc.gamma, draw, key, a.g);
    };
    using yes = std::true_type;
    using no = std::false_type;
    if (g.noclip) {
        if (g.b == 1)
            item(std::integral_constant<int, 1>{}, no{});
        else if (g.b == 2)
            item(std::integral_constant<int, 2>{}, no{});
        else
            item(std::integral_constant<int, 3>{}, no{});
    } else {
        if (g.b == 1)
            item(std::integral_constant<int, 1>{}, yes{});
        else if (g.b == 2)
            item(std::integral_constant<int, 2>{}, yes{});
        else
            item(std::integral_constant<int, 3>{}, yes{});
    }
}

// Graphs whose single-graph sweep runs on the column-blocked copy (large
// patterns) keep that copy here, built by the same rule, so each of them is
// swept with the same work items and arithmetic as alone.
struct BBlkView {
    const uint16_t* ent;
    const int64_t* base;
    const int32_t* off;
    float2* partial;
    int32_t nb, bits;
    float eh0, eh1, eh2, eh3;  // -b e_d per hop
    float clip;                // clip / (2b)
    int32_t noclip;            // the clip cannot bind (attract_clip_free)
};

struct BBlkArgs {
    int32_t count, t, flat, lanes;
    const int4* items;   // (block, first row, end row, graph)
    const int4* groups;  // (first item, items, graph, -): consecutive items of one block
    const BBlkView* views;
    const BGraph* gt;
    const BSched* sched;
    const float4* rec;
};

// One launch per exponent b (the groups of the graphs with that b), so
// each kernel holds the code of one b, as the single-graph kernel does.
template <int NH, int F, int B>
__global__ __launch_bounds__(STREAM_BLOCK) void k_b_sweep_blocked(BBlkArgs a) {
    extern __shared__ float4 s_dyn[];
    const int4 gr = a.groups[xcd_block((int32_t)blockIdx.x, (int32_t)gridDim.x)];
    const int32_t c = gr.z;
    if (a.sched[(int64_t)a.t * a.count + c].level < 0) return;  // the whole workgroup leaves
    const int4* its = a.items + gr.x;
    const int32_t blk = its[0].x;
    const BGraph g = a.gt[c];
    const BBlkView v = a.views[c];
    BlockedArgs la{};
    la.n0 = g.n;
    la.bits = v.bits;
    la.ent = v.ent;
    la.base = v.base;
    la.off = v.off;
    la.rec = a.rec + g.base;
    la.partial = v.partial;
    la.eh0 = v.eh0;
    la.eh1 = v.eh1;
    la.eh2 = v.eh2;
    la.eh3 = v.eh3;
    la.clip = v.clip;
    la.noclip = v.noclip;
    la.lanes = a.lanes;
    la.flat = a.flat;
    blk_layout_items<B, NH, F>(la, s_dyn, blk, its, gr.y);
}

template <int NH, int B>
static auto b_blk_kernel_nhb(int form) {
    return form == 4   ? k_b_sweep_blocked<NH, 4, B>
           : form == 2 ? k_b_sweep_blocked<NH, 2, B>
                       : k_b_sweep_blocked<NH, 0, B>;
}

template <int NH>
static auto b_blk_kernel_nh(int form, int b) {
    return b == 1 ? b_blk_kernel_nhb<NH, 1>(form)
                  : (b == 2 ? b_blk_kernel_nhb<NH, 2>(form) : b_blk_kernel_nhb<NH, 3>(form));
}

// the batch's blocked-sweep kernel for NH hop weights, sweep form F and exponent b
static auto b_blk_kernel(int NH, int form, int b) {
    return NH == 1 ? b_blk_kernel_nh<1>(form, b)
                   : (NH == 2 ? b_blk_kernel_nh<2>(form, b) : b_blk_kernel_nh<4>(form, b));
}

struct BFinArgs {
    int32_t nblk, count, t;
    const int32_t* boff;    // [nblk+1] node prefix over the blocked graphs
    const int32_t* bgraph;  // [nblk] their graph ids
    const BBlkView* views;
    const BGraph* gt;
    const BSched* sched;
    const int64_t* prp;
    const float4* rec;
    const float* qt;
    const uint64_t* C;
    const int32_t* guide;
    float2* g;
};

// One thread per node of a blocked graph: its partials and own negatives.
__global__ void k_b_finish(BFinArgs a) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= a.boff[a.nblk]) return;
    const int32_t k = find_owner(a.boff, a.nblk, x);
    const int32_t c = a.bgraph[k];
    const BSched sc = a.sched[(int64_t)a.t * a.count + c];
    if (sc.level < 0) return;
    const BGraph g = a.gt[c];
    const BBlkView v = a.views[c];
    const int32_t u = (int32_t)(x - a.boff[k]);
    const int64_t i = (int64_t)g.base + u;
    float2 gi = make_float2(0.0f, 0.0f);
    if (a.prp[i + 1] > a.prp[i]) {
        const float4* R = a.rec + g.base;
        auto draw = [&](uint64_t w) { return draw_in_graph(w, a.C, a.guide, g); };
        const float gq = sc.gamma * a.qt[i];
        if (g.b == 1)
            gi = blk_finish_row<1>(v.partial, v.nb, g.n, u, R, R[u], g.M, g.seed, (uint64_t)a.t,
                                   u, draw, gq, g.clip);
        else if (g.b == 2)
            gi = blk_finish_row<2>(v.partial, v.nb, g.n, u, R, R[u], g.M, g.seed, (uint64_t)a.t,
                                   u, draw, gq, g.clip);
        else
            gi = blk_finish_row<3>(v.partial, v.nb, g.n, u, R, R[u], g.M, g.seed, (uint64_t)a.t,
                                   u, draw, gq, g.clip);
    }
    a.g[i] = gi;
}

// One lane per node of each graph's current level (off: this phase's
// prefix); coarse-level nodes with many members are summed by the whole wave,
// as in the single-graph kernel.
__global__ void k_b_apply(int32_t total, int32_t count, int32_t t, const int32_t* __restrict__ off,
                          const BGraph* __restrict__ gt, const BLevel* __restrict__ lt,
                          const BSched* __restrict__ sched, const float2* __restrict__ g,
                          const float* __restrict__ qt, float2* __restrict__ y) {
    const int64_t x0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (__ballot(x0 < total) == 0) return;  // the whole wave leaves
    const bool in = x0 < total;
    const int64_t x = in ? x0 : total - 1;
    const int32_t c = find_owner(off, count, x);
    const BSched sc = sched[(int64_t)t * count + c];
    const BGraph gg = gt[c];
    const BLevel d = lt[gg.lv_off + sc.level];
    const int32_t v = (int32_t)(x - off[c]);
    if (sc.level == 0 && in) {
        const int64_t i = (int64_t)gg.base + v;
        apply_node<float>(g[i], qt[i], y + d.yoff + v, sc.eta);
    }
    const bool coarse = in && sc.level > 0;
    apply_level_wave<float>(coarse, coarse ? d.seg[v] : 0, coarse ? d.seg[v + 1] : 0, d.perm,
                            d.pbase, g, qt, y + d.yoff + v, sc.eta);
}

// y_{l-1}[u] = y_l[map_l[u]] for the graphs of one prolongation round.
__global__ void k_b_prolong(int32_t total, int32_t m, const int32_t* __restrict__ off,
                            const int2* __restrict__ ops, const BGraph* __restrict__ gt,
                            const BLevel* __restrict__ lt, float2* __restrict__ y) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= total) return;
    const int32_t k = find_owner(off, m, x);
    const int2 op = ops[k];  // (graph, level left)
    const BGraph g = gt[op.x];
    const BLevel d = lt[g.lv_off + op.y];
    const BLevel f = lt[g.lv_off + op.y - 1];
    const int32_t u = (int32_t)(x - off[k]);
    y[f.yoff + u] = y[d.yoff + d.map[u]];
}

}  // namespace drg

// ------------------------------------------------------------------ the batch
struct drg_batch {
    int device = 0;
    int32_t count = 0, T = 0;
    int64_t n_total = 0, nnz_total = 0, y_total = 0;
    std::vector<int32_t> base, levels;
    std::unique_ptr<drg_sim, void (*)(drg_sim*)> sim{nullptr, drg_sim_destroy};
    drg::UnionHier hier;
    drg::DevBuf<drg::BGraph> gt;
    drg::DevBuf<drg::BLevel> lt;
    drg::DevBuf<drg::BSched> sched;
    drg::DevBuf<int32_t> gid, guide, woff, init_off, phase_off, pro_off;
    drg::DevBuf<drg::WinItem> win_items;        // items of the chosen windowed form
    std::vector<std::unique_ptr<drg::BlkLayout>> blk;  // column-blocked copies (large graphs)
    drg::DevBuf<int4> blk_items;
    drg::DevBuf<int4> blk_groups;
    drg::DevBuf<drg::BBlkView> blk_views;
    drg::DevBuf<int32_t> blk_off, blk_graph;
    int32_t blk_ngroups = 0, blk_count = 0, blk_nodes = 0;
    int32_t blk_b_first[3] = {0, 0, 0}, blk_b_count[3] = {0, 0, 0};  // groups per exponent
    drg::SweepForm form;                        // chosen sweep form
    std::vector<std::pair<drg::SweepForm, float>> tune;  // candidates and their times
    drg::DevBuf<int2> pro_ops;
    drg::DevBuf<float2> y;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~drg_batch() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

namespace drg {

void check_layout_params(const drg_layout_params* p) {
    if (!p) throw Error(DRG_E_INVALID, "params is NULL");
    if (p->T < 0) throw Error(DRG_E_INVALID, "T must be >= 0");
    if (p->M < 0 || p->b < 1 || p->b > 3) throw Error(DRG_E_INVALID, "M >= 0, b in 1..3");
    if (!(p->clip > 0.0f)) throw Error(DRG_E_INVALID, "clip must be > 0");
    if (p->mode != DRG_MODE_SYNC && p->mode != DRG_MODE_ASYNC)
        throw Error(DRG_E_INVALID, "unknown mode");
    if (p->dim != 0 && p->dim != 2 && p->dim != 3)
        throw Error(DRG_E_INVALID, "dim must be 2 (or 0) or 3");
    check_shape(p->b, p->b_half);
    if (p->perplexity != 0.0 && !(p->perplexity >= 1.0 && p->perplexity < 1e300))
        throw Error(DRG_E_INVALID, "perplexity must be 0 (global sigma) or >= 1 and finite");
}

template <typename T>
static void upload(DevBuf<T>& d, const std::vector<T>& h, hipStream_t st) {
    d.alloc((int64_t)h.size());
    if (!h.empty())
        DRG_HIP(hipMemcpyAsync(d.get(), h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice, st));
}

static int read_flag(DevBuf<int>& f, hipStream_t s) {
    int h = 0;
    DRG_HIP(hipMemcpyAsync(&h, f.get(), sizeof(int), hipMemcpyDeviceToHost, s));
    DRG_HIP(hipStreamSynchronize(s));
    return h;
}

drg_batch* batch_create(drg_ctx* ctx, const drg_csr* graphs, int32_t count,
                        const drg_layout_params* params) {
    if (!graphs || !params) throw Error(DRG_E_INVALID, "graphs or params is NULL");
    if (count < 1) throw Error(DRG_E_INVALID, "count must be >= 1");
    for (int32_t c = 0; c < count; ++c) {
        const drg_layout_params& p = params[c];
        check_layout_params(&p);
        if (p.mode != DRG_MODE_SYNC)
            throw Error(DRG_E_UNSUPPORTED, "batched layout: synchronous mode only");
        if (p.dim == 3)
            throw Error(DRG_E_UNSUPPORTED, "batched layout: 2-D layouts only");
        if (p.b_half)
            throw Error(DRG_E_UNSUPPORTED, "batched layout: whole b only");
        if (p.perplexity != 0.0)
            throw Error(DRG_E_UNSUPPORTED, "batched layout: one global sigma only");
        if (p.k != params[0].k || p.sigma != params[0].sigma)
            throw Error(DRG_E_INVALID, "batched layout: k and sigma must agree over the batch");
        if (!(p.rho > 0.0 && p.rho <= 1.0) || p.max_levels < 1 || p.min_nodes < 0)
            throw Error(DRG_E_INVALID, "batched layout: bad coarsening parameters");
        const drg_csr& g = graphs[c];
        if (g.n <= 0 || g.nnz < 0 || !g.row_ptr || (g.nnz > 0 && !g.col))
            throw Error(DRG_E_INVALID, "batched layout: bad CSR of graph " + std::to_string(c));
    }
    hipStream_t st = ctx->stream;
    auto b = std::make_unique<drg_batch>();
    b->device = ctx->device;
    b->count = count;
    // ---- union graph
    std::vector<int32_t> nbase(count + 1, 0), ebase(count + 1, 0);
    std::vector<UGraph> ug(count);
    int32_t max_comp = 0;
    for (int32_t c = 0; c < count; ++c) {
        const int64_t nb = (int64_t)nbase[c] + graphs[c].n;
        const int64_t eb = (int64_t)ebase[c] + graphs[c].nnz;
        if (nb >= ((int64_t)1 << 30) || eb >= ((int64_t)1 << 31))
            throw Error(DRG_E_INVALID, "batched layout: union exceeds 2^30 nodes or 2^31 edges");
        nbase[c + 1] = (int32_t)nb;
        ebase[c + 1] = (int32_t)eb;
        ug[c] = UGraph{graphs[c].row_ptr, graphs[c].col, nbase[c], graphs[c].n, ebase[c],
                       (int32_t)graphs[c].nnz};
        max_comp = std::max(max_comp, graphs[c].n);
    }
    const int32_t N = nbase[count], E = ebase[count];
    b->n_total = N;
    b->base = nbase;
    DevBuf<UGraph> dug;
    DevBuf<int32_t> dnb, deb, urp((int64_t)N + 1), ucol(E), node_base(N);
    upload(dug, ug, st);
    upload(dnb, nbase, st);
    upload(deb, ebase, st);
    b->gid.alloc(N);
    hipLaunchKernelGGL(k_union_nodes, dim3(ceil_div(N, 256)), dim3(256), 0, st, N, count,
                       dnb.get(), dug.get(), urp.get(), node_base.get(), b->gid.get());
    DRG_LAUNCH_CHECK();
    if (E > 0) {
        hipLaunchKernelGGL(k_union_edges, dim3(ceil_div(E, 256)), dim3(256), 0, st, E, count,
                           deb.get(), dug.get(), ucol.get());
        DRG_LAUNCH_CHECK();
    }
    {
        DevBuf<int> bad(1);
        DRG_HIP(hipMemsetAsync(bad.get(), 0, sizeof(int), st));
        hipLaunchKernelGGL(k_check_union_rows, dim3(ceil_div(N, 256)), dim3(256), 0, st, N,
                           b->gid.get(), dug.get(), urp.get(), bad.get());
        DRG_LAUNCH_CHECK();
        if (read_flag(bad, st)) throw Error(DRG_E_GRAPH, "row_ptr is not a valid offset array");
        hipLaunchKernelGGL(k_check_union_cols, dim3(ceil_div(N, 256)), dim3(256), 0, st, N,
                           b->gid.get(), dug.get(), urp.get(), ucol.get(), bad.get());
        DRG_LAUNCH_CHECK();
        if (read_flag(bad, st)) throw Error(DRG_E_GRAPH, "column index out of range");
    }
    // ---- similarity of the union
    drg_csr uc{N, E, urp.get(), ucol.get()};
    UnionInfo ui;
    ui.count = count;
    ui.base = nbase;
    ui.node_base = node_base.get();
    ui.max_comp = max_comp;
    b->sim.reset(build_similarity(ctx, &uc, params[0].k, params[0].sigma, 0, &ui));
    drg_sim* s = b->sim.get();
    b->nnz_total = s->nnz;
    // per-graph active rows, row-length statistics and sampling totals
    std::vector<int32_t> nact(count, 0);
    std::vector<uint64_t> Cb(count + 1, 0);
    std::vector<unsigned long long> len2(count, 0);  // sum of squared row lengths
    {
        DevBuf<int32_t> cnt(count);
        DevBuf<unsigned long long> l2(count);
        count_nonempty_by_group<int64_t>(s->row_ptr.get(), b->gid.get(), N, cnt.get(), count, st);
        sum_len2_by_group(s->row_ptr.get(), b->gid.get(), N, l2.get(), count, st);
        DRG_HIP(hipMemcpyAsync(nact.data(), cnt.get(), sizeof(int32_t) * count,
                               hipMemcpyDeviceToHost, st));
        DRG_HIP(hipMemcpyAsync(len2.data(), l2.get(), sizeof(unsigned long long) * count,
                               hipMemcpyDeviceToHost, st));
        for (int32_t c = 0; c <= count; ++c)
            DRG_HIP(hipMemcpyAsync(&Cb[c], s->C.get() + nbase[c], sizeof(uint64_t),
                                   hipMemcpyDeviceToHost, st));
        DRG_HIP(hipStreamSynchronize(st));
    }
    // ---- hierarchies of all graphs, level by level over the union
    build_hierarchy_union(ctx, &uc, b->gid.get(), nbase, params, b->hier);
    // ---- per-graph tables
    std::vector<BGraph> gt(count);
    std::vector<BLevel> lt;
    std::vector<int32_t> goff(count + 1, 0), woff(count + 1, 0);
    b->levels.resize(count);
    int64_t yoff = N;  // finest coordinates first, in union order
    for (int32_t c = 0; c < count; ++c) {
        const drg_layout_params& p = params[c];
        const int32_t L = (int32_t)b->hier.n[c].size();
        const int32_t n = graphs[c].n;
        BGraph& g = gt[c];
        g.base = nbase[c];
        g.n = n;
        // the lanes per row of the graph's own single-graph sweep
        g.G = sweep_group(ui.nnz[c] > 0 ? (double)len2[c] / (double)ui.nnz[c] : 0.0, nact[c]);
        g.blk = blocked_wanted_for(ctx, n, ui.nnz[c]) ? 1 : 0;
        g.b = p.b;
        g.S = Cb[c + 1] - Cb[c];
        g.Cbase = Cb[c];
        g.M = g.S > 0 ? p.M : 0;
        g.L = L;
        int gbits = 1;
        while (gbits < 30 && ((int64_t)1 << gbits) < n) ++gbits;
        g.gbits = gbits;
        g.guide_off = goff[c];
        goff[c + 1] = goff[c] + (1 << gbits) + 1;
        g.lv_off = (int32_t)lt.size();
        g.seed = p.seed;
        g.clip = p.clip;
        g.noclip = attract_clip_free(p.b, p.clip) ? 1 : 0;
        const int64_t w = g.blk ? 0 : ((int64_t)n + WAVE / g.G - 1) / (WAVE / g.G);
        if ((int64_t)woff[c] + w >= ((int64_t)1 << 31))
            throw Error(DRG_E_INVALID, "batched layout: too many rows");
        woff[c + 1] = woff[c] + (int32_t)w;
        b->levels[c] = L;
        for (int32_t l = 0; l < L; ++l) {
            BLevel d{};
            d.n = b->hier.n[c][l];
            d.pbase = nbase[c];
            if (l == 0) {
                d.yoff = nbase[c];
            } else {
                const UnionHier::Pool& P = b->hier.lv[l];
                d.yoff = yoff;
                yoff += d.n;
                d.cmap = P.cmap.get() + P.co[c];
                d.seg = P.seg.get() + P.so[c];
                d.perm = P.perm.get() + P.co[c];
                d.map = P.map.get() + P.mo[c];
            }
            lt.push_back(d);
        }
    }
    b->y_total = yoff;
    upload(b->gt, gt, st);
    upload(b->lt, lt, st);
    upload(b->woff, woff, st);
    {
        DevBuf<int32_t> dgoff;
        upload(dgoff, goff, st);
        b->guide.alloc(goff[count]);
        hipLaunchKernelGGL(k_b_guide, dim3(ceil_div(goff[count], 256)), dim3(256), 0, st,
                           goff[count], count, dgoff.get(), b->gt.get(), s->C.get(),
                           b->guide.get());
        DRG_LAUNCH_CHECK();
        DRG_HIP(hipStreamSynchronize(st));
    }
    // ---- schedules: graph c spends T_c / L_c iterations per level, coarsest
    // first, the remainder at the finest; prolongation after each coarse level
    int32_t T = 0;
    for (int32_t c = 0; c < count; ++c) T = std::max(T, params[c].T);
    b->T = T;
    std::vector<BSched> sch((size_t)T * count);
    // prolongation rounds before iteration t (t = 0..T): (t, round) -> ops
    std::map<std::pair<int32_t, int32_t>, std::vector<int2>> pro;
    for (int32_t c = 0; c < count; ++c) {
        const drg_layout_params& p = params[c];
        const int32_t L = gt[c].L;
        const int32_t per = p.T / L;
        int32_t t = 0;
        for (int32_t l = L - 1; l >= 0; --l) {
            const int32_t Tl = per + (l == 0 ? p.T - per * L : 0);
            const float gam = (l == L - 1 && L > 1) ? p.gamma_coarsest : p.gamma;
            for (int32_t s2 = 0; s2 < Tl; ++s2, ++t) {
                BSched& e = sch[(size_t)t * count + c];
                e.level = l;
                e.eta = (float)((double)p.eta0 * (1.0 - (double)s2 / (double)Tl));
                e.gamma = gam;
            }
            if (l > 0) {
                int32_t round = 0;
                while (pro.count({t, round}) && !pro[{t, round}].empty() &&
                       pro[{t, round}].back().x == c)
                    ++round;
                pro[{t, round}].push_back(make_int2(c, l));
            }
        }
        for (; t < T; ++t) sch[(size_t)t * count + c].level = -1;
    }
    upload(b->sched, sch, st);
    // apply phases: runs of iterations with the same level in every graph
    std::vector<int32_t> phase_of(T, 0), ph;
    std::vector<int32_t> phase_total;
    for (int32_t t = 0; t < T; ++t) {
        bool same = t > 0;
        for (int32_t c = 0; same && c < count; ++c)
            same = sch[(size_t)t * count + c].level == sch[(size_t)(t - 1) * count + c].level;
        if (!same) {
            const size_t o = ph.size();
            ph.resize(o + count + 1);
            ph[o] = 0;
            for (int32_t c = 0; c < count; ++c) {
                const int32_t l = sch[(size_t)t * count + c].level;
                ph[o + c + 1] = ph[o + c] + (l < 0 ? 0 : lt[gt[c].lv_off + l].n);
            }
            phase_total.push_back(ph[o + count]);
        }
        phase_of[t] = (int32_t)phase_total.size() - 1;
    }
    upload(b->phase_off, ph, st);
    // prolongation rounds: ops and per-op node prefix, concatenated
    struct Round {
        int32_t t, ofirst, pfirst, m, total;
    };
    std::vector<Round> rounds;
    std::vector<int2> ops;
    std::vector<int32_t> poff;
    for (auto& kv : pro) {  // ascending (t, round)
        Round r{kv.first.first, (int32_t)ops.size(), (int32_t)poff.size(),
                (int32_t)kv.second.size(), 0};
        poff.push_back(0);
        for (const int2& op : kv.second) {
            ops.push_back(op);
            poff.push_back(poff.back() + lt[gt[op.x].lv_off + op.y - 1].n);
        }
        r.total = poff.back();
        rounds.push_back(r);
    }
    upload(b->pro_ops, ops, st);
    upload(b->pro_off, poff, st);
    std::vector<int32_t> ioff(count + 1, 0);
    for (int32_t c = 0; c < count; ++c)
        ioff[c + 1] = ioff[c] + lt[gt[c].lv_off + gt[c].L - 1].n;
    upload(b->init_off, ioff, st);
    b->y.alloc(b->y_total);
    DRG_HIP(hipStreamSynchronize(st));
    // ---- graphs swept on their column-blocked copy, as they would be alone
    const int NH = s->k == 1 ? 1 : (s->k == 2 ? 2 : 4);
    const int blk_cpl = blk_flat_cpl(), blk_ln = blk_lanes();
    size_t blk_lds = 0;
    {
        std::vector<BBlkView> views(count);
        std::vector<int4> bitems, bgroups;
        std::vector<int32_t> boff(1, 0), bgraph;
        int bits = 0;
        for (int32_t c = 0; c < count; ++c) {
            if (!gt[c].blk) continue;
            const drg_layout_params& p = params[c];
            auto L = std::make_unique<BlkLayout>();
            build_blocked_core(ctx, gt[c].n, ui.nnz[c], s->row_ptr.get() + nbase[c],
                               s->colhop.get(), nbase[c], *L);
            BBlkView& v = views[c];
            v.ent = L->ent.get();
            v.base = L->base.get();
            v.off = L->off.get();
            v.partial = L->partial.get();
            v.nb = L->nb;
            v.bits = L->bits;
            v.eh0 = (float)(-p.b * s->e[0]);
            v.eh1 = (float)(-p.b * s->e[1]);
            v.eh2 = (float)(-p.b * s->e[2]);
            v.eh3 = (float)(-p.b * s->e[3]);
            v.clip = p.clip / (float)(2 * p.b);
            v.noclip = attract_clip_free(p.b, p.clip) ? 1 : 0;
            bits = L->bits;
            std::vector<int4> h(L->nitems);
            DRG_HIP(hipMemcpy(h.data(), L->items.get(), sizeof(int4) * L->nitems,
                              hipMemcpyDeviceToHost));
            // a workgroup takes up to `per` consecutive items of one block
            // (about 2^18 entries), staging the block's records once
            const int32_t per = (int32_t)std::max<int64_t>(1, ((int64_t)1 << 18) / L->chunk);
            for (int4 it : h) {
                it.w = c;
                const int4 last = bgroups.empty() ? make_int4(0, 0, -1, 0) : bgroups.back();
                const bool extend = last.z == c && last.y < per && bitems[last.x].x == it.x;
                if (extend)
                    bgroups.back().y += 1;
                else
                    bgroups.push_back(make_int4((int32_t)bitems.size(), 1, c, 0));
                bitems.push_back(it);
            }
            bgraph.push_back(c);
            boff.push_back(boff.back() + gt[c].n);
            b->blk.push_back(std::move(L));
        }
        b->blk_count = (int32_t)bgraph.size();
        // groups ordered by exponent (stable), one launch per exponent
        std::vector<int4> sorted;
        for (int bb = 1; bb <= 3; ++bb) {
            b->blk_b_first[bb - 1] = (int32_t)sorted.size();
            for (const int4& gq : bgroups)
                if (gt[gq.z].b == bb) sorted.push_back(gq);
            b->blk_b_count[bb - 1] = (int32_t)sorted.size() - b->blk_b_first[bb - 1];
        }
        bgroups.swap(sorted);
        b->blk_ngroups = (int32_t)bgroups.size();
        b->blk_nodes = boff.back();
        if (b->blk_count > 0) {
            upload(b->blk_views, views, st);
            upload(b->blk_items, bitems, st);
            upload(b->blk_groups, bgroups, st);
            upload(b->blk_off, boff, st);
            upload(b->blk_graph, bgraph, st);
            blk_lds = blk_lds_bytes(bits);
            for (int bb = 1; bb <= 3; ++bb) {
                auto fn = b_blk_kernel(NH, blk_form(blk_cpl), bb);
                DRG_HIP(hipFuncSetAttribute((const void*)fn,
                                            hipFuncAttributeMaxDynamicSharedMemorySize,
                                            (int)blk_lds));
            }
            DRG_HIP(hipStreamSynchronize(st));
        }
    }
    auto launch_blocked = [&](int32_t t, hipStream_t stream) {
        if (b->blk_count == 0) return;
        BBlkArgs ba{};
        ba.count = count;
        ba.t = t;
        ba.flat = blk_cpl;
        ba.lanes = blk_ln;
        ba.items = b->blk_items.get();
        ba.groups = b->blk_groups.get();
        ba.views = b->blk_views.get();
        ba.gt = b->gt.get();
        ba.sched = b->sched.get();
        ba.rec = s->rec.get();
        for (int bb = 1; bb <= 3; ++bb) {
            if (b->blk_b_count[bb - 1] == 0) continue;
            BBlkArgs bx = ba;
            bx.groups = b->blk_groups.get() + b->blk_b_first[bb - 1];
            auto fn = b_blk_kernel(NH, blk_form(blk_cpl), bb);
            hipLaunchKernelGGL(fn, dim3(b->blk_b_count[bb - 1]), dim3(STREAM_BLOCK), blk_lds,
                               stream, bx);
            DRG_LAUNCH_CHECK();
        }
        BFinArgs fa{};
        fa.nblk = b->blk_count;
        fa.count = count;
        fa.t = t;
        fa.boff = b->blk_off.get();
        fa.bgraph = b->blk_graph.get();
        fa.views = b->blk_views.get();
        fa.gt = b->gt.get();
        fa.sched = b->sched.get();
        fa.prp = s->row_ptr.get();
        fa.rec = s->rec.get();
        fa.qt = s->qtf.get();
        fa.C = s->C.get();
        fa.guide = b->guide.get();
        fa.g = s->g.get();
        hipLaunchKernelGGL(k_b_finish, dim3(ceil_div(b->blk_nodes, 256)), dim3(256), 0, stream, fa);
        DRG_LAUNCH_CHECK();
    };
    // ---- the sweep: row form (k_b_sweep) or windowed form (k_b_sweep_win,
    // RPL rows per group, CH records per LDS chunk).  Both give the same bits;
    // the faster one on this batch is picked by timing each candidate once on
    // the first iteration's records (env DRG_BATCH_SWEEP=row|win forces one).
    BSweepArgs sa{};
    sa.count = count;
    sa.woff = b->woff.get();
    sa.gt = b->gt.get();
    sa.sched = b->sched.get();
    sa.prp = s->row_ptr.get();
    sa.colhop = s->colhop.get();
    sa.rec = s->rec.get();
    sa.qt = s->qtf.get();
    sa.C = s->C.get();
    sa.guide = b->guide.get();
    sa.g = s->g.get();
    sa.eh = HalfE<double>{0.5 * s->e[0], 0.5 * s->e[1], 0.5 * s->e[2], 0.5 * s->e[3]};
    const int64_t sweep_blocks = std::max<int64_t>(1, ((int64_t)woff[count] + 3) / 4);
    BWinArgs wa{};
    wa.count = count;
    wa.gt = sa.gt;
    wa.sched = sa.sched;
    wa.prp = sa.prp;
    wa.colhop = sa.colhop;
    wa.rec = sa.rec;
    wa.qt = sa.qt;
    wa.C = sa.C;
    wa.guide = sa.guide;
    wa.g = sa.g;
    wa.eh = sa.eh;
    std::map<int, std::pair<std::unique_ptr<DevBuf<WinItem>>, int32_t>> items;  // rpl -> items
    auto items_for = [&](int rpl) -> std::pair<const WinItem*, int32_t> {
        auto it = items.find(rpl);
        if (it == items.end()) {
            std::vector<int32_t> R(count);
            for (int32_t c = 0; c < count; ++c) R[c] = (WIN_BLOCK / gt[c].G) * rpl;
            auto buf = std::make_unique<DevBuf<WinItem>>();
            const int32_t ni = build_window_items(ctx, s, nbase, R, *buf);
            it = items.emplace(rpl, std::make_pair(std::move(buf), ni)).first;
        }
        return {it->second.first->get(), it->second.second};
    };
    auto win_kernel = [](int rpl) -> void (*)(BWinArgs) {
        return rpl == 1 ? k_b_sweep_win<1>
                        : (rpl == 2 ? k_b_sweep_win<2> : (rpl == 4 ? k_b_sweep_win<4> : k_b_sweep_win<8>));
    };
    const int max_ch = (ctx->max_lds - 1024) / (int)sizeof(float4);
    auto launch_form = [&](const SweepForm& f, int32_t t, hipStream_t stream) {
        if (f.rpl == 0) {
            sa.t = t;
            hipLaunchKernelGGL(k_b_sweep, dim3((unsigned)sweep_blocks), dim3(256), 0, stream, sa);
        } else {
            const auto its = items_for(f.rpl);
            if (its.second == 0) return;
            wa.t = t;
            wa.CH = f.ch;
            wa.items = its.first;
            auto fn = win_kernel(f.rpl);
            const size_t lds = (size_t)f.ch * sizeof(float4);
            DRG_HIP(hipFuncSetAttribute((const void*)fn,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            hipLaunchKernelGGL(fn, dim3(its.second), dim3(WIN_BLOCK), lds, stream, wa);
        }
        DRG_LAUNCH_CHECK();
    };
    std::vector<SweepForm> cands;
    const char* force = std::getenv("DRG_BATCH_SWEEP");
    if (force && std::string(force) == "row") {
        cands.push_back({0, 0});
    } else if (force && std::string(force) == "win") {
        cands.push_back({win_rpl(), win_chunk(ctx)});
    } else {
        cands.push_back({0, 0});
        for (int rpl : {2, 4, 8})
            if (8192 <= max_ch) cands.push_back({rpl, 8192});
        if (4096 <= max_ch) cands.push_back({4, 4096});
    }
    b->form = cands[0];
    b->tune.clear();
    if (cands.size() > 1) {
        // records of iteration 0, then one warm and one timed launch per candidate
        hipLaunchKernelGGL(k_b_init, dim3(ceil_div(std::max(ioff[count], 1), 256)), dim3(256), 0,
                           st, ioff[count], count, b->init_off.get(), b->gt.get(), b->lt.get(),
                           b->y.get());
        DRG_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_b_stage, dim3(ceil_div(N, 256)), dim3(256), 0, st, N, count, 0,
                           b->gid.get(), b->gt.get(), b->lt.get(), b->sched.get(), s->invZf.get(),
                           s->invZlo.get(), b->y.get(), s->rec.get());
        DRG_LAUNCH_CHECK();
        hipEvent_t e0, e1;
        DRG_HIP(hipEventCreate(&e0));
        DRG_HIP(hipEventCreate(&e1));
        float best = 0.0f;
        for (const SweepForm& f : cands) {
            launch_form(f, 0, st);
            DRG_HIP(hipEventRecord(e0, st));
            launch_form(f, 0, st);
            DRG_HIP(hipEventRecord(e1, st));
            DRG_HIP(hipEventSynchronize(e1));
            float ms = 0.0f;
            DRG_HIP(hipEventElapsedTime(&ms, e0, e1));
            b->tune.push_back({f, ms});
            if (b->tune.size() == 1 || ms < best) {
                best = ms;
                b->form = f;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    } else if (b->form.rpl > 0) {
        items_for(b->form.rpl);
    }
    // ---- record the whole run into a graph
    hipStream_t cap = nullptr;
    DRG_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    struct StreamGuard {
        hipStream_t s;
        ~StreamGuard() { (void)hipStreamDestroy(s); }
    } guard{cap};
    DRG_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    try {
        hipLaunchKernelGGL(k_b_init, dim3(ceil_div(ioff[count], 256)), dim3(256), 0, cap,
                           ioff[count], count, b->init_off.get(), b->gt.get(), b->lt.get(),
                           b->y.get());
        DRG_LAUNCH_CHECK();
        size_t ri = 0;
        auto prolong_rounds = [&](int32_t t) {
            for (; ri < rounds.size() && rounds[ri].t == t; ++ri) {
                const Round& r = rounds[ri];
                if (r.total > 0) {
                    hipLaunchKernelGGL(k_b_prolong, dim3(ceil_div(r.total, 256)), dim3(256), 0,
                                       cap, r.total, r.m, b->pro_off.get() + r.pfirst,
                                       b->pro_ops.get() + r.ofirst, b->gt.get(), b->lt.get(),
                                       b->y.get());
                    DRG_LAUNCH_CHECK();
                }
            }
        };
        for (int32_t t = 0; t < T; ++t) {
            prolong_rounds(t);
            hipLaunchKernelGGL(k_b_stage, dim3(ceil_div(N, 256)), dim3(256), 0, cap, N, count, t,
                               b->gid.get(), b->gt.get(), b->lt.get(), b->sched.get(),
                               s->invZf.get(), s->invZlo.get(), b->y.get(), s->rec.get());
            DRG_LAUNCH_CHECK();
            if (b->blk_count < count) launch_form(b->form, t, cap);
            launch_blocked(t, cap);
            const int32_t p = phase_of[t];
            const int32_t tot = phase_total[p];
            if (tot > 0) {
                hipLaunchKernelGGL(k_b_apply, dim3(ceil_div(tot, 256)), dim3(256), 0, cap, tot,
                                   count, t, b->phase_off.get() + (int64_t)p * (count + 1),
                                   b->gt.get(), b->lt.get(), b->sched.get(), s->g.get(),
                                   s->qtf.get(), b->y.get());
                DRG_LAUNCH_CHECK();
            }
        }
        prolong_rounds(T);
    } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(cap, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    DRG_HIP(hipStreamEndCapture(cap, &b->graph));
    if (b->form.rpl > 0) b->win_items = std::move(*items[b->form.rpl].first);
    DRG_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    return b.release();
}

void batch_run(drg_ctx* ctx, drg_batch* b, float* y_out) {
    if (!b || !y_out) throw Error(DRG_E_INVALID, "batch or y_out is NULL");
    if (b->device != ctx->device) throw Error(DRG_E_INVALID, "batch is of another device");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ctx->profiling) {
        DRG_HIP(hipEventCreate(&e0));
        DRG_HIP(hipEventCreate(&e1));
        DRG_HIP(hipEventRecord(e0, ctx->stream));
    }
    DRG_HIP(hipGraphLaunch(b->exec, ctx->stream));
    if (ctx->profiling) {
        DRG_HIP(hipEventRecord(e1, ctx->stream));
        ctx->events.emplace_back(e0, e1);
    }
    DRG_HIP(hipMemcpyAsync(y_out, b->y.get(), sizeof(float2) * b->n_total,
                           hipMemcpyDeviceToDevice, ctx->stream));
    DRG_HIP(hipStreamSynchronize(ctx->stream));
}

void batch_destroy(drg_batch* b) {
    if (!b) return;
    (void)hipSetDevice(b->device);
    delete b;
}

void batch_tuning(const drg_batch* b, int32_t cap, int32_t* n, int32_t* chosen, int32_t* rpl,
                  int32_t* ch, float* ms) {
    if (!b || !n) throw Error(DRG_E_INVALID, "batch or n is NULL");
    *n = (int32_t)b->tune.size();
    if (chosen) *chosen = -1;
    for (int32_t i = 0; i < (int32_t)b->tune.size(); ++i) {
        const auto& e = b->tune[i];
        if (chosen && e.first.rpl == b->form.rpl && e.first.ch == b->form.ch) *chosen = i;
        if (i >= cap) continue;
        if (rpl) rpl[i] = e.first.rpl;
        if (ch) ch[i] = e.first.ch;
        if (ms) ms[i] = e.second;
    }
}

void batch_info(const drg_batch* b, int64_t* n_total, int64_t* nnz_total, int32_t* T,
                int32_t* nodes, int32_t* levels) {
    if (!b) throw Error(DRG_E_INVALID, "batch is NULL");
    if (n_total) *n_total = b->n_total;
    if (nnz_total) *nnz_total = b->nnz_total;
    if (T) *T = b->T;
    for (int32_t c = 0; c < b->count; ++c) {
        if (nodes) nodes[c] = b->base[c + 1] - b->base[c];
        if (levels) levels[c] = b->levels[c];
    }
}

}  // namespace drg
