// layout.hip -- one optimisation iteration of the layout (Sec. 3.2.2,
// Eq. gradient) with the gradient sharing across levels (Sec. 3.2.3), the
// random initial layout and the refinement step.
//
// Sync iteration at level l, three launches on one stream:
//   stage : rec[j] = (y_l[c_l(j)], 1/Z_j) for every finest node j, so the
//           sweep gathers one record per neighbour at every level;
//   sweep : for every non-isolated finest node i, G lanes walk row i of P~
//           (coalesced 4-byte entries, gathered records), then draw M
//           negatives from (seed, iter, i, m) and gather theirs; the lane
//           partials are reduced in a fixed order into g_i;
//   apply : y_l[a] += eta * (sum g_i) / (sum qt_i) over the members i of a,
//           in ascending id (no atomics: the iteration is bit-for-bit
//           repeatable).  Node i is chosen about qt_i times per iteration by
//           the paper's SGD; applied at once from one snapshot, those steps
//           become one step along their average.
// Async iteration: one launch; each g_i is computed from the live y and
// eta g_i / w_{c(i)} is added to y_l[c_l(i)] at once (Hogwild-style).
//
// Every kernel is templated on the coordinate type: float is the product
// path; the double instance runs the same arithmetic for trajectory checks.
#include <type_traits>

#include "drg_forces.hpp"
#include "drg_internal.hpp"

namespace drg {

template <typename T>
__global__ void k_init(int32_t n, uint64_t seed, int32_t level, typename VT<T>::v2* __restrict__ y) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) y[v] = init_point<T>((int32_t)v, level, seed);
}

template <typename T>
__global__ void k_prolong(int32_t n, const int32_t* __restrict__ map,
                          const typename VT<T>::v2* __restrict__ yl,
                          typename VT<T>::v2* __restrict__ yf) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u < n) yf[u] = yl[map[u]];
}

// invZlo (FP32 records only, else NULL): 1/Z_j - (float)(1/Z_j), so the
// record carries 1/Z_j to about 48 bits for the FP64 pair arithmetic.
template <typename T>
__global__ void k_stage(int32_t n0, const int32_t* __restrict__ cmap,
                        const typename VT<T>::v2* __restrict__ y, const T* __restrict__ invZ,
                        const float* __restrict__ invZlo, typename VT<T>::v4* __restrict__ rec) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n0) return;
    const typename VT<T>::v2 p = y[cmap ? cmap[j] : (int32_t)j];
    rec[j] = mk4<T>(p.x, p.y, invZ[j], invZlo ? (T)invZlo[j] : T(0));
}

template <typename T>
struct SweepArgs {
    using v2 = typename VT<T>::v2;
    using v4 = typename VT<T>::v4;
    int32_t n0;
    int32_t M;
    const int64_t* prp;
    const uint32_t* colhop;
    const T* qt;
    const v4* rec;
    v2* g;
    const uint64_t* C;
    const int32_t* guide;
    int32_t gbits;
    uint64_t S;
    double eh0, eh1, eh2, eh3;  // e_d / 2
    T gamma, clip;
    int32_t noclip;        // the attraction clip cannot bind (attract_clip_free)
    int32_t half;          // b = B + 1/2
    const double* A;       // node-wise sigma: P~ table [n0][4] (NULL: global sigma)
    const double* Ex;      // weighted graph: E per entry [nnz] (NULL: e_d by hop)
    uint64_t seed, iter;
    // async only
    v2* y;
    const int32_t* cmap;
    const T* invZ;
    const T* w;            // anchor weight of each level node
    T eta;
};

template <typename T>
__device__ __forceinline__ T half_e(const SweepArgs<T>& a, uint32_t h) {
    return (T)(h == 0 ? a.eh0 : (h == 1 ? a.eh1 : (h == 2 ? a.eh2 : a.eh3)));
}

// WM: the pair-weight form (PW_HOP, PW_NODE, PW_ENTRY), one kernel each so
// that the common form keeps its register budget
template <typename T, int B, int G, int WM>
__global__ __launch_bounds__(256) void k_sweep(SweepArgs<T> a) {
    const int lane = threadIdx.x % G;
    const int64_t grp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    const int64_t ngrp = (int64_t)gridDim.x * blockDim.x / G;
    const HalfE<double> eh{a.eh0, a.eh1, a.eh2, a.eh3};
    auto rows = [&](auto clip_c) {
        constexpr bool CLIP = decltype(clip_c)::value;
        for (int64_t i = grp; i < a.n0; i += ngrp) {
            const int64_t rs = a.prp[i], re = a.prp[i + 1];
            typename VT<T>::v2 gi = mk2<T>(T(0), T(0));
            if (rs < re)
                gi = sweep_row<T, B, CLIP, WM>(a.rec[i], rs, re, lane, G, a.colhop, a.rec, eh,
                                               (double)a.clip, a.half != 0,
                                               a.M, a.seed, a.iter, (int32_t)i,
                                               [&](uint64_t w) {
                                                   return draw_node(w, a.C, a.guide, a.gbits,
                                                                    a.S);
                                               },
                                               (double)a.gamma * (double)a.qt[i],
                                               pair_w(a.A, a.Ex, i));
            if (lane == 0) a.g[i] = gi;
        }
    };
    // the node-wise and per-entry weights run with the clamp in place
    if (WM == PW_HOP && a.noclip)
        rows(std::false_type{});
    else
        rows(std::true_type{});
}

// Windowed form of k_sweep (same result bit for bit): one workgroup per item.
template <int B, int RPL>
__global__ __launch_bounds__(WIN_BLOCK) void k_sweep_win(const WinItem* __restrict__ items, int G,
                                                         int CH, SweepArgs<float> a) {
    extern __shared__ float4 s_rec[];
    const HalfE<double> eh{a.eh0, a.eh1, a.eh2, a.eh3};
    const WinItem it = items[xcd_block((int32_t)blockIdx.x, (int32_t)gridDim.x)];
    auto draw = [&](uint64_t w) { return draw_node(w, a.C, a.guide, a.gbits, a.S); };
    auto key = [&](int64_t i) { return (int32_t)i; };
    if (a.noclip)
        window_item<B, false, RPL, WIN_BLOCK>(it, G, s_rec, CH, a.prp, a.colhop, a.rec, a.qt, eh,
                                              a.clip, a.half != 0, a.M, a.seed, a.iter, a.gamma,
                                              draw, key, a.g);
    else
        window_item<B, true, RPL, WIN_BLOCK>(it, G, s_rec, CH, a.prp, a.colhop, a.rec, a.qt, eh,
                                             a.clip, a.half != 0, a.M, a.seed, a.iter, a.gamma,
                                             draw, key, a.g);
}

template <int B, int RPL>
static void launch_win_rpl(drg_ctx* ctx, drg_sim* s, const SweepArgs<float>& a, int G) {
    const int CH = win_chunk(ctx);
    const size_t lds = (size_t)CH * sizeof(float4);
    auto fn = k_sweep_win<B, RPL>;
    DRG_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds));
    hipLaunchKernelGGL(fn, dim3(s->win_n), dim3(WIN_BLOCK), lds, ctx->stream, s->win_items.get(),
                       G, CH, a);
    DRG_LAUNCH_CHECK();
}

template <int B>
static void launch_win(drg_ctx* ctx, drg_sim* s, const SweepArgs<float>& a, int G) {
    switch (s->win_rpl) {
        case 1: launch_win_rpl<B, 1>(ctx, s, a, G); break;
        case 2: launch_win_rpl<B, 2>(ctx, s, a, G); break;
        case 4: launch_win_rpl<B, 4>(ctx, s, a, G); break;
        default: launch_win_rpl<B, 8>(ctx, s, a, G); break;
    }
}

// rec (nullable): the records of the next iteration at this level take the
// new positions here, so that iteration needs no staging pass.
template <typename T>
__global__ void k_apply0(int32_t n, const typename VT<T>::v2* __restrict__ g,
                         const T* __restrict__ qt, typename VT<T>::v2* __restrict__ y, T eta,
                         typename VT<T>::v4* __restrict__ rec) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    apply_node<T>(g[i], qt[i], y + i, eta);
    if (rec) {
        const typename VT<T>::v2 p = y[i];
        rec[i].x = p.x;
        rec[i].y = p.y;
    }
}

// One lane per level node: the members' steps and anchor weights summed in
// ascending member id, by the whole wave for nodes with many members.
template <typename T>
__global__ __launch_bounds__(256) void k_apply_level(int32_t nl, const int32_t* __restrict__ seg,
                                                     const int32_t* __restrict__ perm,
                                                     const typename VT<T>::v2* __restrict__ g,
                                                     const T* __restrict__ qt,
                                                     typename VT<T>::v2* __restrict__ y, T eta) {
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = a < nl;
    const int64_t v = valid ? a : 0;
    if (__ballot(valid) == 0) return;  // the whole wave leaves
    apply_level_wave<T>(valid, valid ? seg[v] : 0, valid ? seg[v + 1] : 0, perm, 0, g, qt, y + v,
                        eta);
}

template <typename T>
__global__ void k_level_weights(int32_t nl, const int32_t* __restrict__ seg,
                                const int32_t* __restrict__ perm, const T* __restrict__ qt,
                                T* __restrict__ w) {
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= nl) return;
    T s = T(0);
    for (int32_t x = seg[a]; x < seg[a + 1]; ++x) s += qt[perm[x]];
    w[a] = s;
}

// A node's two coordinates as one 64-bit access, so a concurrent reader sees
// both from before or both from after an update (never x from one and y
// from the other, a position the layout never held).
__device__ __forceinline__ float2 pos_load(const float2* p) {
    const uint64_t v = __hip_atomic_load(reinterpret_cast<uint64_t*>(const_cast<float2*>(p)),
                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return make_float2(__uint_as_float((uint32_t)v), __uint_as_float((uint32_t)(v >> 32)));
}
__device__ __forceinline__ void pos_store(float2* p, float x, float y) {
    const uint64_t v = (uint64_t)__float_as_uint(x) | ((uint64_t)__float_as_uint(y) << 32);
    __hip_atomic_store(reinterpret_cast<uint64_t*>(p), v, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// Hogwild: reads the live coordinates, adds eta g_i / w_{c(i)} to y[c(i)] at once.
template <int B, int G>
__global__ __launch_bounds__(256) void k_sweep_async(SweepArgs<float> a) {
    const int lane = threadIdx.x % G;
    const int64_t grp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    const int64_t ngrp = (int64_t)gridDim.x * blockDim.x / G;
    for (int64_t i = grp; i < a.n0; i += ngrp) {
        const int64_t rs = a.prp[i], re = a.prp[i + 1];
        if (rs >= re) continue;
        const int32_t ci = a.cmap ? a.cmap[i] : (int32_t)i;
        const float2 pi = pos_load(a.y + ci);
        const float yix = pi.x, yiy = pi.y;
        const float zi = a.invZ[i];
        const PairW pw = pair_w(a.A, a.Ex, i);
        float ax = 0.0f, ay = 0.0f;
        for (int64_t x = rs + lane; x < re; x += G) {
            const uint32_t e = a.colhop[x];
            const int32_t j = (int32_t)(e & COL_MASK);
            const int32_t cj = a.cmap ? a.cmap[j] : j;
            const float2 pj = pos_load(a.y + cj);
            const float dx = yix - pj.x, dy = yiy - pj.y;
            const float d2 = dx * dx + dy * dy;
            if (d2 > 0.0f) {
                const float k = attract_coef_b<B, float>(d2, a.half != 0);
                const float w = pw.A ? (float)((pw.Ai[e >> 30] + pw.A[4 * j + (e >> 30)]) * 0.5)
                                : (pw.Ex ? (float)(0.5 * pw.Ex[x]) : half_e(a, e >> 30)) *
                                      (zi + a.invZ[j]);
                ax += w * clampT2(k * dx, a.clip);
                ay += w * clampT2(k * dy, a.clip);
            }
        }
        float rx = 0.0f, ry = 0.0f;
        for (int m = lane; m < a.M; m += G) {
            const uint64_t w = neg_word(a.seed, a.iter, (int32_t)i, m);
            const int32_t v = draw_node(w, a.C, a.guide, a.gbits, a.S);
            const int32_t cv = a.cmap ? a.cmap[v] : v;
            const float2 pv = pos_load(a.y + cv);
            const float dx = yix - pv.x, dy = yiy - pv.y;
            const float d2 = dx * dx + dy * dy;
            if (d2 > 0.0f) {
                const float k = repel_coef_b<B, float>(d2, a.half != 0);
                rx += repelT(k, dx, a.clip);
                ry += repelT(k, dy, a.clip);
            }
        }
        ax = group_sum<G>(ax);
        ay = group_sum<G>(ay);
        rx = group_sum<G>(rx);
        ry = group_sum<G>(ry);
        if (lane == 0) {
            const float wc = a.w[ci];
            if (wc > 0.0f) {
                const float gq = a.gamma * a.qt[i];
                const float sx = a.eta * ((ax + gq * rx) / wc);
                const float sy = a.eta * ((ay + gq * ry) / wc);
                if (a.cmap) {
                    atomicAdd(&a.y[ci].x, sx);
                    atomicAdd(&a.y[ci].y, sy);
                } else {
                    pos_store(a.y + ci, yix + sx, yiy + sy);
                }
            }
        }
    }
}

template <typename T, int B, int G>
static void launch_one(hipStream_t st, const SweepArgs<T>& a, bool async) {
    const int64_t groups = a.n0;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((groups * G + 255) / 256,
                                                                 (int64_t)1 << 22));
    if constexpr (std::is_same<T, float>::value) {
        if (async) {
            hipLaunchKernelGGL((k_sweep_async<B, G>), dim3(grid), dim3(256), 0, st, a);
            DRG_LAUNCH_CHECK();
            return;
        }
    }
    switch (a.A ? PW_NODE : (a.Ex ? PW_ENTRY : PW_HOP)) {
        case PW_NODE:
            hipLaunchKernelGGL((k_sweep<T, B, G, PW_NODE>), dim3(grid), dim3(256), 0, st, a);
            break;
        case PW_ENTRY:
            hipLaunchKernelGGL((k_sweep<T, B, G, PW_ENTRY>), dim3(grid), dim3(256), 0, st, a);
            break;
        default: hipLaunchKernelGGL((k_sweep<T, B, G, PW_HOP>), dim3(grid), dim3(256), 0, st, a);
    }
    DRG_LAUNCH_CHECK();
}

template <typename T, int B>
static void launch_sweep(hipStream_t st, const SweepArgs<T>& a, int G, bool async) {
    switch (G) {
        case 4: launch_one<T, B, 4>(st, a, async); break;
        case 8: launch_one<T, B, 8>(st, a, async); break;
        case 16: launch_one<T, B, 16>(st, a, async); break;
        case 32: launch_one<T, B, 32>(st, a, async); break;
        default: launch_one<T, B, 64>(st, a, async); break;
    }
}

template <typename T>
void init_layout_t(drg_ctx* ctx, int32_t n, uint64_t seed, int32_t level, T* y) {
    if (n <= 0 || !y) throw Error(DRG_E_INVALID, "init_layout: n must be > 0 and y non-NULL");
    hipLaunchKernelGGL(k_init<T>, dim3(ceil_div(n, 256)), dim3(256), 0, ctx->stream, n, seed,
                       level, reinterpret_cast<typename VT<T>::v2*>(y));
    DRG_LAUNCH_CHECK();
}

template <typename T>
void prolong_t(drg_ctx* ctx, const drg_hier* h, int32_t level, const T* yl, T* yf) {
    if (!h || level < 1 || level >= (int32_t)h->lv.size() || !yl || !yf)
        throw Error(DRG_E_INVALID, "prolong: bad level or NULL pointer");
    const int32_t nf = h->lv[level - 1].n;
    hipLaunchKernelGGL(k_prolong<T>, dim3(ceil_div(nf, 256)), dim3(256), 0, ctx->stream, nf,
                       h->lv[level].map.get(), reinterpret_cast<const typename VT<T>::v2*>(yl),
                       reinterpret_cast<typename VT<T>::v2*>(yf));
    DRG_LAUNCH_CHECK();
}

template void init_layout_t<float>(drg_ctx*, int32_t, uint64_t, int32_t, float*);
template void init_layout_t<double>(drg_ctx*, int32_t, uint64_t, int32_t, double*);
template void prolong_t<float>(drg_ctx*, const drg_hier*, int32_t, const float*, float*);
template void prolong_t<double>(drg_ctx*, const drg_hier*, int32_t, const double*, double*);

void init_layout(drg_ctx* ctx, int32_t n, uint64_t seed, int32_t level, float* y) {
    init_layout_t<float>(ctx, n, seed, level, y);
}
void prolong(drg_ctx* ctx, const drg_hier* h, int32_t level, const float* yl, float* yf) {
    prolong_t<float>(ctx, h, level, yl, yf);
}

template <typename T>
void layout_step_t(drg_ctx* ctx, drg_sim* s, const drg_hier* h, const drg_step_params* p, T* y,
                   bool staged, bool restage) {
    constexpr bool F32 = std::is_same<T, float>::value;
    if (!s || !p || !y) throw Error(DRG_E_INVALID, "layout_step: NULL argument");
    check_shape(p->b, p->b_half);
    if (p->M < 0) throw Error(DRG_E_INVALID, "layout_step: M >= 0");
    if (!(p->clip > 0.0f)) throw Error(DRG_E_INVALID, "layout_step: clip must be > 0");
    if (p->mode != DRG_MODE_SYNC && p->mode != DRG_MODE_ASYNC)
        throw Error(DRG_E_INVALID, "layout_step: unknown mode");
    if (!F32 && p->mode == DRG_MODE_ASYNC)
        throw Error(DRG_E_UNSUPPORTED, "layout_step: the FP64 instance is synchronous only");
    const bool half = p->b_half != 0;
    const int32_t level = p->level;
    if (level < 0 || (level > 0 && (!h || level >= (int32_t)h->lv.size())))
        throw Error(DRG_E_INVALID, "layout_step: level out of range");
    if (h && h->n0 != s->n)
        throw Error(DRG_E_INVALID, "layout_step: hierarchy is of another graph");
    hipStream_t st = ctx->stream;
    const int32_t n0 = s->n;
    const int32_t nl = level == 0 ? n0 : h->lv[level].n;
    const int32_t* cmap = level == 0 ? nullptr : h->lv[level].cmap.get();
    using v2 = typename VT<T>::v2;
    using v4 = typename VT<T>::v4;
    const T* invZ;
    const T* qt;
    v4* rec;
    v2* g;
    if constexpr (F32) {
        invZ = s->invZf.get();
        qt = s->qtf.get();
        rec = s->rec.get();
        g = s->g.get();
    } else {
        if (!s->rec64.get()) s->rec64.alloc(n0);
        if (!s->g64.get()) s->g64.alloc(n0);
        invZ = s->invZ.get();
        qt = s->qt.get();
        rec = s->rec64.get();
        g = s->g64.get();
    }
    SweepArgs<T> a{};
    a.n0 = n0;
    a.M = s->S > 0 ? p->M : 0;
    a.prp = s->row_ptr.get();
    a.colhop = s->colhop.get();
    a.qt = qt;
    a.rec = rec;
    a.g = g;
    a.C = s->C.get();
    a.guide = s->guide.get();
    a.gbits = s->gbits;
    a.S = s->S;
    a.eh0 = 0.5 * s->e[0];
    a.eh1 = 0.5 * s->e[1];
    a.eh2 = 0.5 * s->e[2];
    a.eh3 = 0.5 * s->e[3];
    a.gamma = (T)p->gamma;
    a.clip = (T)p->clip;
    a.noclip = attract_clip_free(p->b + (half ? 0.5 : 0.0), p->clip) ? 1 : 0;
    a.half = half ? 1 : 0;
    a.A = s->A.get();
    a.Ex = s->Ex.get();
    a.seed = p->seed;
    a.iter = p->iter;
    a.y = reinterpret_cast<v2*>(y);
    a.cmap = cmap;
    a.invZ = invZ;
    a.eta = (T)p->eta;
    const int G = sweep_group(s->len_wmean, s->n_active);
    // Both modes stage the records on the column-blocked layout: its Hogwild
    // form reads neighbours from LDS copies of the records and updates them
    // in place as windows of rows finish.
    // the blocked sweep: whole b, one global sigma (node-wise sims have no
    // blocked copy)
    const bool blocked = F32 && s->blk_nb > 0 && !half && !a.A && !a.Ex;
    const bool async = p->mode == DRG_MODE_ASYNC;
    if (async) {
        if (level == 0) {
            a.w = qt;
        } else {
            if (!s->wlev.get()) s->wlev.alloc(n0);
            // a level node's anchor weight (its members' q~ summed) is fixed
            // for the level: computed once per (hierarchy, level)
            if (s->wlev_hier != h->uid || s->wlev_level != level) {
                const drg_level& L = h->lv[level];
                hipLaunchKernelGGL(k_level_weights<float>, dim3(ceil_div(nl, 256)), dim3(256), 0, st,
                                   nl, L.seg.get(), L.perm.get(), s->qtf.get(), s->wlev.get());
                DRG_LAUNCH_CHECK();
                s->wlev_hier = h->uid;
                s->wlev_level = level;
            }
            a.w = reinterpret_cast<const T*>(s->wlev.get());
        }
    }
    // staged: the records already hold y (the previous level-0 sync step of
    // a schedule wrote them); restage: this level-0 sync step writes them
    if (async || level != 0) staged = restage = false;
    if ((!async || blocked) && !staged) {
        hipLaunchKernelGGL(k_stage<T>, dim3(ceil_div(n0, 256)), dim3(256), 0, st, n0, cmap,
                           reinterpret_cast<const v2*>(y), invZ, F32 ? s->invZlo.get() : nullptr,
                           rec);
        DRG_LAUNCH_CHECK();
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ctx->profiling) {
        DRG_HIP(hipEventCreate(&e0));
        DRG_HIP(hipEventCreate(&e1));
    }
    if constexpr (F32) {
        if (blocked && async) {
            sweep_blocked_async(ctx, s, p->b, a.M, a.gamma, a.clip, a.eta, a.seed, a.iter, y,
                                cmap, a.w, e0, e1);
            if (ctx->profiling) ctx->events.emplace_back(e0, e1);
            ctx->last_sweep = DRG_SWEEP_BLOCKED_ASYNC;
            return;
        }
        if (blocked) {
            // LDS-staged sweep over the column-blocked pattern
            ctx->last_sweep = DRG_SWEEP_BLOCKED;
            sweep_blocked(ctx, s, p->b, a.M, a.gamma, a.clip, a.seed, a.iter, g, e0, e1);
            if (ctx->profiling) ctx->events.emplace_back(e0, e1);
            if (level == 0) {
                hipLaunchKernelGGL(k_apply0<T>, dim3(ceil_div(n0, 256)), dim3(256), 0, st, n0, g,
                                   qt, reinterpret_cast<v2*>(y), (T)p->eta,
                                   restage ? rec : nullptr);
            } else {
                const drg_level& L = h->lv[level];
                hipLaunchKernelGGL(k_apply_level<T>, dim3(ceil_div(nl, 256)), dim3(256), 0, st, nl,
                                   L.seg.get(), L.perm.get(), g, qt, reinterpret_cast<v2*>(y),
                                   (T)p->eta);
            }
            DRG_LAUNCH_CHECK();
            return;
        }
    }
    bool win = false;
    if constexpr (F32) {
        if (!async && !a.A && !a.Ex && window_wanted(s)) {
            const int rpl = win_rpl();
            if (s->win_rpl != rpl) {
                s->win_n = build_window_items(ctx, s, {0, n0}, {(WIN_BLOCK / G) * rpl},
                                              s->win_items);
                s->win_rpl = rpl;
            }
            win = s->win_n > 0;
        }
    }
    ctx->last_sweep = async ? DRG_SWEEP_ROW_ASYNC : (win ? DRG_SWEEP_WINDOW : DRG_SWEEP_ROW);
    if (ctx->profiling) DRG_HIP(hipEventRecord(e0, st));
    if (win) {
        if constexpr (F32) {
            switch (p->b) {
                case 1: launch_win<1>(ctx, s, a, G); break;
                case 2: launch_win<2>(ctx, s, a, G); break;
                default: launch_win<3>(ctx, s, a, G); break;
            }
        }
    } else {
        switch (p->b) {
            case 1: launch_sweep<T, 1>(st, a, G, async); break;
            case 2: launch_sweep<T, 2>(st, a, G, async); break;
            default: launch_sweep<T, 3>(st, a, G, async); break;
        }
    }
    if (ctx->profiling) {
        DRG_HIP(hipEventRecord(e1, st));
        ctx->events.emplace_back(e0, e1);
    }
    if (!async) {
        if (level == 0) {
            hipLaunchKernelGGL(k_apply0<T>, dim3(ceil_div(n0, 256)), dim3(256), 0, st, n0, g, qt,
                               reinterpret_cast<v2*>(y), (T)p->eta, restage ? rec : nullptr);
        } else {
            const drg_level& L = h->lv[level];
            hipLaunchKernelGGL(k_apply_level<T>, dim3(ceil_div(nl, 256)), dim3(256), 0, st, nl,
                               L.seg.get(), L.perm.get(), g, qt, reinterpret_cast<v2*>(y),
                               (T)p->eta);
        }
        DRG_LAUNCH_CHECK();
    }
}

template void layout_step_t<float>(drg_ctx*, drg_sim*, const drg_hier*, const drg_step_params*,
                                   float*, bool, bool);
template void layout_step_t<double>(drg_ctx*, drg_sim*, const drg_hier*, const drg_step_params*,
                                    double*, bool, bool);

void layout_step(drg_ctx* ctx, drg_sim* s, const drg_hier* h, const drg_step_params* p,
                 float* y, bool staged, bool restage) {
    layout_step_t<float>(ctx, s, h, p, y, staged, restage);
}

// Everything a synchronous FP32 step builds on first use, built now (before
// a step is recorded into a graph).
void prepare_sync_step(drg_ctx* ctx, drg_sim* s) {
    if (s->blk_nb > 0 || s->A.get() || s->Ex.get() || !window_wanted(s)) return;
    const int G = sweep_group(s->len_wmean, s->n_active);
    const int rpl = win_rpl();
    if (s->win_rpl != rpl) {
        s->win_n = build_window_items(ctx, s, {0, s->n}, {(WIN_BLOCK / G) * rpl}, s->win_items);
        s->win_rpl = rpl;
    }
}

}  // namespace drg
