// layout3d.hip -- the layout iteration with positions in R^3 (Sec. 3.1:
// the positions may lie in R^2 or R^3).  The forces of Eq. gradient act
// along the offset y_i - y_j in any dimension, so the step is the 2-D one
// with a third component: attraction over the row of P~, gamma qt_i times
// the M drawn negatives, the members' steps averaged into their level node
// (Sec. 3.2.3), refinement by copying.  Coordinates are stored [n][3].
//
// This form runs the row sweep only (a group of lanes per row, records
// gathered from global memory): the column-blocked copy and the batched
// form hold 2-D records.  As in 2-D, every pair and every row sum is
// computed in FP64 from the records (x, y, z, 1/Z high part) plus the
// low part of 1/Z, whatever the coordinate type.
#include <type_traits>

#include "drg_forces.hpp"
#include "drg_internal.hpp"

namespace drg {

template <typename T>
__global__ void k_init3(int32_t n, uint64_t seed, int32_t level, T* __restrict__ y) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const U64x4 r =
        philox4x64((uint64_t)(uint32_t)v, (uint64_t)(uint32_t)level, 0, 0, seed, TAG_INIT);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const T u = (T)(uint32_t)(r.w[c] >> 40) * (T(1) / T(16777216));
        y[3 * v + c] = T(2) * u - T(1);
    }
}

template <typename T>
__global__ void k_prolong3(int32_t n, const int32_t* __restrict__ map, const T* __restrict__ yl,
                           T* __restrict__ yf) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    const int64_t a = map[u];
#pragma unroll
    for (int c = 0; c < 3; ++c) yf[3 * u + c] = yl[3 * a + c];
}

// rec[j] = (y_c(j), 1/Z_j high part)
template <typename T>
__global__ void k_stage3(int32_t n0, const int32_t* __restrict__ cmap, const T* __restrict__ y,
                         const T* __restrict__ invZ, typename VT<T>::v4* __restrict__ rec) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n0) return;
    const int64_t a = cmap ? cmap[j] : j;
    rec[j] = mk4<T>(y[3 * a], y[3 * a + 1], y[3 * a + 2], invZ[j]);
}

struct Sum3 {
    double x, y, z;
};

// g_i of row i, computed by the G lanes of a group (lane = 0..G-1): lane l
// takes pattern entries rs+l, rs+l+G, ... and negative slots l, l+G, ...;
// the lane partials are summed by a butterfly over the group.  lo: the low
// parts of 1/Z (NULL: the records hold 1/Z whole).
template <typename T, int B, bool CLIP, typename Draw>
__device__ __forceinline__ Sum3 sweep_row3(const typename VT<T>::v4& ri, double zi, int64_t rs,
                                           int64_t re, int lane, int G,
                                           const uint32_t* __restrict__ colhop,
                                           const typename VT<T>::v4* __restrict__ rec,
                                           const float* __restrict__ lo, const HalfE<double>& eh,
                                           double clip, bool half, int M, uint64_t seed,
                                           uint64_t iter, int32_t key, Draw draw, double gq,
                                           PairW pw) {
    double ax = 0.0, ay = 0.0, az = 0.0;
    for (int64_t x = rs + lane; x < re; x += G) {
        const uint32_t e = colhop[x];
        const int32_t j = (int32_t)(e & COL_MASK);
        const typename VT<T>::v4 rj = rec[j];
        const double dx = (double)ri.x - (double)rj.x, dy = (double)ri.y - (double)rj.y,
                     dz = (double)ri.z - (double)rj.z;
        const double d2 = dx * dx + dy * dy + dz * dz;
        const double k = attract_coef_b<B, double>(d2, half);
        double w;
        if (pw.A) {
            w = (pw.Ai[e >> 30] + pw.A[4 * (int64_t)j + (e >> 30)]) * 0.5;
        } else {
            const double zj = (double)rj.w + (lo ? (double)lo[j] : 0.0);
            w = (pw.Ex ? 0.5 * pw.Ex[x] : eh(e >> 30)) * (zi + zj);
        }
        if constexpr (CLIP) {
            ax += w * clampT2(k * dx, clip);
            ay += w * clampT2(k * dy, clip);
            az += w * clampT2(k * dz, clip);
        } else {
            const double wk = w * k;
            ax += wk * dx;
            ay += wk * dy;
            az += wk * dz;
        }
    }
    double rx = 0.0, ry = 0.0, rz = 0.0;
    for (int m = lane; m < M; m += G) {
        const typename VT<T>::v4 rv = rec[draw(neg_word(seed, iter, key, m))];
        const double dx = (double)ri.x - (double)rv.x, dy = (double)ri.y - (double)rv.y,
                     dz = (double)ri.z - (double)rv.z;
        const double d2 = dx * dx + dy * dy + dz * dz;
        if (d2 > 0.0) {
            const double k = repel_coef_b<B, double>(d2, half);
            rx += clampT2(k * dx, clip);
            ry += clampT2(k * dy, clip);
            rz += clampT2(k * dz, clip);
        }
    }
    // each lane's attraction + gq * repulsion, then one butterfly per axis
    double tx = ax + gq * rx, ty = ay + gq * ry, tz = az + gq * rz;
    tx = group_sum_rt(tx, G);
    ty = group_sum_rt(ty, G);
    tz = group_sum_rt(tz, G);
    return Sum3{tx, ty, tz};
}

template <typename T>
struct Sweep3Args {
    using v4 = typename VT<T>::v4;
    int32_t n0, M;
    const int64_t* prp;
    const uint32_t* colhop;
    const T* qt;
    const v4* rec;
    const float* lo;
    T* g;  // [n0][3] one-sided steps
    const uint64_t* C;
    const int32_t* guide;
    int32_t gbits;
    uint64_t S;
    double eh0, eh1, eh2, eh3;  // e_d / 2
    double gamma, clip;
    int32_t noclip;
    int32_t half;  // 1: the shape is b + 1/2
    const double* A;  // node-wise sigma: P~ table [n0][4] (NULL: global sigma)
    const double* Ex;  // weighted graph: E per entry [nnz] (NULL: e_d by hop)
    uint64_t seed, iter;
    // async only
    T* y;
    const int32_t* cmap;
    const T* invZ;
    const T* w;
    T eta;
};

template <typename T, int B, int G>
__global__ __launch_bounds__(256) void k_sweep3(Sweep3Args<T> a) {
    const int lane = threadIdx.x % G;
    const int64_t grp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    const int64_t ngrp = (int64_t)gridDim.x * blockDim.x / G;
    const HalfE<double> eh{a.eh0, a.eh1, a.eh2, a.eh3};
    auto draw = [&](uint64_t w) { return draw_node(w, a.C, a.guide, a.gbits, a.S); };
    for (int64_t i = grp; i < a.n0; i += ngrp) {
        const int64_t rs = a.prp[i], re = a.prp[i + 1];
        Sum3 gi{0.0, 0.0, 0.0};
        if (rs < re) {
            const typename VT<T>::v4 ri = a.rec[i];
            const double zi = (double)ri.w + (a.lo ? (double)a.lo[i] : 0.0);
            const double gq = a.gamma * (double)a.qt[i];
            if (a.noclip)
                gi = sweep_row3<T, B, false>(ri, zi, rs, re, lane, G, a.colhop, a.rec, a.lo, eh,
                                             a.clip, a.half != 0, a.M, a.seed, a.iter, (int32_t)i,
                                             draw, gq, pair_w(a.A, a.Ex, i));
            else
                gi = sweep_row3<T, B, true>(ri, zi, rs, re, lane, G, a.colhop, a.rec, a.lo, eh,
                                            a.clip, a.half != 0, a.M, a.seed, a.iter, (int32_t)i,
                                            draw, gq, pair_w(a.A, a.Ex, i));
        }
        if (lane == 0) {
            a.g[3 * i] = (T)gi.x;
            a.g[3 * i + 1] = (T)gi.y;
            a.g[3 * i + 2] = (T)gi.z;
        }
    }
}

// Hogwild: g_i from the live coordinates, eta g_i / w_c(i) added to y_c(i) at once
template <int B, int G>
__global__ __launch_bounds__(256) void k_sweep3_async(Sweep3Args<float> a) {
    const int lane = threadIdx.x % G;
    const int64_t grp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    const int64_t ngrp = (int64_t)gridDim.x * blockDim.x / G;
    volatile float* yv = a.y;
    for (int64_t i = grp; i < a.n0; i += ngrp) {
        const int64_t rs = a.prp[i], re = a.prp[i + 1];
        if (rs >= re) continue;
        const int64_t ci = a.cmap ? a.cmap[i] : i;
        const float yi0 = yv[3 * ci], yi1 = yv[3 * ci + 1], yi2 = yv[3 * ci + 2];
        const float zi = a.invZ[i];
        const PairW pw = pair_w(a.A, a.Ex, i);
        float ax = 0.0f, ay = 0.0f, az = 0.0f;
        for (int64_t x = rs + lane; x < re; x += G) {
            const uint32_t e = a.colhop[x];
            const int32_t j = (int32_t)(e & COL_MASK);
            const int64_t cj = a.cmap ? a.cmap[j] : j;
            const float dx = yi0 - yv[3 * cj], dy = yi1 - yv[3 * cj + 1], dz = yi2 - yv[3 * cj + 2];
            const float d2 = dx * dx + dy * dy + dz * dz;
            if (d2 > 0.0f) {
                const float k = attract_coef_b<B, float>(d2, a.half != 0);
                const uint32_t h = e >> 30;
                const float eh = (float)(h == 0 ? a.eh0 : (h == 1 ? a.eh1 : (h == 2 ? a.eh2 : a.eh3)));
                const float w = pw.A ? (float)((pw.Ai[h] + pw.A[4 * (int64_t)j + h]) * 0.5)
                                     : (pw.Ex ? (float)(0.5 * pw.Ex[x]) : eh) * (zi + a.invZ[j]);
                const float c = (float)a.clip;
                ax += w * clampT2(k * dx, c);
                ay += w * clampT2(k * dy, c);
                az += w * clampT2(k * dz, c);
            }
        }
        float rx = 0.0f, ry = 0.0f, rz = 0.0f;
        for (int m = lane; m < a.M; m += G) {
            const int32_t v = draw_node(neg_word(a.seed, a.iter, (int32_t)i, m), a.C, a.guide,
                                        a.gbits, a.S);
            const int64_t cv = a.cmap ? a.cmap[v] : v;
            const float dx = yi0 - yv[3 * cv], dy = yi1 - yv[3 * cv + 1], dz = yi2 - yv[3 * cv + 2];
            const float d2 = dx * dx + dy * dy + dz * dz;
            if (d2 > 0.0f) {
                const float k = repel_coef_b<B, float>(d2, a.half != 0);
                const float c = (float)a.clip;
                rx += repel_component(k, dx, c);
                ry += repel_component(k, dy, c);
                rz += repel_component(k, dz, c);
            }
        }
        ax = group_sum<G>(ax);
        ay = group_sum<G>(ay);
        az = group_sum<G>(az);
        rx = group_sum<G>(rx);
        ry = group_sum<G>(ry);
        rz = group_sum<G>(rz);
        if (lane == 0) {
            const float wc = a.w[ci];
            if (wc > 0.0f) {
                const float gq = (float)a.gamma * a.qt[i];
                const float s0 = a.eta * ((ax + gq * rx) / wc);
                const float s1 = a.eta * ((ay + gq * ry) / wc);
                const float s2 = a.eta * ((az + gq * rz) / wc);
                if (a.cmap) {
                    atomicAdd(&a.y[3 * ci], s0);
                    atomicAdd(&a.y[3 * ci + 1], s1);
                    atomicAdd(&a.y[3 * ci + 2], s2);
                } else {
                    yv[3 * ci] = yi0 + s0;
                    yv[3 * ci + 1] = yi1 + s1;
                    yv[3 * ci + 2] = yi2 + s2;
                }
            }
        }
    }
}

// Level-0 step: y_i += eta g_i / qt_i (nodes with qt_i = 0 stay)
template <typename T>
__global__ void k_apply3_0(int32_t n, const T* __restrict__ g, const T* __restrict__ qt,
                           T* __restrict__ y, T eta) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const T w = qt[i];
    if (!(w > T(0))) return;
#pragma unroll
    for (int c = 0; c < 3; ++c) y[3 * i + c] += eta * (g[3 * i + c] / w);
}

// Coarse-level step of level node a: its members' steps and anchor weights
// summed in ascending member id.
template <typename T>
__global__ void k_apply3_level(int32_t nl, const int32_t* __restrict__ seg,
                               const int32_t* __restrict__ perm, const T* __restrict__ g,
                               const T* __restrict__ qt, T* __restrict__ y, T eta) {
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= nl) return;
    T s0 = T(0), s1 = T(0), s2 = T(0), sw = T(0);
    for (int32_t x = seg[a]; x < seg[a + 1]; ++x) {
        const int64_t i = perm[x];
        s0 += g[3 * i];
        s1 += g[3 * i + 1];
        s2 += g[3 * i + 2];
        sw += qt[i];
    }
    if (!(sw > T(0))) return;
    y[3 * a] += eta * (s0 / sw);
    y[3 * a + 1] += eta * (s1 / sw);
    y[3 * a + 2] += eta * (s2 / sw);
}

template <typename T>
__global__ void k_level_weights3(int32_t nl, const int32_t* __restrict__ seg,
                                 const int32_t* __restrict__ perm, const T* __restrict__ qt,
                                 T* __restrict__ w) {
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= nl) return;
    T s = T(0);
    for (int32_t x = seg[a]; x < seg[a + 1]; ++x) s += qt[perm[x]];
    w[a] = s;
}

// ------------------------------------------------------------------ host
template <typename T, int B, int G>
static void launch3_one(hipStream_t st, const Sweep3Args<T>& a, bool async) {
    const int grid = (int)std::max<int64_t>(
        1, std::min<int64_t>(((int64_t)a.n0 * G + 255) / 256, (int64_t)1 << 22));
    if constexpr (std::is_same<T, float>::value) {
        if (async) {
            hipLaunchKernelGGL((k_sweep3_async<B, G>), dim3(grid), dim3(256), 0, st, a);
            DRG_LAUNCH_CHECK();
            return;
        }
    }
    hipLaunchKernelGGL((k_sweep3<T, B, G>), dim3(grid), dim3(256), 0, st, a);
    DRG_LAUNCH_CHECK();
}

template <typename T, int B>
static void launch3(hipStream_t st, const Sweep3Args<T>& a, int G, bool async) {
    switch (G) {
        case 4: launch3_one<T, B, 4>(st, a, async); break;
        case 8: launch3_one<T, B, 8>(st, a, async); break;
        case 16: launch3_one<T, B, 16>(st, a, async); break;
        case 32: launch3_one<T, B, 32>(st, a, async); break;
        default: launch3_one<T, B, 64>(st, a, async); break;
    }
}

template <typename T>
void init_layout3_t(drg_ctx* ctx, int32_t n, uint64_t seed, int32_t level, T* y) {
    if (n <= 0 || !y) throw Error(DRG_E_INVALID, "init_layout: n must be > 0 and y non-NULL");
    hipLaunchKernelGGL(k_init3<T>, dim3(ceil_div(n, 256)), dim3(256), 0, ctx->stream, n, seed,
                       level, y);
    DRG_LAUNCH_CHECK();
}

template <typename T>
void prolong3_t(drg_ctx* ctx, const drg_hier* h, int32_t level, const T* yl, T* yf) {
    if (!h || level < 1 || level >= (int32_t)h->lv.size() || !yl || !yf)
        throw Error(DRG_E_INVALID, "prolong: bad level or NULL pointer");
    const int32_t nf = h->lv[level - 1].n;
    hipLaunchKernelGGL(k_prolong3<T>, dim3(ceil_div(nf, 256)), dim3(256), 0, ctx->stream, nf,
                       h->lv[level].map.get(), yl, yf);
    DRG_LAUNCH_CHECK();
}

template <typename T>
void layout_step3_t(drg_ctx* ctx, drg_sim* s, const drg_hier* h, const drg_step_params* p, T* y) {
    constexpr bool F32 = std::is_same<T, float>::value;
    if (!s || !p || !y) throw Error(DRG_E_INVALID, "layout_step: NULL argument");
    if (p->M < 0) throw Error(DRG_E_INVALID, "layout_step: M >= 0");
    check_shape(p->b, p->b_half);
    if (!(p->clip > 0.0f)) throw Error(DRG_E_INVALID, "layout_step: clip must be > 0");
    if (p->mode != DRG_MODE_SYNC && p->mode != DRG_MODE_ASYNC)
        throw Error(DRG_E_INVALID, "layout_step: unknown mode");
    if (!F32 && p->mode == DRG_MODE_ASYNC)
        throw Error(DRG_E_UNSUPPORTED, "layout_step: the FP64 instance is synchronous only");
    const int32_t level = p->level;
    if (level < 0 || (level > 0 && (!h || level >= (int32_t)h->lv.size())))
        throw Error(DRG_E_INVALID, "layout_step: level out of range");
    if (h && h->n0 != s->n) throw Error(DRG_E_INVALID, "layout_step: hierarchy is of another graph");
    hipStream_t st = ctx->stream;
    const int32_t n0 = s->n;
    const int32_t nl = level == 0 ? n0 : h->lv[level].n;
    const int32_t* cmap = level == 0 ? nullptr : h->lv[level].cmap.get();
    using v4 = typename VT<T>::v4;
    const T* invZ;
    const T* qt;
    v4* rec;
    T* g;
    if constexpr (F32) {
        invZ = s->invZf.get();
        qt = s->qtf.get();
        rec = s->rec.get();
        if (!s->g3.get()) s->g3.alloc(3 * (int64_t)n0);
        g = s->g3.get();
    } else {
        if (!s->rec64.get()) s->rec64.alloc(n0);
        if (!s->g3_64.get()) s->g3_64.alloc(3 * (int64_t)n0);
        invZ = s->invZ.get();
        qt = s->qt.get();
        rec = s->rec64.get();
        g = s->g3_64.get();
    }
    Sweep3Args<T> a{};
    a.n0 = n0;
    a.M = s->S > 0 ? p->M : 0;
    a.prp = s->row_ptr.get();
    a.colhop = s->colhop.get();
    a.qt = qt;
    a.rec = rec;
    a.lo = F32 ? s->invZlo.get() : nullptr;
    a.g = g;
    a.C = s->C.get();
    a.guide = s->guide.get();
    a.gbits = s->gbits;
    a.S = s->S;
    a.eh0 = 0.5 * s->e[0];
    a.eh1 = 0.5 * s->e[1];
    a.eh2 = 0.5 * s->e[2];
    a.eh3 = 0.5 * s->e[3];
    a.gamma = (double)p->gamma;
    a.clip = (double)p->clip;
    a.noclip = attract_clip_free(p->b + (p->b_half ? 0.5 : 0.0), p->clip) ? 1 : 0;
    a.half = p->b_half ? 1 : 0;
    a.A = s->A.get();
    a.Ex = s->Ex.get();
    a.seed = p->seed;
    a.iter = p->iter;
    a.y = y;
    a.cmap = cmap;
    a.invZ = invZ;
    a.eta = (T)p->eta;
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
                hipLaunchKernelGGL(k_level_weights3<float>, dim3(ceil_div(nl, 256)), dim3(256), 0, st,
                                   nl, L.seg.get(), L.perm.get(), s->qtf.get(), s->wlev.get());
                DRG_LAUNCH_CHECK();
                s->wlev_hier = h->uid;
                s->wlev_level = level;
            }
            a.w = reinterpret_cast<const T*>(s->wlev.get());
        }
    } else {
        hipLaunchKernelGGL(k_stage3<T>, dim3(ceil_div(n0, 256)), dim3(256), 0, st, n0, cmap, y,
                           invZ, rec);
        DRG_LAUNCH_CHECK();
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ctx->profiling) {
        DRG_HIP(hipEventCreate(&e0));
        DRG_HIP(hipEventCreate(&e1));
        DRG_HIP(hipEventRecord(e0, st));
    }
    const int G = sweep_group(s->len_wmean, s->n_active);
    switch (p->b) {
        case 1: launch3<T, 1>(st, a, G, async); break;
        case 2: launch3<T, 2>(st, a, G, async); break;
        default: launch3<T, 3>(st, a, G, async); break;
    }
    if (ctx->profiling) {
        DRG_HIP(hipEventRecord(e1, st));
        ctx->events.emplace_back(e0, e1);
    }
    ctx->last_sweep = async ? DRG_SWEEP_ROW_ASYNC : DRG_SWEEP_ROW;
    if (async) return;
    if (level == 0) {
        hipLaunchKernelGGL(k_apply3_0<T>, dim3(ceil_div(n0, 256)), dim3(256), 0, st, n0, g, qt, y,
                           (T)p->eta);
    } else {
        const drg_level& L = h->lv[level];
        hipLaunchKernelGGL(k_apply3_level<T>, dim3(ceil_div(nl, 256)), dim3(256), 0, st, nl,
                           L.seg.get(), L.perm.get(), g, qt, y, (T)p->eta);
    }
    DRG_LAUNCH_CHECK();
}

template void init_layout3_t<float>(drg_ctx*, int32_t, uint64_t, int32_t, float*);
template void init_layout3_t<double>(drg_ctx*, int32_t, uint64_t, int32_t, double*);
template void prolong3_t<float>(drg_ctx*, const drg_hier*, int32_t, const float*, float*);
template void prolong3_t<double>(drg_ctx*, const drg_hier*, int32_t, const double*, double*);
template void layout_step3_t<float>(drg_ctx*, drg_sim*, const drg_hier*, const drg_step_params*,
                                    float*);
template void layout_step3_t<double>(drg_ctx*, drg_sim*, const drg_hier*, const drg_step_params*,
                                     double*);

}  // namespace drg
