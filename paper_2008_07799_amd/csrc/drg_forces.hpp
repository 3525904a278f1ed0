// drg_forces.hpp -- the per-pair forces of Eq. gradient and small vector
// helpers, shared by the single-graph and the batched iteration kernels so
// both evaluate every pair with the same operations.
#pragma once
#include "drg_common.hpp"

namespace drg {

template <typename T>
struct VT;
template <>
struct VT<float> {
    using v2 = float2;
    using v4 = float4;
};
template <>
struct VT<double> {
    using v2 = double2;
    using v4 = double4;
};

template <typename T>
__device__ __forceinline__ typename VT<T>::v2 mk2(T a, T b) {
    typename VT<T>::v2 r;
    r.x = a;
    r.y = b;
    return r;
}
template <typename T>
__device__ __forceinline__ typename VT<T>::v4 mk4(T a, T b, T c, T d) {
    typename VT<T>::v4 r;
    r.x = a;
    r.y = b;
    r.z = c;
    r.w = d;
    return r;
}

template <typename T>
__device__ __forceinline__ T clampT(T v, T c) {
    return v > c ? c : (v < -c ? -c : v);
}

template <int B, typename T>
__device__ __forceinline__ T powT(T x) {
    if constexpr (B == 0) return T(1);
    else if constexpr (B == 1) return x;
    else if constexpr (B == 2) return x * x;
    else return x * x * x;
}

// 1/x in FP64 for x > 0: the hardware estimate (v_rcp_f64) refined by two
// Newton-Raphson steps, each squaring the relative error; within an ulp of
// the correctly rounded quotient at a fraction of the cost of the full
// division sequence.  x = +inf gives 0, as the division does.  (From FP32
// coordinates the arguments below are at least 2^-298, far above the
// denormal range.)
__device__ __forceinline__ double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    return x <= 1.7976931348623157e308 ? r : 0.0;
}

// attraction coefficient -2b d^{2b-2}/(1+d^{2b}); repulsion 2b/(d^2 (1+d^{2b}));
// FP32 uses the hardware reciprocal (1 ulp), FP64 the refined one.
template <typename T>
__device__ __forceinline__ T recipT(T x) {
    if constexpr (std::is_same<T, float>::value) return rcp_fast(x);
    else return rcp_nr(x);
}
template <int B, typename T>
__device__ __forceinline__ T attract_coef(T d2) {
    return T(-2 * B) * powT<B - 1>(d2) * recipT(T(1) + powT<B>(d2));
}
template <int B, typename T>
__device__ __forceinline__ T repel_coef(T d2) {
    return T(2 * B) * recipT(d2 * (T(1) + powT<B>(d2)));
}

// The same for b = B + 1/2 (half = true): d^{2b} = (d^2)^B d and
// d^{2b-2} = (d^2)^{B-1} d with d = sqrt(d^2).  half is uniform over a
// launch; a whole b takes the functions above unchanged.
template <typename T>
__device__ __forceinline__ T sqrtT(T x) {
    if constexpr (std::is_same<T, float>::value) return __builtin_sqrtf(x);
    else return __builtin_sqrt(x);
}
template <int B, typename T>
__device__ __forceinline__ T attract_coef_b(T d2, bool half) {
    if (!half) return attract_coef<B, T>(d2);
    const T d = sqrtT(d2);
    return T(-(2 * B + 1)) * (powT<B - 1>(d2) * d) * recipT(T(1) + powT<B>(d2) * d);
}
template <int B, typename T>
__device__ __forceinline__ T repel_coef_b(T d2, bool half) {
    if (!half) return repel_coef<B, T>(d2);
    const T d = sqrtT(d2);
    return T(2 * B + 1) * recipT(d2 * (T(1) + powT<B>(d2) * d));
}

template <typename T>
__device__ __forceinline__ T clampT2(T v, T c) {
    if constexpr (std::is_same<T, float>::value) return clampf(v, c);
    else return v > c ? c : (v < -c ? -c : v);
}
template <typename T>
__device__ __forceinline__ T repelT(T k, T d, T c) {
    if constexpr (std::is_same<T, float>::value) return repel_component(k, d, c);
    else return clampT2(k * d, c);
}

// ------------------------------------------------------------------ per-node steps
// These bodies are the whole arithmetic of one node in the iteration; the
// single-graph and the batched kernels call them with the same arguments, so
// a graph laid out inside a batch reproduces its single-graph layout bit for
// bit.

// Random initial point of node v at `level`: uniform in [-1, 1)^2 from the
// top 24 bits of two Philox words.
template <typename T>
__device__ __forceinline__ typename VT<T>::v2 init_point(int32_t v, int32_t level, uint64_t seed) {
    const U64x4 r =
        philox4x64((uint64_t)(uint32_t)v, (uint64_t)(uint32_t)level, 0, 0, seed, TAG_INIT);
    const T ux = (T)(uint32_t)(r.w[0] >> 40) * (T(1) / T(16777216));
    const T uy = (T)(uint32_t)(r.w[1] >> 40) * (T(1) / T(16777216));
    return mk2<T>(T(2) * ux - T(1), T(2) * uy - T(1));
}

// e_d / 2 for hops 1..4
template <typename T>
struct HalfE {
    T h0, h1, h2, h3;
    // two selects on the bits of h (no branches)
    __device__ __forceinline__ T operator()(uint32_t h) const {
        const T lo = (h & 1u) ? h1 : h0;
        const T hi = (h & 1u) ? h3 : h2;
        return (h & 2u) ? hi : lo;
    }
};

// Pair weight P~_ij of pattern entry x, by form WM (a compile-time choice,
// so the default form carries no per-pair branch):
//   PW_HOP   one global sigma: e_d/2 (1/Z_i + 1/Z_j) from the records;
//   PW_NODE  node-wise sigma: (A_i[d] + A_j[d]) / 2 from the table A [n][4]
//            (A_i[d] = NS_{j|i} at hop d+1; Ai = A + 4 i);
//   PW_ENTRY weighted graph: E_x/2 (1/Z_i + 1/Z_j) with E per entry.
constexpr int PW_HOP = 0, PW_NODE = 1, PW_ENTRY = 2;
struct PairW {
    const double* A = nullptr;   // the node table (PW_NODE)
    const double* Ai = nullptr;  // row i's four values (PW_NODE)
    const double* Ex = nullptr;  // per-entry E (PW_ENTRY)
};
__device__ __forceinline__ PairW pair_w(const double* __restrict__ A,
                                        const double* __restrict__ Ex, int64_t i) {
    PairW p;
    p.A = A;
    p.Ai = A ? A + 4 * i : nullptr;
    p.Ex = Ex;
    return p;
}
// Attraction of one pattern entry e (record rj) on the node with record ri,
// added to the lane's partial (ax, ay).  Records hold (x, y, 1/Z high part,
// 1/Z low part) in the coordinate type T; the pair's arithmetic and the
// partials are FP64 whatever T is: these row forms are bound by the gathers,
// not by arithmetic, and FP64 terms keep the FP32 trajectory within the
// rounding of its stored coordinates.  Coincident nodes contribute nothing;
// no test is needed for that: at d2 = 0 the coefficient is finite (-2b for
// b = 1, -0 otherwise) and dx = dy = +0, so both terms are zeros, which leave
// the partial's value unchanged.  CLIP = false when the clip cannot bind
// (|k dx| stays below it for every offset): the clamp would return its
// argument, so it is left out and the weight is folded into k first.
template <typename T, int B, bool CLIP = true, int WM = PW_HOP>
__device__ __forceinline__ void attract_pair(const typename VT<T>::v4& ri, uint32_t e,
                                             const typename VT<T>::v4& rj, const HalfE<double>& eh,
                                             double clip, bool half, double& ax, double& ay,
                                             const PairW& pw = PairW{}, int64_t x = 0) {
    const double dx = (double)ri.x - (double)rj.x, dy = (double)ri.y - (double)rj.y;
    const double d2 = dx * dx + dy * dy;
    const double k = attract_coef_b<B, double>(d2, half);
    double w;
    if constexpr (WM == PW_NODE) {
        w = (pw.Ai[e >> 30] + pw.A[4 * (int64_t)(e & COL_MASK) + (e >> 30)]) * 0.5;
    } else {
        const double zi = (double)ri.z + (double)ri.w, zj = (double)rj.z + (double)rj.w;
        if constexpr (WM == PW_ENTRY)
            w = (0.5 * pw.Ex[x]) * (zi + zj);
        else
            w = eh(e >> 30) * (zi + zj);
    }
    if constexpr (CLIP) {
        ax += w * clampT2(k * dx, clip);
        ay += w * clampT2(k * dy, clip);
    } else {
        const double wk = w * k;
        ax += wk * dx;
        ay += wk * dy;
    }
}

// Repulsion partial of lane `lane` of G: negative slots lane, lane+G, ...
template <typename T, int B, typename Draw>
__device__ __forceinline__ void repel_lane(const typename VT<T>::v4& ri,
                                           const typename VT<T>::v4* __restrict__ rec, int lane,
                                           int G, int M, uint64_t seed, uint64_t iter, int32_t key,
                                           Draw draw, double clip, bool half, double& rx,
                                           double& ry) {
    rx = 0.0;
    ry = 0.0;
    for (int m = lane; m < M; m += G) {
        const uint64_t w = neg_word(seed, iter, key, m);
        const typename VT<T>::v4 rv = rec[draw(w)];
        const double dx = (double)ri.x - (double)rv.x, dy = (double)ri.y - (double)rv.y;
        const double d2 = dx * dx + dy * dy;
        if (d2 > 0.0) {
            const double k = repel_coef_b<B, double>(d2, half);
            rx += clampT2(k * dx, clip);
            ry += clampT2(k * dy, clip);
        }
    }
}

// g_i = attraction + gq * repulsion: each lane combines its own partials,
// then butterfly sums over the group (two values, not four: the butterflies
// are a large part of a short row's work), rounded once to the coordinate
// type.
template <typename T>
__device__ __forceinline__ typename VT<T>::v2 row_total(double ax, double ay, double rx,
                                                        double ry, int G, double gq) {
    double tx = ax + gq * rx, ty = ay + gq * ry;
    tx = group_sum_rt(tx, G);
    ty = group_sum_rt(ty, G);
    return mk2<T>((T)tx, (T)ty);
}

// One row of the sweep, computed by the G lanes of a group (lane = 0..G-1):
// lane l takes pattern entries rs+l, rs+l+G, ... in that order and negative
// slots l, l+G, ...; the lane partials are then summed by a butterfly over
// the group.  Returns g_i (valid in every lane) = attraction + gq *
// repulsion, where `key` is the node's own id for the negative words and
// draw(w) turns a word into the record index of the drawn node.
template <typename T, int B, bool CLIP, int WM = PW_HOP, int U = 2, typename Draw>
__device__ __forceinline__ typename VT<T>::v2 sweep_row(
    const typename VT<T>::v4& ri, int64_t rs, int64_t re, int lane, int G,
    const uint32_t* __restrict__ colhop, const typename VT<T>::v4* __restrict__ rec,
    const HalfE<double>& eh, double clip, bool half, int M, uint64_t seed, uint64_t iter,
    int32_t key, Draw draw, double gq, const PairW& pw = PairW{}) {
    using v4 = typename VT<T>::v4;
    double ax = 0.0, ay = 0.0;
    // U entries per step; the next step's entries are loaded while this
    // step's records are gathered and used (the terms still go in order, so
    // U does not change the result).  Two by default: with FP64 pair terms
    // four in flight need 92-96 VGPRs (5 waves per SIMD) against 70-72 (7
    // waves), and the more waves hide the gathers better (R-MAT 2^20 at
    // k = 1: 1.04 vs 1.15 ms per sweep; the 512-graph batch's row sweep 1.46
    // vs 1.65 ms per iteration).
    const int64_t step = (int64_t)U * G;
    int64_t x = rs + lane;
    uint32_t e[U];
    bool full = x + (int64_t)(U - 1) * G < re;
    if (full) {
#pragma unroll
        for (int q = 0; q < U; ++q) e[q] = colhop[x + (int64_t)q * G];
    }
    while (full) {
        v4 rj[U];
#pragma unroll
        for (int q = 0; q < U; ++q) rj[q] = rec[e[q] & COL_MASK];
        const int64_t xn = x + step;
        const bool next = xn + (int64_t)(U - 1) * G < re;
        // past the row the loads are clamped to its last entry (and unused)
        const int64_t xl = next ? xn : re - 1 - (int64_t)(U - 1) * G;
        uint32_t en[U];
#pragma unroll
        for (int q = 0; q < U; ++q) en[q] = colhop[max(xl + (int64_t)q * G, x)];
#pragma unroll
        for (int q = 0; q < U; ++q)
            attract_pair<T, B, CLIP, WM>(ri, e[q], rj[q], eh, clip, half, ax, ay, pw,
                                         x + (int64_t)q * G);
#pragma unroll
        for (int q = 0; q < U; ++q) e[q] = en[q];
        x = xn;
        full = next;
    }
    for (; x < re; x += G) {
        const uint32_t e = colhop[x];
        attract_pair<T, B, CLIP, WM>(ri, e, rec[e & COL_MASK], eh, clip, half, ax, ay, pw, x);
    }
    double rx, ry;
    repel_lane<T, B>(ri, rec, lane, G, M, seed, iter, key, draw, clip, half, rx, ry);
    return row_total<T>(ax, ay, rx, ry, G, gq);
}

// ------------------------------------------------------------------ windowed sweep
// The same per-lane order with the gathered records taken from LDS: a
// workgroup owns the rows of one item (rows r0 .. r0+nrows-1 of one graph,
// all columns inside [c0, c1)).  Its groups of G lanes each hold RPL rows;
// the column window is staged chunk by chunk (CH records) and every lane
// continues its rows' entries, in ascending position, up to the chunk's end.
// Each lane thus adds exactly the terms it adds in sweep_row, in the same
// order, so the result is bit-identical to sweep_row; only the source of the
// neighbour records (LDS instead of global memory) differs.
struct WinItem {
    int32_t graph;     // batch graph index (0 for a single graph)
    int32_t r0, nrows; // rows
    int32_t c0, c1;    // column window
    int32_t pad[3];
};

template <int B, bool CLIP, int RPL, int BLOCK, typename Draw, typename Key>
__device__ __forceinline__ void window_item(
    const WinItem& it, int G, float4* __restrict__ lds, int CH,
    const int64_t* __restrict__ prp, const uint32_t* __restrict__ colhop,
    const float4* __restrict__ rec, const float* __restrict__ qt, const HalfE<double>& eh,
    double clip, bool half, int M, uint64_t seed, uint64_t iter, double gamma, Draw draw, Key key,
    float2* __restrict__ g) {
    const int tid = threadIdx.x;
    const int NG = BLOCK / G;
    const int lane = tid % G, grp = tid / G;
    double ax[RPL], ay[RPL];
    int64_t xs[RPL], xe[RPL];
    float4 ri[RPL];
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
        const int32_t r = grp + k * NG;
        ax[k] = 0.0;
        ay[k] = 0.0;
        xs[k] = 0;
        xe[k] = 0;
        if (r < it.nrows) {
            const int64_t i = (int64_t)it.r0 + r;
            xs[k] = prp[i] + lane;
            xe[k] = prp[i + 1];
            ri[k] = rec[i];
        }
    }
    for (int32_t b0 = it.c0; b0 < it.c1; b0 += CH) {
        const int32_t b1 = min(b0 + CH, it.c1);
        __syncthreads();
        for (int32_t j = tid; j < b1 - b0; j += BLOCK) lds[j] = rec[b0 + j];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            int64_t x = xs[k];
            const int64_t e_end = xe[k];
            double sx = ax[k], sy = ay[k];
            constexpr int U = 4;  // entry loads in flight; past-the-end slots read a sentinel
            while (x < e_end) {
                uint32_t e[U];
#pragma unroll
                for (int q = 0; q < U; ++q) {
                    const int64_t xq = x + (int64_t)q * G;
                    e[q] = xq < e_end ? colhop[xq] : 0xFFFFFFFFu;
                }
                int q = 0;
#pragma unroll
                for (; q < U; ++q) {
                    const int32_t c = (int32_t)(e[q] & COL_MASK);
                    if (c >= b1) break;
                    attract_pair<float, B, CLIP>(ri[k], e[q], lds[c - b0], eh, clip, half, sx,
                                                 sy);
                }
                x += (int64_t)q * G;
                if (q < U) break;
            }
            xs[k] = x;
            ax[k] = sx;
            ay[k] = sy;
        }
    }
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
        const int32_t r = grp + k * NG;
        if (r >= it.nrows) continue;
        const int64_t i = (int64_t)it.r0 + r;
        float2 gi = make_float2(0.0f, 0.0f);
        if (prp[i] < prp[i + 1]) {
            double rx, ry;
            repel_lane<float, B>(ri[k], rec, lane, G, M, seed, iter, key(i), draw, clip, half, rx,
                                 ry);
            gi = row_total<float>(ax[k], ay[k], rx, ry, G, gamma * (double)qt[i]);
        }
        if (lane == 0) g[i] = gi;
    }
}

// Finest-level step of node i: y_i += eta g_i / qt_i (nodes with qt_i = 0 stay).
template <typename T>
__device__ __forceinline__ void apply_node(const typename VT<T>::v2& s, T w,
                                           typename VT<T>::v2* __restrict__ yp, T eta) {
    if (!(w > T(0))) return;
    typename VT<T>::v2 p = *yp;
    p.x += eta * (s.x / w);
    p.y += eta * (s.y / w);
    *yp = p;
}

// Coarse-level step of level node a: the members' steps and anchor weights
// summed in ascending member id (perm[x] + pbase indexes g and qt).
template <typename T>
__device__ __forceinline__ void apply_group(int32_t xb, int32_t xe, const int32_t* __restrict__ perm,
                                            int64_t pbase, const typename VT<T>::v2* __restrict__ g,
                                            const T* __restrict__ qt,
                                            typename VT<T>::v2* __restrict__ yp, T eta) {
    T sx = T(0), sy = T(0), sw = T(0);
    for (int32_t x = xb; x < xe; ++x) {
        const int64_t i = pbase + perm[x];
        const typename VT<T>::v2 s = g[i];
        sx += s.x;
        sy += s.y;
        sw += qt[i];
    }
    if (sw > T(0)) {
        typename VT<T>::v2 p = *yp;
        p.x += eta * (sx / sw);
        p.y += eta * (sy / sw);
        *yp = p;
    }
}

// Coarse-level steps of the level nodes held by the lanes of one wave (all
// 64 lanes call it; valid = the lane holds a node).  A node with at most
// APPLY_SEQ members is summed by its own lane (apply_group); a larger one by
// the whole wave: lane l adds members l, l+64, ... in ascending order, then
// a fixed butterfly, and the node's lane applies the step.  So a node with
// many members (the centre of a large star) does not hold up its wave for
// thousands of serial steps, and the order of the sums is fixed by the data.
constexpr int APPLY_SEQ = 64;

template <typename T>
__device__ __forceinline__ void apply_level_wave(bool valid, int32_t xb, int32_t xe,
                                                 const int32_t* perm, int64_t pbase,
                                                 const typename VT<T>::v2* __restrict__ g,
                                                 const T* __restrict__ qt,
                                                 typename VT<T>::v2* yp, T eta) {
    const bool big = valid && xe - xb > APPLY_SEQ;
    if (valid && !big) apply_group<T>(xb, xe, perm, pbase, g, qt, yp, eta);
    uint64_t m = __ballot(big);
    const int lane = __lane_id();
    while (m) {
        const int src = __ffsll((unsigned long long)m) - 1;
        m &= m - 1;
        const int32_t b0 = __builtin_amdgcn_readlane(xb, src);
        const int32_t b1 = __builtin_amdgcn_readlane(xe, src);
        const uint64_t pp = (uint64_t)(uintptr_t)perm;
        const uint64_t pu = (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)pp, src) |
                            ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int32_t)(pp >> 32), src) << 32);
        const int32_t* P = reinterpret_cast<const int32_t*>((uintptr_t)pu);
        const int64_t pb = (int64_t)((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)pbase, src) |
                                     ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(
                                          (int32_t)((uint64_t)pbase >> 32), src) << 32));
        T sx = T(0), sy = T(0), sw = T(0);
        for (int32_t x = b0 + lane; x < b1; x += WAVE) {
            const int64_t i = pb + P[x];
            const typename VT<T>::v2 v = g[i];
            sx += v.x;
            sy += v.y;
            sw += qt[i];
        }
        sx = group_sum<WAVE>(sx);
        sy = group_sum<WAVE>(sy);
        sw = group_sum<WAVE>(sw);
        if (lane == src && sw > T(0)) {
            typename VT<T>::v2 p = *yp;
            p.x += eta * (sx / sw);
            p.y += eta * (sy / sw);
            *yp = p;
        }
    }
}

}  // namespace drg
