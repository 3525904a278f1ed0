// objective.hip -- the sampled objective L^ (Eq. objectfunction) and its
// gradient, for use inside an autograd system, plus exports used to check
// it (the drawn negatives, P~ as device COO).
//
//   L^(Y) = sum_i sum_j P~_ij log w_ij + gamma sum_i qt_i sum_{m<M} log(1 - w_{i v_im})
//   log w = -log1p(d^{2b}),  log(1 - w) = b log d^2 - log1p(d^{2b})
//
// b is a whole number B or B + 1/2 (half): d^{2b} = (d^2)^B sqrt(d^2).
//
// A negative equal to its anchor, or at distance 0, contributes nothing.
// Gradient (unclipped): the attraction of row i appears in rows i and j with
// the same P~ (symmetric), so it is twice row i's sum; the repulsion term of
// (u, m) moves both u (own side) and v_um (other side).  The backward draws
// every negative again from its counter; the other-side terms are grouped by
// drawn node with a stable sort of (v, pair index) and summed in pair order,
// so the gradient is deterministic.
#include <cstdlib>

#include <mutex>
#include <string>

#include "drg_internal.hpp"

namespace drg {

template <typename T>
struct OV;
template <>
struct OV<float> {
    using v2 = float2;
};
template <>
struct OV<double> {
    using v2 = double2;
};

template <typename T>
__device__ __forceinline__ typename OV<T>::v2 mk2o(T a, T b) {
    typename OV<T>::v2 r;
    r.x = a;
    r.y = b;
    return r;
}

// 1/x: the hardware reciprocal in FP32 (1 ulp), division in FP64
template <typename T>
__device__ __forceinline__ T orcp(T x) {
    if constexpr (std::is_same<T, float>::value) return rcp_fast(x);
    else return T(1) / x;
}

template <int B, typename T>
__device__ __forceinline__ T opow(T x) {
    if constexpr (B == 0) return T(1);
    else if constexpr (B == 1) return x;
    else if constexpr (B == 2) return x * x;
    else return x * x * x;
}

// d^{2b} and d^{2b-2} from d2 = d^2, b = B or B + 1/2
template <int B, typename T>
__device__ __forceinline__ T opow_b(T d2, bool half) {
    const T u = opow<B>(d2);
    return half ? u * sqrtT(d2) : u;
}
template <int B, typename T>
__device__ __forceinline__ T opow_bm1(T d2, bool half) {
    const T u = opow<B - 1>(d2);
    return half ? u * sqrtT(d2) : u;
}

template <typename T>
struct ObjArgs {
    using v2 = typename OV<T>::v2;
    int32_t n, M;
    const int64_t* prp;
    const uint32_t* colhop;
    const T* invZ;
    const T* qt;
    const v2* y;
    const uint64_t* C;
    const int32_t* guide;
    int32_t gbits;
    uint64_t S;
    T eh0, eh1, eh2, eh3;  // e_d / 2
    T gamma;
    T bv;                  // b as a number: B, or B + 1/2 when half
    int32_t half;          // 1: b = B + 1/2
    const double* A;       // node-wise sigma: P~ table [n][4] (NULL: global sigma)
    const double* Ex;      // weighted graph: E per entry [nnz] (NULL: e_d by hop)
    uint64_t seed, iter;
    const T* dloss;        // backward: scale (NULL = 1)
    T* row_val;            // forward: per-row value
    v2* dy;                // backward: gradient
    const T* y3;           // 3-D layouts: coordinates [n][3]
    T* dy3;                // 3-D layouts: gradient [n][3]
};

template <typename T>
__device__ __forceinline__ T oh(const ObjArgs<T>& a, uint32_t h) {
    return h == 0 ? a.eh0 : (h == 1 ? a.eh1 : (h == 2 ? a.eh2 : a.eh3));
}

// P~_ij of entry x at hop index h: (A_i[h] + A_j[h]) / 2 with node-wise
// sigma, E_x/2 (1/Z_i + 1/Z_j) for a weighted graph, else e_h/2 (1/Z_i + 1/Z_j)
template <typename T>
__device__ __forceinline__ T obj_p(const ObjArgs<T>& a, int64_t i, int32_t j, uint32_t h, T zi,
                                   int64_t x) {
    if (a.A) return (T)((a.A[4 * i + h] + a.A[4 * (int64_t)j + h]) * 0.5);
    return (a.Ex ? (T)(0.5 * a.Ex[x]) : oh(a, h)) * (zi + a.invZ[j]);
}

template <typename T>
__device__ __forceinline__ T log1pT(T x) {
    if constexpr (std::is_same<T, float>::value) return log1p_fast(x);
    else return log1p(x);
}
template <typename T>
__device__ __forceinline__ T logT(T x) {
    if constexpr (std::is_same<T, float>::value) return logf(x);
    else return log(x);
}

template <typename T, int B, int G>
__global__ __launch_bounds__(256) void k_obj_rows(ObjArgs<T> a) {
    const int lane = threadIdx.x % G;
    const int64_t grp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    const int64_t ngrp = (int64_t)gridDim.x * blockDim.x / G;
    for (int64_t i = grp; i < a.n; i += ngrp) {
        const int64_t rs = a.prp[i], re = a.prp[i + 1];
        T val = T(0);
        if (rs < re) {
            const typename OV<T>::v2 yi = a.y[i];
            const T zi = a.invZ[i];
            T att = T(0), rep = T(0);
            for (int64_t x = rs + lane; x < re; x += G) {
                const uint32_t e = a.colhop[x];
                const int32_t j = (int32_t)(e & COL_MASK);
                const typename OV<T>::v2 yj = a.y[j];
                const T dx = yi.x - yj.x, dy = yi.y - yj.y;
                const T d2 = dx * dx + dy * dy;
                const T p = obj_p(a, i, j, e >> 30, zi, x);
                att += p * (-log1pT(opow_b<B>(d2, a.half != 0)));
            }
            for (int m = lane; m < a.M; m += G) {
                const int32_t v =
                    draw_node(neg_word(a.seed, a.iter, (int32_t)i, m), a.C, a.guide, a.gbits, a.S);
                if (v == (int32_t)i) continue;
                const typename OV<T>::v2 yv = a.y[v];
                const T dx = yi.x - yv.x, dy = yi.y - yv.y;
                const T d2 = dx * dx + dy * dy;
                if (d2 > T(0)) rep += a.bv * logT(d2) - log1pT(opow_b<B>(d2, a.half != 0));
            }
            att = group_sum<G>(att);
            rep = group_sum<G>(rep);
            val = att + a.gamma * a.qt[i] * rep;
        }
        if (lane == 0) a.row_val[i] = val;
    }
}

// Sum of n values in a fixed order: block sums of 1024 then one block.
template <typename T>
__global__ __launch_bounds__(1024) void k_sum_blocks(int64_t n, const T* __restrict__ v,
                                                     T* __restrict__ out) {
    __shared__ T s[1024 / WAVE];
    const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    T x = i < n ? v[i] : T(0);
    x = block_sum<1024>(x, s);
    if (threadIdx.x == 0) out[blockIdx.x] = x;
}

template <typename T, int B, int G>
__global__ __launch_bounds__(256) void k_grad_rows(ObjArgs<T> a) {
    const int lane = threadIdx.x % G;
    const int64_t grp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    const int64_t ngrp = (int64_t)gridDim.x * blockDim.x / G;
    const T dl = a.dloss ? *a.dloss : T(1);
    for (int64_t i = grp; i < a.n; i += ngrp) {
        const int64_t rs = a.prp[i], re = a.prp[i + 1];
        T gx = T(0), gy = T(0);
        if (rs < re) {
            const typename OV<T>::v2 yi = a.y[i];
            const T zi = a.invZ[i];
            T ax = T(0), ay = T(0), rx = T(0), ry = T(0);
            for (int64_t x = rs + lane; x < re; x += G) {
                const uint32_t e = a.colhop[x];
                const int32_t j = (int32_t)(e & COL_MASK);
                const typename OV<T>::v2 yj = a.y[j];
                const T dx = yi.x - yj.x, dy = yi.y - yj.y;
                const T d2 = dx * dx + dy * dy;
                const T p = obj_p(a, i, j, e >> 30, zi, x);
                const T k = p * (T(-2) * a.bv) * opow_bm1<B>(d2, a.half != 0) *
                            orcp(T(1) + opow_b<B>(d2, a.half != 0));
                ax += k * dx;
                ay += k * dy;
            }
            for (int m = lane; m < a.M; m += G) {
                const int32_t v =
                    draw_node(neg_word(a.seed, a.iter, (int32_t)i, m), a.C, a.guide, a.gbits, a.S);
                if (v == (int32_t)i) continue;
                const typename OV<T>::v2 yv = a.y[v];
                const T dx = yi.x - yv.x, dy = yi.y - yv.y;
                const T d2 = dx * dx + dy * dy;
                if (d2 > T(0)) {
                    const T k = (T(2) * a.bv) * orcp(d2 * (T(1) + opow_b<B>(d2, a.half != 0)));
                    rx += k * dx;
                    ry += k * dy;
                }
            }
            ax = group_sum<G>(ax);
            ay = group_sum<G>(ay);
            rx = group_sum<G>(rx);
            ry = group_sum<G>(ry);
            const T gq = a.gamma * a.qt[i];
            gx = T(2) * ax + gq * rx;
            gy = T(2) * ay + gq * ry;
        }
        if (lane == 0) a.dy[i] = mk2o<T>(dl * gx, dl * gy);
    }
}

// FP32 with the column-blocked layout: the attraction terms come per (block,
// row) from the flat blocked sweep; one thread per row adds them in block
// order, adds its own negatives and writes the row value (KIND 0) or the
// row's own gradient (KIND 1).
template <int B, int KIND>
__global__ void k_obj_finish(ObjArgs<float> a, int32_t nb, const float2* __restrict__ partial) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const float dl = (KIND == 1 && a.dloss) ? *a.dloss : 1.0f;
    if (a.prp[i] >= a.prp[i + 1]) {
        if constexpr (KIND == 0) a.row_val[i] = 0.0f;
        else a.dy[i] = make_float2(0.0f, 0.0f);
        return;
    }
    float ax = 0.0f, ay = 0.0f;
    for (int32_t b = 0; b < nb; ++b) {
        const float2 p = partial[(int64_t)b * a.n + i];
        ax += p.x;
        ay += p.y;
    }
    const float2 yi = a.y[i];
    float rx = 0.0f, ry = 0.0f;
    for (int m = 0; m < a.M; ++m) {
        const int32_t v =
            draw_node(neg_word(a.seed, a.iter, (int32_t)i, m), a.C, a.guide, a.gbits, a.S);
        if (v == (int32_t)i) continue;
        const float2 yv = a.y[v];
        const float dx = yi.x - yv.x, dy = yi.y - yv.y;
        const float d2 = dx * dx + dy * dy;
        if (!(d2 > 0.0f)) continue;
        if constexpr (KIND == 0) {
            rx += (float)B * logf(d2) - log1p_fast(opow<B>(d2));
        } else {
            const float k = (float)(2 * B) * rcp_fast(d2 * (1.0f + opow<B>(d2)));
            rx += k * dx;
            ry += k * dy;
        }
    }
    const float gq = a.gamma * a.qt[i];
    if constexpr (KIND == 0) {
        a.row_val[i] = ax + gq * rx;
    } else {
        a.dy[i] = make_float2(dl * (2.0f * ax + gq * rx), dl * (2.0f * ay + gq * ry));
    }
}

// key = drawn node (n for "none": inactive anchor or self draw), value = u*M+m
__global__ void k_neg_keys(int32_t n, int32_t M, const int64_t* __restrict__ prp,
                           const uint64_t* __restrict__ C, const int32_t* __restrict__ guide,
                           int32_t gbits, uint64_t S, uint64_t seed, uint64_t iter,
                           uint32_t* __restrict__ keys, int32_t* __restrict__ vals) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (int64_t)n * M) return;
    const int32_t u = (int32_t)(p / M), m = (int32_t)(p % M);
    uint32_t key = (uint32_t)n;
    if (prp[u + 1] > prp[u] && S > 0) {
        const int32_t v = draw_node(neg_word(seed, iter, u, m), C, guide, gbits, S);
        if (v != u) key = (uint32_t)v;
    }
    keys[p] = key;
    vals[p] = (int32_t)p;
}

__global__ void k_key_bounds(int64_t np, int32_t n, const uint32_t* __restrict__ keys,
                             int32_t* __restrict__ seg) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c > n) return;
    int64_t lo = 0, hi = np;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)keys[mid] < c)
            lo = mid + 1;
        else
            hi = mid;
    }
    seg[c] = (int32_t)lo;
}

// dy[v] += dl * sum over the pairs (u, m) that drew v, in pair order, of
// gamma qt_u R(y_v - y_u)
template <typename T, int B>
__global__ void k_other_side(ObjArgs<T> a, const int32_t* __restrict__ seg,
                             const int32_t* __restrict__ pairs) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= a.n) return;
    const int32_t s = seg[v], e = seg[v + 1];
    if (s == e) return;
    const T dl = a.dloss ? *a.dloss : T(1);
    const typename OV<T>::v2 yv = a.y[v];
    T gx = T(0), gy = T(0);
    for (int32_t x = s; x < e; ++x) {
        const int32_t u = pairs[x] / a.M;
        const typename OV<T>::v2 yu = a.y[u];
        const T dx = yv.x - yu.x, dy = yv.y - yu.y;
        const T d2 = dx * dx + dy * dy;
        if (d2 > T(0)) {
            const T k = a.gamma * a.qt[u] * (T(2) * a.bv) /
                        (d2 * (T(1) + opow_b<B>(d2, a.half != 0)));
            gx += k * dx;
            gy += k * dy;
        }
    }
    typename OV<T>::v2 o = a.dy[v];
    o.x += dl * gx;
    o.y += dl * gy;
    a.dy[v] = o;
}

// ------------------------------------------------------------------ 3-D layouts
// The same objective and gradient with positions in R^3 (Sec. 3.1): the terms
// depend on the squared distance only, the forces act along the offset.
template <typename T>
__device__ __forceinline__ T off3(const T* __restrict__ y, int64_t i, int64_t j, T& dx, T& dy,
                                  T& dz) {
    dx = y[3 * i] - y[3 * j];
    dy = y[3 * i + 1] - y[3 * j + 1];
    dz = y[3 * i + 2] - y[3 * j + 2];
    return dx * dx + dy * dy + dz * dz;
}

template <typename T, int B, int G>
__global__ __launch_bounds__(256) void k_obj_rows3(ObjArgs<T> a) {
    const int lane = threadIdx.x % G;
    const int64_t grp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    const int64_t ngrp = (int64_t)gridDim.x * blockDim.x / G;
    for (int64_t i = grp; i < a.n; i += ngrp) {
        const int64_t rs = a.prp[i], re = a.prp[i + 1];
        T val = T(0);
        if (rs < re) {
            const T zi = a.invZ[i];
            T att = T(0), rep = T(0), dx, dy, dz;
            for (int64_t x = rs + lane; x < re; x += G) {
                const uint32_t e = a.colhop[x];
                const int32_t j = (int32_t)(e & COL_MASK);
                const T d2 = off3(a.y3, i, j, dx, dy, dz);
                att += obj_p(a, i, j, e >> 30, zi, x) * (-log1pT(opow_b<B>(d2, a.half != 0)));
            }
            for (int m = lane; m < a.M; m += G) {
                const int32_t v =
                    draw_node(neg_word(a.seed, a.iter, (int32_t)i, m), a.C, a.guide, a.gbits, a.S);
                if (v == (int32_t)i) continue;
                const T d2 = off3(a.y3, i, v, dx, dy, dz);
                if (d2 > T(0)) rep += a.bv * logT(d2) - log1pT(opow_b<B>(d2, a.half != 0));
            }
            att = group_sum<G>(att);
            rep = group_sum<G>(rep);
            val = att + a.gamma * a.qt[i] * rep;
        }
        if (lane == 0) a.row_val[i] = val;
    }
}

template <typename T, int B, int G>
__global__ __launch_bounds__(256) void k_grad_rows3(ObjArgs<T> a) {
    const int lane = threadIdx.x % G;
    const int64_t grp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    const int64_t ngrp = (int64_t)gridDim.x * blockDim.x / G;
    const T dl = a.dloss ? *a.dloss : T(1);
    for (int64_t i = grp; i < a.n; i += ngrp) {
        const int64_t rs = a.prp[i], re = a.prp[i + 1];
        T g0 = T(0), g1 = T(0), g2 = T(0);
        if (rs < re) {
            const T zi = a.invZ[i];
            T ax = T(0), ay = T(0), az = T(0), rx = T(0), ry = T(0), rz = T(0), dx, dy, dz;
            for (int64_t x = rs + lane; x < re; x += G) {
                const uint32_t e = a.colhop[x];
                const int32_t j = (int32_t)(e & COL_MASK);
                const T d2 = off3(a.y3, i, j, dx, dy, dz);
                const T p = obj_p(a, i, j, e >> 30, zi, x);
                const T k = p * (T(-2) * a.bv) * opow_bm1<B>(d2, a.half != 0) *
                            orcp(T(1) + opow_b<B>(d2, a.half != 0));
                ax += k * dx;
                ay += k * dy;
                az += k * dz;
            }
            for (int m = lane; m < a.M; m += G) {
                const int32_t v =
                    draw_node(neg_word(a.seed, a.iter, (int32_t)i, m), a.C, a.guide, a.gbits, a.S);
                if (v == (int32_t)i) continue;
                const T d2 = off3(a.y3, i, v, dx, dy, dz);
                if (d2 > T(0)) {
                    const T k = (T(2) * a.bv) * orcp(d2 * (T(1) + opow_b<B>(d2, a.half != 0)));
                    rx += k * dx;
                    ry += k * dy;
                    rz += k * dz;
                }
            }
            ax = group_sum<G>(ax);
            ay = group_sum<G>(ay);
            az = group_sum<G>(az);
            rx = group_sum<G>(rx);
            ry = group_sum<G>(ry);
            rz = group_sum<G>(rz);
            const T gq = a.gamma * a.qt[i];
            g0 = T(2) * ax + gq * rx;
            g1 = T(2) * ay + gq * ry;
            g2 = T(2) * az + gq * rz;
        }
        if (lane == 0) {
            a.dy3[3 * i] = dl * g0;
            a.dy3[3 * i + 1] = dl * g1;
            a.dy3[3 * i + 2] = dl * g2;
        }
    }
}

template <typename T, int B>
__global__ void k_other_side3(ObjArgs<T> a, const int32_t* __restrict__ seg,
                              const int32_t* __restrict__ pairs) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= a.n) return;
    const int32_t s = seg[v], e = seg[v + 1];
    if (s == e) return;
    const T dl = a.dloss ? *a.dloss : T(1);
    T g0 = T(0), g1 = T(0), g2 = T(0), dx, dy, dz;
    for (int32_t x = s; x < e; ++x) {
        const int32_t u = pairs[x] / a.M;
        const T d2 = off3(a.y3, v, u, dx, dy, dz);
        if (d2 > T(0)) {
            const T k = a.gamma * a.qt[u] * (T(2) * a.bv) /
                        (d2 * (T(1) + opow_b<B>(d2, a.half != 0)));
            g0 += k * dx;
            g1 += k * dy;
            g2 += k * dz;
        }
    }
    a.dy3[3 * v] += dl * g0;
    a.dy3[3 * v + 1] += dl * g1;
    a.dy3[3 * v + 2] += dl * g2;
}

__global__ void k_negatives(int32_t n, int32_t M, const int64_t* __restrict__ prp,
                            const uint64_t* __restrict__ C, const int32_t* __restrict__ guide,
                            int32_t gbits, uint64_t S, uint64_t seed, uint64_t iter,
                            int32_t* __restrict__ out) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (int64_t)n * M) return;
    const int32_t u = (int32_t)(p / M), m = (int32_t)(p % M);
    out[p] = (prp[u + 1] > prp[u] && S > 0)
                 ? draw_node(neg_word(seed, iter, u, m), C, guide, gbits, S)
                 : -1;
}

__global__ void k_coo(int32_t n, const int64_t* __restrict__ prp, const uint32_t* __restrict__ ch,
                      const float* __restrict__ invZf, float eh0, float eh1, float eh2, float eh3,
                      const double* __restrict__ A, const double* __restrict__ Ex,
                      int32_t* __restrict__ rows,
                      int32_t* __restrict__ cols, float* __restrict__ P) {
    const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const int lane = __lane_id();
    if (i >= n) return;
    for (int64_t x = prp[i] + lane; x < prp[i + 1]; x += WAVE) {
        const uint32_t e = ch[x];
        const int32_t j = (int32_t)(e & COL_MASK);
        const uint32_t h = e >> 30;
        const float eh = h == 0 ? eh0 : (h == 1 ? eh1 : (h == 2 ? eh2 : eh3));
        if (rows) rows[x] = (int32_t)i;
        if (cols) cols[x] = j;
        if (P) P[x] = A ? (float)((A[4 * i + h] + A[4 * (int64_t)j + h]) * 0.5)
                        : (Ex ? (float)(0.5 * Ex[x]) : eh) * (invZf[i] + invZf[j]);
    }
}

// ------------------------------------------------------------------ host
template <typename T>
static ObjArgs<T> obj_args(drg_sim* s, const drg_obj_params* p, const T* y) {
    ObjArgs<T> a{};
    a.n = s->n;
    a.M = s->S > 0 ? p->M : 0;
    a.prp = s->row_ptr.get();
    a.colhop = s->colhop.get();
    if constexpr (std::is_same<T, float>::value) {
        a.invZ = s->invZf.get();
        a.qt = s->qtf.get();
    } else {
        a.invZ = s->invZ.get();
        a.qt = s->qt.get();
    }
    a.y = reinterpret_cast<const typename OV<T>::v2*>(y);
    a.y3 = y;
    a.C = s->C.get();
    a.guide = s->guide.get();
    a.gbits = s->gbits;
    a.S = s->S;
    a.eh0 = (T)(0.5 * s->e[0]);
    a.eh1 = (T)(0.5 * s->e[1]);
    a.eh2 = (T)(0.5 * s->e[2]);
    a.eh3 = (T)(0.5 * s->e[3]);
    a.gamma = (T)p->gamma;
    a.half = p->b_half ? 1 : 0;
    a.A = s->A.get();
    a.Ex = s->Ex.get();
    a.bv = (T)((double)p->b + (p->b_half ? 0.5 : 0.0));
    a.seed = p->seed;
    a.iter = p->iter;
    return a;
}

static void check_obj(const drg_sim* s, const drg_obj_params* p, const void* y) {
    if (!s || !p || !y) throw Error(DRG_E_INVALID, "objective: NULL argument");
    if (p->M < 0) throw Error(DRG_E_INVALID, "objective: M >= 0");
    check_shape(p->b, p->b_half);
    if (p->dim != 0 && p->dim != 2 && p->dim != 3)
        throw Error(DRG_E_INVALID, "objective: dim must be 2 (or 0) or 3");
}

static int obj_group(const drg_sim* s) {
    const double mean = (double)s->nnz / (double)std::max(1, s->n_active);
    return mean <= 8 ? 8 : (mean <= 32 ? 32 : 64);
}

template <typename T, int B, int G>
static void launch_obj(hipStream_t st, const ObjArgs<T>& a, bool grad, bool three) {
    const int grid = (int)std::max<int64_t>(
        1, std::min<int64_t>(((int64_t)a.n * G + 255) / 256, (int64_t)1 << 22));
    if (three) {
        if (grad)
            hipLaunchKernelGGL((k_grad_rows3<T, B, G>), dim3(grid), dim3(256), 0, st, a);
        else
            hipLaunchKernelGGL((k_obj_rows3<T, B, G>), dim3(grid), dim3(256), 0, st, a);
    } else if (grad) {
        hipLaunchKernelGGL((k_grad_rows<T, B, G>), dim3(grid), dim3(256), 0, st, a);
    } else {
        hipLaunchKernelGGL((k_obj_rows<T, B, G>), dim3(grid), dim3(256), 0, st, a);
    }
    DRG_LAUNCH_CHECK();
}

template <typename T, int B>
static void launch_obj_g(hipStream_t st, const ObjArgs<T>& a, int G, bool grad, bool three) {
    if (G == 8) launch_obj<T, B, 8>(st, a, grad, three);
    else if (G == 32) launch_obj<T, B, 32>(st, a, grad, three);
    else launch_obj<T, B, 64>(st, a, grad, three);
}

static bool obj_blocked_wanted() {
    const char* v = std::getenv("DRG_OBJ_BLOCKED");
    return !(v && *v == '0');
}

// Attraction and own-side terms of every row: the blocked flat sweep when the
// similarity has the column-blocked copy (FP32, 2-D), else the row kernels.
template <typename T>
static void obj_rows(drg_ctx* ctx, drg_sim* s, const drg_obj_params* p, const ObjArgs<T>& a,
                     bool grad) {
    hipStream_t st = ctx->stream;
    const bool three = p->dim == 3;
    if constexpr (std::is_same<T, float>::value) {
        if (!three && !p->b_half && !a.A && !a.Ex && s->blk_nb > 0 && obj_blocked_wanted()) {
            sweep_blocked_objective(ctx, s, p->b, reinterpret_cast<const float*>(a.y), grad ? 1 : 0);
            const float2* part = s->blk_partial.get();
#define DRG_FIN(BB)                                                                          \
    case BB:                                                                                 \
        if (grad)                                                                            \
            hipLaunchKernelGGL((k_obj_finish<BB, 1>), dim3(ceil_div(s->n, 256)), dim3(256), 0, \
                               st, a, s->blk_nb, part);                                      \
        else                                                                                 \
            hipLaunchKernelGGL((k_obj_finish<BB, 0>), dim3(ceil_div(s->n, 256)), dim3(256), 0, \
                               st, a, s->blk_nb, part);                                      \
        break;
            switch (p->b) {
                DRG_FIN(1)
                DRG_FIN(2)
                default:
                DRG_FIN(3)
            }
#undef DRG_FIN
            DRG_LAUNCH_CHECK();
            return;
        }
    }
    const int G = obj_group(s);
    switch (p->b) {
        case 1: launch_obj_g<T, 1>(st, a, G, grad, three); break;
        case 2: launch_obj_g<T, 2>(st, a, G, grad, three); break;
        default: launch_obj_g<T, 3>(st, a, G, grad, three); break;
    }
}

template <typename T>
void objective_fwd_t(drg_ctx* ctx, drg_sim* s, const drg_obj_params* p, const T* y, T* loss,
                     T* rows) {
    check_obj(s, p, y);
    if (!loss && !rows) throw Error(DRG_E_INVALID, "objective: loss and rows are NULL");
    hipStream_t st = ctx->stream;
    DevBuf<T> rv;
    if (!rows) rv.alloc(s->n);
    ObjArgs<T> a = obj_args<T>(s, p, y);
    a.row_val = rows ? rows : rv.get();
    obj_rows<T>(ctx, s, p, a, false);
    if (!loss) {
        DRG_HIP(hipStreamSynchronize(st));
        return;
    }
    // fixed-order reduction to one value
    int64_t m = s->n;
    DevBuf<T> buf1((m + 1023) / 1024), buf2((m + 1023) / 1024);
    const T* src = a.row_val;
    T* dst = buf1.get();
    while (true) {
        const int64_t nb = (m + 1023) / 1024;
        hipLaunchKernelGGL(k_sum_blocks<T>, dim3((unsigned)nb), dim3(1024), 0, st, m, src,
                           nb == 1 ? loss : dst);
        DRG_LAUNCH_CHECK();
        if (nb == 1) break;
        src = dst;
        dst = (dst == buf1.get()) ? buf2.get() : buf1.get();
        m = nb;
    }
    DRG_HIP(hipStreamSynchronize(st));
}

template <typename T>
void objective_bwd_t(drg_ctx* ctx, drg_sim* s, const drg_obj_params* p, const T* y,
                     const T* dloss, T* dy) {
    check_obj(s, p, y);
    if (!dy) throw Error(DRG_E_INVALID, "objective: dy is NULL");
    hipStream_t st = ctx->stream;
    ObjArgs<T> a = obj_args<T>(s, p, y);
    a.dloss = dloss;
    a.dy = reinterpret_cast<typename OV<T>::v2*>(dy);
    a.dy3 = dy;
    const bool three = p->dim == 3;
    obj_rows<T>(ctx, s, p, a, true);
    if (a.M == 0) return;
    const int64_t np = (int64_t)s->n * a.M;
    if (np >= ((int64_t)1 << 31)) throw Error(DRG_E_UNSUPPORTED, "objective: n*M >= 2^31");
    DevBuf<uint32_t> keys(np);
    DevBuf<int32_t> pairs(np), seg((int64_t)s->n + 2);
    hipLaunchKernelGGL(k_neg_keys, dim3(ceil_div(np, 256)), dim3(256), 0, st, s->n, a.M,
                       s->row_ptr.get(), s->C.get(), s->guide.get(), s->gbits, s->S, p->seed,
                       p->iter, keys.get(), pairs.get());
    DRG_LAUNCH_CHECK();
    int bits = 1;
    while (bits < 32 && ((int64_t)1 << bits) <= s->n) ++bits;
    radix_sort_pairs(keys.get(), pairs.get(), np, bits, st);
    hipLaunchKernelGGL(k_key_bounds, dim3(ceil_div((int64_t)s->n + 1, 256)), dim3(256), 0, st, np,
                       s->n, keys.get(), seg.get());
    DRG_LAUNCH_CHECK();
    const dim3 og(ceil_div(s->n, 256));
    if (three) {
        switch (p->b) {
            case 1: hipLaunchKernelGGL((k_other_side3<T, 1>), og, dim3(256), 0, st, a, seg.get(), pairs.get()); break;
            case 2: hipLaunchKernelGGL((k_other_side3<T, 2>), og, dim3(256), 0, st, a, seg.get(), pairs.get()); break;
            default: hipLaunchKernelGGL((k_other_side3<T, 3>), og, dim3(256), 0, st, a, seg.get(), pairs.get()); break;
        }
    } else {
        switch (p->b) {
            case 1: hipLaunchKernelGGL((k_other_side<T, 1>), og, dim3(256), 0, st, a, seg.get(), pairs.get()); break;
            case 2: hipLaunchKernelGGL((k_other_side<T, 2>), og, dim3(256), 0, st, a, seg.get(), pairs.get()); break;
            default: hipLaunchKernelGGL((k_other_side<T, 3>), og, dim3(256), 0, st, a, seg.get(), pairs.get()); break;
        }
    }
    DRG_LAUNCH_CHECK();
    DRG_HIP(hipStreamSynchronize(st));
}

// ------------------------------------------------------------------ no-allocation forward
// The FP32 forward with its scratch (row values, then the block sums of the
// fixed-order reduction) in a file-scope device array instead of library
// allocations.  Host code reaches the array only through the address that
// hipGetSymbolAddress returns for the current device (kept per device):
// the array's own name is not a device address in host code.
constexpr int64_t OBJ_NA_SUMS = (OBJ_NOALLOC_MAX_N + 1023) / 1024;
static __device__ __align__(256) float scratch[OBJ_NOALLOC_MAX_N + 2 * OBJ_NA_SUMS];

static float* obj_scratch(int device) {
    constexpr int MAXDEV = 64;
    static std::mutex mu;
    static float* addr[MAXDEV] = {};
    if (device < 0 || device >= MAXDEV) throw Error(DRG_E_UNSUPPORTED, "objective: device id >= 64");
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        void* p = nullptr;
        const hipError_t rc = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (rc != hipSuccess || !p)
            throw Error(DRG_E_DEVICE, std::string("objective: hipGetSymbolAddress: ") +
                                          hipGetErrorString(rc));
        addr[device] = static_cast<float*>(p);
    }
    return addr[device];
}

void objective_fwd_noalloc(drg_ctx* ctx, drg_sim* s, const drg_obj_params* p, const float* y,
                           float* loss) {
    check_obj(s, p, y);
    if (!loss) throw Error(DRG_E_INVALID, "objective: loss is NULL");
    if ((int64_t)s->n > OBJ_NOALLOC_MAX_N)
        throw Error(DRG_E_INVALID, "objective (no allocation): n = " + std::to_string(s->n) +
                                       " exceeds the static scratch of " +
                                       std::to_string(OBJ_NOALLOC_MAX_N) + " nodes");
    float* base = obj_scratch(ctx->device);  // ctx->device is current
    hipStream_t st = ctx->stream;
    ObjArgs<float> a = obj_args<float>(s, p, y);
    a.row_val = base;  // every row is written, isolated rows with 0
    obj_rows<float>(ctx, s, p, a, false);
    // the same fixed-order reduction as objective_fwd_t, ping-ponging
    // between the two block-sum areas after the row values
    float* buf1 = base + OBJ_NOALLOC_MAX_N;
    float* buf2 = buf1 + OBJ_NA_SUMS;
    int64_t m = s->n;
    const float* src = a.row_val;
    float* dst = buf1;
    while (true) {
        const int64_t nb = (m + 1023) / 1024;
        hipLaunchKernelGGL(k_sum_blocks<float>, dim3((unsigned)nb), dim3(1024), 0, st, m, src,
                           nb == 1 ? loss : dst);
        DRG_LAUNCH_CHECK();
        if (nb == 1) break;
        src = dst;
        dst = (dst == buf1) ? buf2 : buf1;
        m = nb;
    }
}

template void objective_fwd_t<float>(drg_ctx*, drg_sim*, const drg_obj_params*, const float*, float*, float*);
template void objective_fwd_t<double>(drg_ctx*, drg_sim*, const drg_obj_params*, const double*, double*, double*);
template void objective_bwd_t<float>(drg_ctx*, drg_sim*, const drg_obj_params*, const float*, const float*, float*);
template void objective_bwd_t<double>(drg_ctx*, drg_sim*, const drg_obj_params*, const double*, const double*, double*);

void sample_negatives(drg_ctx* ctx, drg_sim* s, int32_t M, uint64_t seed, uint64_t iter,
                      int32_t* out) {
    if (!s || !out || M < 0) throw Error(DRG_E_INVALID, "sample_negatives: bad argument");
    const int64_t np = (int64_t)s->n * M;
    if (np == 0) return;
    hipLaunchKernelGGL(k_negatives, dim3(ceil_div(np, 256)), dim3(256), 0, ctx->stream, s->n, M,
                       s->row_ptr.get(), s->C.get(), s->guide.get(), s->gbits, s->S, seed, iter,
                       out);
    DRG_LAUNCH_CHECK();
}

void sim_coo(drg_ctx* ctx, drg_sim* s, int32_t* rows, int32_t* cols, float* P) {
    if (!s) throw Error(DRG_E_INVALID, "sim_coo: sim is NULL");
    hipLaunchKernelGGL(k_coo, dim3(ceil_div((int64_t)s->n * WAVE, 256)), dim3(256), 0, ctx->stream,
                       s->n, s->row_ptr.get(), s->colhop.get(), s->invZf.get(),
                       (float)(0.5 * s->e[0]), (float)(0.5 * s->e[1]), (float)(0.5 * s->e[2]),
                       (float)(0.5 * s->e[3]), s->A.get(), s->Ex.get(), rows, cols, P);
    DRG_LAUNCH_CHECK();
}

}  // namespace drg
