// evaluate.hip -- layout quality on the GPU: neighbourhood preservation NP
// (Sec. 4.1, Eq. NP) of chosen nodes.
//
// For node v with graph neighbourhood N_G(v) = NNG(v, k) (the rows of a
// similarity built with k = k_eval) and m = |N_G(v)| > 0, the layout
// neighbourhood N_L(v) is the set of the m nodes u != v nearest to y_v, ties
// in distance broken by the smaller id; NP_v = |N_G & N_L| / |N_G | N_L|.
//
// One workgroup per node selects the m-th smallest key (d^2, id) over all
// nodes exactly: d^2 = dx*dx + dy*dy in FP64 from the FP32 coordinates (no
// contraction, so every node's key is the same number on any machine), the
// key ordered as (bits of d^2, id) and found digit by digit (radix select:
// eight 8-bit digits of d^2, then the id); then every entry of the row is
// tested against that key.  Exact, so it matches a plain sort of all
// distances.
#include <algorithm>

#include <vector>

#include "drg_internal.hpp"

namespace drg {

constexpr int NP_BLOCK = 1024;

__device__ __forceinline__ uint64_t np_key(const float2* __restrict__ y, double vx, double vy,
                                           int32_t j) {
#pragma clang fp contract(off)
    const float2 p = y[j];
    const double dx = vx - (double)p.x;
    const double dy = vy - (double)p.y;
    const double a = dx * dx;
    const double b = dy * dy;
    const double d2 = a + b;
    return (uint64_t)__double_as_longlong(d2);  // d2 >= 0: bit order = value order
}

// hist[dg] += 1 for the calling lanes, one LDS atomic per distinct digit of
// the wave (distances cluster, so most lanes of a wave share a digit)
__device__ __forceinline__ void hist_add(int32_t* hist, uint32_t dg) {
    // each round serves the digit of the first lane still waiting, so every
    // round retires at least that lane
    while (true) {
        const uint32_t lead = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)dg);
        const uint64_t same = __ballot(dg == lead);
        if (dg == lead) {
            if (__lane_id() == (uint32_t)(__ffsll((unsigned long long)same) - 1))
                atomicAdd(&hist[lead], __popcll(same));
            break;
        }
    }
}

__global__ void k_check_ids(int32_t count, const int32_t* __restrict__ ids, int32_t n,
                            int* __restrict__ bad) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count && (ids[t] < 0 || ids[t] >= n)) atomicOr(bad, 1);
}

// Block-wide: the digit (0..255) at which the running count over hist
// reaches `need` (1-based rank), and the count of smaller digits.
__device__ __forceinline__ void np_pick(const int32_t* hist, int64_t need, int32_t* s_pick,
                                        int64_t* s_below) {
    if (threadIdx.x == 0) {
        int64_t acc = 0;
        int d = 0;
        for (; d < 255; ++d) {
            if (acc + hist[d] >= need) break;
            acc += hist[d];
        }
        *s_pick = d;
        *s_below = acc;
    }
    __syncthreads();
}

__global__ __launch_bounds__(NP_BLOCK) void k_np(int32_t n, const int64_t* __restrict__ prp,
                                                 const uint32_t* __restrict__ colhop,
                                                 const float2* __restrict__ y,
                                                 const int32_t* __restrict__ nodes,
                                                 double* __restrict__ out) {
    __shared__ int32_t s_hist[256];
    __shared__ int32_t s_pick;
    __shared__ int64_t s_below;
    __shared__ unsigned long long s_inter;
    const int32_t v = nodes[blockIdx.x];
    const int64_t rs = prp[v], re = prp[v + 1];
    const int64_t m = re - rs;
    if (m == 0) {  // no graph neighbourhood: no value
        if (threadIdx.x == 0) out[blockIdx.x] = -1.0;
        return;
    }
    const float2 pv = y[v];
    const double vx = pv.x, vy = pv.y;
    // key (hi, lo) = (d2 bits, id); the node itself never counts
    uint64_t hi_pre = 0, hi_mask = 0;
    uint32_t lo_pre = 0, lo_mask = 0;
    int64_t need = m;  // rank still to place inside the current prefix
    for (int pass = 0; pass < 11; ++pass) {
        // passes 0..7: bytes of d2 from the top; 8..10: id bits 23..16, 15..8, 7..0
        const bool on_hi = pass < 8;
        const int shift = on_hi ? 56 - 8 * pass : 16 - 8 * (pass - 8);
        for (int t = threadIdx.x; t < 256; t += NP_BLOCK) s_hist[t] = 0;
        __syncthreads();
        for (int32_t j = threadIdx.x; j < n; j += NP_BLOCK) {
            if (j == v) continue;
            const uint64_t kh = np_key(y, vx, vy, j);
            if ((kh & hi_mask) != hi_pre) continue;
            const uint32_t kl = (uint32_t)j;
            if ((kl & lo_mask) != lo_pre) continue;
            const uint32_t dg = on_hi ? (uint32_t)(kh >> shift) & 255u : (kl >> shift) & 255u;
            hist_add(s_hist, dg);
        }
        __syncthreads();
        np_pick(s_hist, need, &s_pick, &s_below);
        const uint32_t d = (uint32_t)s_pick;
        need -= s_below;
        if (on_hi) {
            hi_pre |= (uint64_t)d << shift;
            hi_mask |= (uint64_t)255 << shift;
        } else {
            lo_pre |= d << shift;
            lo_mask |= 255u << shift;
        }
        __syncthreads();  // s_pick / s_below read by all before the next pass
    }
    // (hi_pre, lo_pre) is the m-th smallest key; N_L(v) = keys <= it
    if (threadIdx.x == 0) s_inter = 0;
    __syncthreads();
    unsigned long long cnt = 0;
    for (int64_t x = rs + threadIdx.x; x < re; x += NP_BLOCK) {
        const int32_t j = (int32_t)(colhop[x] & COL_MASK);
        const uint64_t kh = np_key(y, vx, vy, j);
        const bool in = kh < hi_pre || (kh == hi_pre && (uint32_t)j <= lo_pre);
        cnt += in ? 1u : 0u;
    }
    cnt = group_sum<WAVE>(cnt);
    if (__lane_id() == 0 && cnt) atomicAdd(&s_inter, cnt);
    __syncthreads();
    if (threadIdx.x == 0) {
        const double inter = (double)s_inter;
        out[blockIdx.x] = inter / (2.0 * (double)m - inter);
    }
}

void neighbourhood_preservation(drg_ctx* ctx, const drg_sim* s, const float* y, int32_t count,
                                const int32_t* nodes, double* out) {
    if (count < 0) throw Error(DRG_E_INVALID, "count >= 0");
    if (count == 0) return;
    if (!y || !nodes || !out) throw Error(DRG_E_INVALID, "y, nodes and out are required");
    if (s->n >= (1 << 24)) throw Error(DRG_E_UNSUPPORTED, "NP: n < 2^24");
    // the node ids are checked on the device before any kernel reads them
    DevBuf<int> bad(1);
    DRG_HIP(hipMemsetAsync(bad.get(), 0, sizeof(int), ctx->stream));
    hipLaunchKernelGGL(k_check_ids, dim3(ceil_div(count, 256)), dim3(256), 0, ctx->stream, count,
                       nodes, s->n, bad.get());
    DRG_LAUNCH_CHECK();
    int h = 0;
    DRG_HIP(hipMemcpyAsync(&h, bad.get(), sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    DRG_HIP(hipStreamSynchronize(ctx->stream));
    if (h) throw Error(DRG_E_INVALID, "node id out of range");
    hipLaunchKernelGGL(k_np, dim3(count), dim3(NP_BLOCK), 0, ctx->stream, s->n, s->row_ptr.get(),
                       s->colhop.get(), reinterpret_cast<const float2*>(y), nodes, out);
    DRG_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ stress
// Normalised stress (Sec. 4.1) needs shortest-path distances D_sj; with the
// optimal scale alpha it is (P - A^2 / B) / |V|^2 over the pairs summed, where
// A = sum L/D, B = sum L^2/D^2, P = number of pairs (L = layout distance,
// weight 1/D^2).  A sampled estimate takes the pairs (s, j) of chosen
// sources s with all nodes j reachable from them.  One workgroup per source:
// breadth-first search over the whole graph (visited set as a bitmap, LDS or
// global), the distance of every node recorded, then the sums in ascending
// node id (fixed order: repeatable).

constexpr int ST_BLOCK = 1024;

struct StressArgs {
    int32_t n, nwords;
    const int32_t* rp;
    const int32_t* col;
    const float2* y;
    const int32_t* src;
    int32_t* dist;     // [grid][n], zero on entry, left zero
    int32_t* queue;    // [grid][n]
    uint32_t* gbm;     // [grid][nwords] when the bitmap is not in LDS
    double* out;       // [count][3]: A, B, P
};

template <bool LDS_BM>
__global__ __launch_bounds__(ST_BLOCK) void k_stress(StressArgs a) {
#pragma clang fp contract(off)
    extern __shared__ uint32_t s_bm[];
    __shared__ int32_t s_tail;
    __shared__ double s_red[3][ST_BLOCK / WAVE];
    uint32_t* bm = LDS_BM ? s_bm : a.gbm + (size_t)blockIdx.x * (size_t)a.nwords;
    int32_t* dist = a.dist + (size_t)blockIdx.x * (size_t)a.n;
    int32_t* q = a.queue + (size_t)blockIdx.x * (size_t)a.n;
    const int tid = threadIdx.x;
    const int32_t s = a.src[blockIdx.x];
    for (int w = tid; w < a.nwords; w += ST_BLOCK) bm[w] = 0;
    if (tid == 0) {
        q[0] = s;
        s_tail = 1;
    }
    __syncthreads();
    if (tid == 0) atomicOr(&bm[s >> 5], 1u << (s & 31));
    __syncthreads();
    // level by level: frontier q[fb..fe) at distance d, G = 64 lanes per node
    int32_t fb = 0, fe = 1;
    for (int32_t d = 1; fb < fe; ++d) {
        for (int32_t fi = fb + tid / WAVE; fi < fe; fi += ST_BLOCK / WAVE) {
            const int32_t u = q[fi];
            for (int32_t x = a.rp[u] + __lane_id(); x < a.rp[u + 1]; x += WAVE) {
                const int32_t v = a.col[x];
                const uint32_t bit = 1u << (v & 31);
                const uint32_t old = atomicOr(&bm[v >> 5], bit);
                const bool fresh = !(old & bit);
                if (fresh) dist[v] = d;
                const uint64_t act = __ballot(1);
                const uint64_t fm = __ballot(fresh);
                if (fm) {
                    const int leader = __ffsll((unsigned long long)act) - 1;
                    int qpos = 0;
                    if (__lane_id() == leader) qpos = atomicAdd(&s_tail, __popcll(fm));
                    qpos = __shfl(qpos, leader);
                    if (fresh) q[qpos + __popcll(fm & lanemask_lt())] = v;
                }
            }
        }
        __syncthreads();
        fb = fe;
        fe = s_tail;
        __syncthreads();
    }
    // the sums, in ascending node id per thread, then a fixed tree
    const float2 ps = a.y[s];
    const double sx = ps.x, sy = ps.y;
    double A = 0.0, B = 0.0, P = 0.0;
    for (int32_t j = tid; j < a.n; j += ST_BLOCK) {
        const int32_t dj = dist[j];
        if (dj > 0) {
            dist[j] = 0;
            const float2 p = a.y[j];
            const double dx = sx - (double)p.x;
            const double dy = sy - (double)p.y;
            const double e = dx * dx;
            const double f = dy * dy;
            const double L = sqrt(e + f);
            const double D = (double)dj;
            const double r = L / D;
            A = A + r;
            B = B + r * r;
            P = P + 1.0;
        }
    }
    A = group_sum<WAVE>(A);
    B = group_sum<WAVE>(B);
    P = group_sum<WAVE>(P);
    if (__lane_id() == 0) {
        s_red[0][tid / WAVE] = A;
        s_red[1][tid / WAVE] = B;
        s_red[2][tid / WAVE] = P;
    }
    __syncthreads();
    if (tid < 3) {
        double t = 0.0;
        for (int w = 0; w < ST_BLOCK / WAVE; ++w) t = t + s_red[tid][w];
        a.out[(size_t)blockIdx.x * 3 + tid] = t;
    }
}

void stress_sampled(drg_ctx* ctx, const drg_csr* g, const float* y, int32_t count,
                    const int32_t* sources, double* out, double* estimate) {
    if (count < 0) throw Error(DRG_E_INVALID, "count >= 0");
    if (estimate) *estimate = 0.0;
    if (count == 0) return;
    if (!y || !sources || !out) throw Error(DRG_E_INVALID, "y, sources and out are required");
    validate_csr_impl(ctx, g, false);
    hipStream_t st = ctx->stream;
    const int32_t n = g->n;
    DevBuf<int> bad(1);
    DRG_HIP(hipMemsetAsync(bad.get(), 0, sizeof(int), st));
    hipLaunchKernelGGL(k_check_ids, dim3(ceil_div(count, 256)), dim3(256), 0, st, count, sources,
                       n, bad.get());
    DRG_LAUNCH_CHECK();
    int h = 0;
    DRG_HIP(hipMemcpyAsync(&h, bad.get(), sizeof(int), hipMemcpyDeviceToHost, st));
    DRG_HIP(hipStreamSynchronize(st));
    if (h) throw Error(DRG_E_INVALID, "source id out of range");
    const int nwords = (n + 31) / 32;
    const size_t lds = (size_t)nwords * 4;
    const bool in_lds = lds + 4096 <= (size_t)ctx->max_lds;
    // sources in rounds of at most `per` workgroups (scratch: distances and
    // queue of n ints each per workgroup)
    const int32_t per = std::max<int32_t>(1, std::min<int32_t>(ctx->num_cu, count));
    DevBuf<int32_t> dist((int64_t)per * n);
    DevBuf<int32_t> queue((int64_t)per * n);
    DevBuf<uint32_t> gbm;
    if (!in_lds) gbm.alloc((int64_t)per * nwords);
    DRG_HIP(hipMemsetAsync(dist.get(), 0, sizeof(int32_t) * (size_t)per * n, st));
    for (int32_t c0 = 0; c0 < count; c0 += per) {
        const int32_t m = std::min(per, count - c0);
        StressArgs a{};
        a.n = n;
        a.nwords = nwords;
        a.rp = g->row_ptr;
        a.col = g->col;
        a.y = reinterpret_cast<const float2*>(y);
        a.src = sources + c0;
        a.dist = dist.get();
        a.queue = queue.get();
        a.gbm = gbm.get();
        a.out = out + (size_t)c0 * 3;
        if (in_lds) {
            DRG_HIP(hipFuncSetAttribute((const void*)k_stress<true>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            hipLaunchKernelGGL(k_stress<true>, dim3(m), dim3(ST_BLOCK), lds, st, a);
        } else {
            hipLaunchKernelGGL(k_stress<false>, dim3(m), dim3(ST_BLOCK), 0, st, a);
        }
        DRG_LAUNCH_CHECK();
    }
    if (estimate) {
        // (n / count) (sum P - (sum A)^2 / sum B) / n^2, the sums taken over
        // the sources in the order given
        std::vector<double> h((size_t)count * 3);
        DRG_HIP(hipMemcpyAsync(h.data(), out, sizeof(double) * h.size(), hipMemcpyDeviceToHost,
                               st));
        DRG_HIP(hipStreamSynchronize(st));
        double A = 0.0, B = 0.0, P = 0.0;
        for (int32_t t = 0; t < count; ++t) {
            A += h[3 * (size_t)t];
            B += h[3 * (size_t)t + 1];
            P += h[3 * (size_t)t + 2];
        }
        const double nn = (double)n;
        *estimate = B > 0.0 ? (nn / (double)count) * (P - A * A / B) / (nn * nn) : 0.0;
    }
    DRG_HIP(hipStreamSynchronize(st));
}

}  // namespace drg
