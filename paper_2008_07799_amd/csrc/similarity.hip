// similarity.hip -- sparse distance matrix and node similarity (Sec. 3.2.1,
// Eq. NS) plus the node-weight sampling table of the negatives (Sec. 3.2.2).
//
// Pattern: for every source s the set NNG(s, k) with hop counts, by a
// breadth-first search bounded at depth k.  One workgroup owns one source at
// a time (sources are handed out through an atomic counter).  The visited set
// is a bitmap over all n nodes held in LDS (global memory when n is too large),
// so a row comes out sorted by scanning the bitmap: each thread popcounts a
// few bitmap words and a block prefix sum places the set bits.  Frontier
// levels 2..k-1 are kept in a per-workgroup queue filled with wave-ballot
// compaction; hop counts < k are patched into the sorted row afterwards.
// Two passes: count (hop histogram per row) -> prefix sum -> fill.
#include <cmath>
#include <memory>
#include <vector>

#include "drg_bitmap.hpp"
#include "drg_internal.hpp"

namespace drg {

// ------------------------------------------------------------------ checks
__global__ void k_check_rowptr(int32_t n, int32_t nnz, const int32_t* __restrict__ rp,
                               int* __restrict__ bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    const int32_t v = rp[i];
    bool ok = v >= 0 && v <= nnz;
    if (i == 0) ok = ok && v == 0;
    if (i == n) ok = ok && v == nnz;
    if (i < n) ok = ok && rp[i + 1] >= v;
    if (!ok) atomicOr(bad, 1);
}

__global__ void k_check_cols(int32_t nnz, int32_t n, const int32_t* __restrict__ col,
                             int* __restrict__ bad) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x < nnz && (col[x] < 0 || col[x] >= n)) atomicOr(bad, 2);
}

// rows sorted strictly ascending (no duplicates), no self-loops, symmetric
__global__ void k_check_structure(int32_t n, const int32_t* __restrict__ rp,
                                  const int32_t* __restrict__ col, int* __restrict__ bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t s = rp[i], e = rp[i + 1];
    int flag = 0;
    for (int32_t x = s; x < e; ++x) {
        const int32_t v = col[x];
        if (v == (int32_t)i) flag |= 4;
        if (x > s && col[x - 1] >= v) flag |= 8;
        int32_t lo = rp[v], hi = rp[v + 1];
        while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            if (col[mid] < (int32_t)i)
                lo = mid + 1;
            else
                hi = mid;
        }
        if (lo >= rp[v + 1] || col[lo] != (int32_t)i) flag |= 16;
    }
    if (flag) atomicOr(bad, flag);
}

static int read_flag(DevBuf<int>& f, hipStream_t s) {
    int h = 0;
    DRG_HIP(hipMemcpyAsync(&h, f.get(), sizeof(int), hipMemcpyDeviceToHost, s));
    DRG_HIP(hipStreamSynchronize(s));
    return h;
}

// Cheap bounds checks always run (they keep later kernels inside their
// buffers); the structural checks run under DRG_VALIDATE.
void validate_csr_impl(drg_ctx* ctx, const drg_csr* g, bool full) {
    hipStream_t st = ctx->stream;
    DevBuf<int> bad(1);
    DRG_HIP(hipMemsetAsync(bad.get(), 0, sizeof(int), st));
    hipLaunchKernelGGL(k_check_rowptr, dim3(ceil_div((int64_t)g->n + 1, 256)), dim3(256), 0, st,
                       g->n, g->nnz, g->row_ptr, bad.get());
    DRG_LAUNCH_CHECK();
    if (read_flag(bad, st)) throw Error(DRG_E_GRAPH, "row_ptr is not a valid offset array");
    if (g->nnz > 0) {
        hipLaunchKernelGGL(k_check_cols, dim3(ceil_div(g->nnz, 256)), dim3(256), 0, st, g->nnz,
                           g->n, g->col, bad.get());
        DRG_LAUNCH_CHECK();
        if (read_flag(bad, st)) throw Error(DRG_E_GRAPH, "column index out of range");
    }
    if (full && g->nnz > 0) {
        hipLaunchKernelGGL(k_check_structure, dim3(ceil_div(g->n, 256)), dim3(256), 0, st, g->n,
                           g->row_ptr, g->col, bad.get());
        DRG_LAUNCH_CHECK();
        const int f = read_flag(bad, st);
        if (f & 4) throw Error(DRG_E_GRAPH, "self-loop in input graph");
        if (f & 8) throw Error(DRG_E_GRAPH, "row not sorted or duplicate edge");
        if (f & 16) throw Error(DRG_E_GRAPH, "input graph is not symmetric");
    }
}

void validate_csr(drg_ctx* ctx, const drg_csr* g) { validate_csr_impl(ctx, g, true); }

// ------------------------------------------------------------------ BFS
constexpr int BFS_BLOCK = 256;
constexpr int EMIT_WPT = 8;

struct BfsArgs {
    int32_t n, k, nwords;
    const int32_t* rp;
    const int32_t* col;
    int32_t* cnt;          // count pass: [n][k] nodes per hop
    const int64_t* prp;    // fill pass: row offsets
    uint32_t* colhop;      // fill pass: entries
    int32_t* queue;        // [grid][qcap] frontier levels 2..k-1
    int64_t qcap;
    uint32_t* gbm;         // [grid][nwords] bitmaps when not in LDS
    int32_t* work;         // next source
    const int32_t* node_base;  // per node: first id of its graph in a batch (NULL: 0)
};

// Sets the hop of id v inside the sorted row ch[lo..hi); v absent (only
// possible for a self-loop in an unvalidated graph) writes nothing.
__device__ __forceinline__ void set_hop(uint32_t* __restrict__ ch, int64_t lo, int64_t hi,
                                        int32_t v, uint32_t hopbits) {
    const int64_t end = hi;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int32_t)(ch[mid] & COL_MASK) < v)
            lo = mid + 1;
        else
            hi = mid;
    }
    if (lo < end && (int32_t)(ch[lo] & COL_MASK) == v) ch[lo] = (uint32_t)v | hopbits;
}

template <bool FILL, bool LDS_BM, int G>
__global__ __launch_bounds__(BFS_BLOCK) void k_khop(BfsArgs a) {
    extern __shared__ uint32_t s_bm[];
    __shared__ int32_t s_src, s_qtail;
    __shared__ int32_t s_lvl[8];
    __shared__ int32_t s_red[BFS_BLOCK / WAVE];
    uint32_t* bm = LDS_BM ? s_bm : a.gbm + (size_t)blockIdx.x * (size_t)a.nwords;
    int32_t* q = a.queue ? a.queue + (size_t)blockIdx.x * (size_t)a.qcap : nullptr;
    const int tid = threadIdx.x;
    for (int w = tid; w < a.nwords; w += BFS_BLOCK) bm[w] = 0;
    __syncthreads();
    for (;;) {
        if (tid == 0) s_src = atomicAdd(a.work, 1);
        __syncthreads();
        const int32_t s = s_src;
        if (s >= a.n) break;
        // bitmap bit of node v is v - base: a source only reaches its own graph
        const int32_t base = a.node_base ? a.node_base[s] : 0;
        const int32_t rs = a.rp[s], re = a.rp[s + 1];
        if (rs == re) {
            if (!FILL && tid < a.k) a.cnt[(int64_t)s * a.k + tid] = 0;
            __syncthreads();
            continue;
        }
        // hop 1: the source itself (visited) and its neighbours
        if (tid == 0) {
            const int32_t sb = s - base;
            atomicOr(&bm[sb >> 5], 1u << (sb & 31));
            s_qtail = 0;
        }
        for (int32_t x = rs + tid; x < re; x += BFS_BLOCK) {
            const int32_t vb = a.col[x] - base;
            atomicOr(&bm[vb >> 5], 1u << (vb & 31));
        }
        __syncthreads();
        // hops 2..k: expand the previous frontier, G lanes per frontier node
        int32_t fb = 0, fe = 0;
        for (int d = 2; d <= a.k; ++d) {
            const bool from_adj = (d == 2);
            const int32_t* F = from_adj ? a.col + rs : q + fb;
            const int32_t flen = from_adj ? (re - rs) : (fe - fb);
            const bool keep = d < a.k;
            // the next frontier node's adjacency range is requested while
            // the current one is expanded
            int32_t fi = tid / G;
            int32_t us_n = 0, ue_n = 0;
            if (fi < flen) {
                const int32_t u = F[fi];
                us_n = a.rp[u];
                ue_n = a.rp[u + 1];
            }
            for (; fi < flen; fi += BFS_BLOCK / G) {
                const int32_t us = us_n, ue = ue_n;
                const int32_t fn = fi + BFS_BLOCK / G;
                if (fn < flen) {
                    const int32_t un = F[fn];
                    us_n = a.rp[un];
                    ue_n = a.rp[un + 1];
                }
                int32_t x = us + (tid % G);
                if (!keep) {
                    // last hop: only marks; four neighbour ids requested
                    // before their bits are set
                    for (; x + 3 * G < ue; x += 4 * G) {
                        int32_t w[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q) w[q] = a.col[x + q * G] - base;
#pragma unroll
                        for (int q = 0; q < 4; ++q) atomicOr(&bm[w[q] >> 5], 1u << (w[q] & 31));
                    }
                }
                for (; x < ue; x += G) {
                    const int32_t v = a.col[x];
                    const int32_t vb = v - base;
                    const uint32_t bit = 1u << (vb & 31);
                    if (keep) {
                        const uint32_t old = atomicOr(&bm[vb >> 5], bit);
                        const bool fresh = !(old & bit);
                        const uint64_t act = __ballot(1);
                        const uint64_t fm = __ballot(fresh);
                        if (fm) {
                            const int leader = __ffsll((unsigned long long)act) - 1;
                            int qpos = 0;
                            if (__lane_id() == leader) qpos = atomicAdd(&s_qtail, __popcll(fm));
                            qpos = __shfl(qpos, leader);
                            if (fresh) q[qpos + __popcll(fm & lanemask_lt())] = v;
                        }
                    } else {
                        atomicOr(&bm[vb >> 5], bit);
                    }
                }
            }
            __syncthreads();
            if (keep) {
                fb = fe;
                fe = s_qtail;
                if (tid == 0) s_lvl[d] = fe;
            }
        }
        if constexpr (!FILL) {
            const int total = bitmap_count_clear<BFS_BLOCK>(bm, a.nwords, s_red);  // with source
            if (tid == 0) {
                const int64_t o = (int64_t)s * a.k;
                int acc = re - rs;
                a.cnt[o] = re - rs;
                int prev = 0;
                for (int d = 2; d < a.k; ++d) {
                    const int cd = s_lvl[d] - prev;
                    a.cnt[o + d - 1] = cd;
                    acc += cd;
                    prev = s_lvl[d];
                }
                if (a.k >= 2) a.cnt[o + a.k - 1] = (total - 1) - acc;
            }
            __syncthreads();
        } else {
            const int64_t row0 = a.prp[s], row1 = a.prp[s + 1];
            const uint32_t hopk = (uint32_t)(a.k - 1) << 30;
            uint32_t* out = a.colhop;
            bitmap_emit_clear<BFS_BLOCK, EMIT_WPT>(
                bm, a.nwords, s - base, row0, s_red,
                [&](int64_t o, uint32_t v) { out[o] = ((uint32_t)base + v) | hopk; });
            __syncthreads();
            if (a.k >= 2) {
                for (int32_t x = rs + tid; x < re; x += BFS_BLOCK)
                    set_hop(a.colhop, row0, row1, a.col[x], 0u);
                int prev = 0;
                for (int d = 2; d < a.k; ++d) {
                    const int end = s_lvl[d];
                    for (int t = prev + tid; t < end; t += BFS_BLOCK)
                        set_hop(a.colhop, row0, row1, q[t], (uint32_t)(d - 1) << 30);
                    prev = end;
                }
            }
            __syncthreads();
        }
    }
}

template <bool FILL, bool LDS_BM>
static void launch_khop(drg_ctx* ctx, const BfsArgs& a, int G, int grid, size_t lds) {
    hipStream_t st = ctx->stream;
#define DRG_KHOP_CASE(GG)                                                                       \
    case GG: {                                                                                  \
        auto fn = k_khop<FILL, LDS_BM, GG>;                                                     \
        if (LDS_BM)                                                                             \
            DRG_HIP(hipFuncSetAttribute((const void*)fn,                                        \
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)); \
        hipLaunchKernelGGL(fn, dim3(grid), dim3(BFS_BLOCK), LDS_BM ? lds : 0, st, a);           \
        break;                                                                                  \
    }
    switch (G) {
        DRG_KHOP_CASE(4)
        DRG_KHOP_CASE(8)
        DRG_KHOP_CASE(16)
        DRG_KHOP_CASE(32)
        default:
        DRG_KHOP_CASE(64)
    }
#undef DRG_KHOP_CASE
    DRG_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ helpers
__global__ void k_deg_counts(int32_t n, const int32_t* __restrict__ rp, int32_t* __restrict__ cnt,
                             int64_t* __restrict__ prp) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) cnt[i] = rp[i + 1] - rp[i];
    if (i <= n) prp[i] = rp[i];
}

__global__ void k_copy_cols(int32_t nnz, const int32_t* __restrict__ col, uint32_t* __restrict__ ch) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x < nnz) ch[x] = (uint32_t)col[x];  // hop 1 -> high bits 0
}

__global__ void k_row_len(int32_t n, int32_t k, const int32_t* __restrict__ cnt,
                          int64_t* __restrict__ len) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t s = 0;
    for (int d = 0; d < k; ++d) s += cnt[i * k + d];
    len[i] = s;
}

__global__ void k_sum_deg2(int32_t n, const int32_t* __restrict__ rp,
                           unsigned long long* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long v = 0;
    if (i < n) {
        const unsigned long long d = (unsigned long long)(rp[i + 1] - rp[i]);
        v = d * d;
    }
    v = group_sum<WAVE>(v);
    if (__lane_id() == 0 && v) atomicAdd(out, v);
}

__device__ __forceinline__ double pick_e(const double* e, uint32_t h) {
    return h == 0 ? e[0] : (h == 1 ? e[1] : (h == 2 ? e[2] : e[3]));
}

struct ECoef {
    double e[4];
};

// Z_i = sum_d cnt_i(d) e_d accumulated from zero in hop order, every
// operation rounded on its own; invZ_i = 1 / Z_i (0 for an isolated node).
__global__ void k_normalise(int32_t n, int32_t k, const int32_t* __restrict__ cnt, ECoef ec,
                            double* __restrict__ invZ, float* __restrict__ invZf,
                            float* __restrict__ invZlo) {
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double z = 0.0;
    for (int d = 0; d < k; ++d) {
        const double c = (double)cnt[i * k + d];
        const double t = c * pick_e(ec.e, (uint32_t)d);
        z = z + t;
    }
    const double iz = z > 0.0 ? 1.0 / z : 0.0;
    invZ[i] = iz;
    const float hi = (float)iz;
    invZf[i] = hi;
    invZlo[i] = (float)(iz - (double)hi);  // exact difference, rounded once
}

// ------------------------------------------------------------------ node-wise sigma
// sigma_i chosen per node so that NS_{.|i} over NNG(i, k) has a given
// perplexity exp(H) (t-SNE's calibration; Eq. NS gives each node its own
// Gaussian).  With t = exp(-1/(2 sigma_i^2)) the Gaussian of hop d is
// t^(d^2), so the distribution depends on t and the node's hop histogram
// only.  Every step is an IEEE-754 operation (frexp, +, -, *, /, compare)
// with contraction off, so any program that performs the same operations in
// the same order obtains the same t bit for bit, and with it the same P~
// and the same integer sampling table.

// ln x for x > 0 finite: x = m 2^e with m in [sqrt(1/2), sqrt(2)); ln m =
// 2 atanh(s), s = (m - 1)/(m + 1), |s| < 0.172, from the odd series of
// atanh by Horner's rule over 13 terms; ln x = e ln 2 + ln m.
__device__ double ln_ieee(double x) {
#pragma clang fp contract(off)
    int ex = 0;
    double m = frexp(x, &ex);  // exact; m in [1/2, 1)
    if (m < 0.70710678118654752440) {
        m = m * 2.0;
        ex = ex - 1;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double s2 = s * s;
    double p = 1.0 / 25.0;
    for (int j = 11; j >= 0; --j) p = p * s2 + 1.0 / (double)(2 * j + 1);
    const double lm = 2.0 * s * p;
    return (double)ex * 0.69314718055994530942 + lm;
}

// t^(d^2) for d = 1..k, each a running product of d^2 factors
__device__ __forceinline__ void gauss_of_t(double t, int k, double* e) {
#pragma clang fp contract(off)
    for (int d = 1; d <= 4; ++d) {
        double p = 1.0;
        if (d <= k)
            for (int r = 0; r < d * d; ++r) p = p * t;
        e[d - 1] = d <= k ? p : 0.0;
    }
}

// Z = sum_d c_d t^(d^2) in hop order; returns the entropy ln Z - ln(t) S / Z
// with S = sum_d c_d d^2 t^(d^2)
__device__ double entropy_of_t(const double* c, int k, double t, double& z) {
#pragma clang fp contract(off)
    double e[4];
    gauss_of_t(t, k, e);
    z = 0.0;
    double sw = 0.0;
    for (int d = 0; d < k; ++d) {
        const double term = c[d] * e[d];
        z = z + term;
        sw = sw + term * (double)((d + 1) * (d + 1));
    }
    const double lt = ln_ieee(t);
    return ln_ieee(z) - lt * (sw / z);
}

// Per node: t by bisection (the entropy grows with t; t = 1, the uniform
// distribution, when the target reaches its largest value ln N), then
// Z_i, 1/Z_i and A[i][d] = t^(d^2) / Z_i = NS_{j|i} for a node j at hop d+1.
__global__ void k_calibrate(int32_t n, int32_t k, const int32_t* __restrict__ cnt, double perp,
                            double* __restrict__ tn, double* __restrict__ A,
                            double* __restrict__ invZ, float* __restrict__ invZf,
                            float* __restrict__ invZlo) {
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double c[4] = {0.0, 0.0, 0.0, 0.0};
    int64_t N = 0;
    for (int d = 0; d < k; ++d) {
        c[d] = (double)cnt[i * k + d];
        N += cnt[i * k + d];
    }
    const double target = ln_ieee(perp);
    if (N == 0) {
        tn[i] = 1.0;
        for (int d = 0; d < 4; ++d) A[4 * i + d] = 0.0;
        invZ[i] = 0.0;
        invZf[i] = 0.0f;
        invZlo[i] = 0.0f;
        return;
    }
    double z = 0.0, t = 1.0;
    if (entropy_of_t(c, k, 1.0, z) > target) {
        double lo = 0.0, hi = 1.0;
        for (int r = 0; r < 64; ++r) {
            const double mid = 0.5 * (lo + hi);
            if (entropy_of_t(c, k, mid, z) < target)
                lo = mid;
            else
                hi = mid;
        }
        t = 0.5 * (lo + hi);
    }
    entropy_of_t(c, k, t, z);
    double e[4];
    gauss_of_t(t, k, e);
    tn[i] = t;
    for (int d = 0; d < 4; ++d) A[4 * i + d] = d < k ? e[d] / z : 0.0;
    const double iz = 1.0 / z;
    invZ[i] = iz;
    const float hi = (float)iz;
    invZf[i] = hi;
    invZlo[i] = (float)(iz - (double)hi);
}

// ------------------------------------------------------------------ weighted graphs
// Positive symmetric edge lengths, one per CSR entry.  GD_ij of Eq. NS is
// the length of the shortest i-j path of at most k edges for j in NNG(i, k)
// (the hop-defined pattern), the smaller of the two directions (path sums
// are rounded in path order); E_ij = exp(-GD_ij^2 / (2 sigma^2)) per entry
// replaces e_d, so P~_ij = E_ij (1/Z_i + 1/Z_j) / 2 with Z_i = sum_l E_il.
// The exponential is computed from IEEE operations only (see exp_neg_ieee),
// so P~ and the integer sampling table are reproducible bit for bit.

// every length positive and finite, and equal to that of the reverse entry
// (the structure is validated first, so the reverse entry exists)
__global__ void k_check_lengths(int32_t n, const int32_t* __restrict__ rp,
                                const int32_t* __restrict__ col, const double* __restrict__ len,
                                int* __restrict__ bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int flag = 0;
    for (int32_t x = rp[i]; x < rp[i + 1]; ++x) {
        const double l = len[x];
        if (!(l > 0.0 && l <= 1.7976931348623157e308)) flag |= 32;
        const int32_t v = col[x];
        int32_t lo = rp[v], hi = rp[v + 1];
        while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            if (col[mid] < (int32_t)i)
                lo = mid + 1;
            else
                hi = mid;
        }
        if (lo < rp[v + 1] && !(len[lo] == l)) flag |= 64;
    }
    if (flag) atomicOr(bad, flag);
}

// e^x for x <= 0: Cody and Waite's reduction n = floor(x / ln2 + 1/2),
// r = (x - n L1) - n L2 (ln 2 = L1 + L2, L1 with 32 significant bits so n L1
// is exact), |r| <= 0.35; e^r by Taylor's series to r^13 (Horner's rule,
// coefficients 1/j! by successive division); e^x = 2^n e^r.  0 below -708,
// where 2^n e^r would leave the normal range.
__device__ double exp_neg_ieee(double x) {
#pragma clang fp contract(off)
    if (x < -708.0) return 0.0;
    const double n = floor(x * 1.44269504088896340736 + 0.5);
    const double r = (x - n * 6.93147180369123816490e-01) - n * 1.90821492927058770002e-10;
    double c[14];
    c[0] = 1.0;
    for (int j = 1; j < 14; ++j) c[j] = c[j - 1] / (double)j;
    double p = c[13];
    for (int j = 12; j >= 0; --j) p = p * r + c[j];
    return ldexp(p, (int)n);
}

__device__ __forceinline__ int64_t row_find(const uint32_t* __restrict__ ch, int64_t lo,
                                            int64_t hi, int32_t key) {
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int32_t)(ch[mid] & COL_MASK) < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

__global__ void k_fill_inf(int64_t m, double* __restrict__ d) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x < m) d[x] = __longlong_as_double(0x7FF0000000000000LL);
}

// One Bellman-Ford round from the previous round's distances only (so round
// r admits paths of at most r edges): entry x of row i (node j) takes the
// least of its own distance and, over the graph neighbours u of j inside
// {i} + NNG(i, k), dist(u) + len(u, j).  One wave per row, lanes over its
// entries; a neighbour's slot is found by binary search in the sorted row.
__global__ __launch_bounds__(256) void k_bf_round(int32_t n, const int64_t* __restrict__ prp,
                                                  const uint32_t* __restrict__ ch,
                                                  const int32_t* __restrict__ rp,
                                                  const int32_t* __restrict__ col,
                                                  const double* __restrict__ len,
                                                  const double* __restrict__ dprev,
                                                  double* __restrict__ dcur) {
#pragma clang fp contract(off)
    const int lane = __lane_id();
    const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const int64_t nw = (int64_t)gridDim.x * blockDim.x / WAVE;
    for (int64_t i = w0; i < n; i += nw) {
        const int64_t rs = prp[i], re = prp[i + 1];
        for (int64_t x = rs + lane; x < re; x += WAVE) {
            const int32_t j = (int32_t)(ch[x] & COL_MASK);
            double best = dprev[x];
            for (int32_t e = rp[j]; e < rp[j + 1]; ++e) {
                const int32_t u = col[e];
                double du;
                if (u == (int32_t)i) {
                    du = 0.0;
                } else {
                    const int64_t y = row_find(ch, rs, re, u);
                    if (y >= re || (int32_t)(ch[y] & COL_MASK) != u) continue;
                    du = dprev[y];
                }
                const double c = du + len[e];
                if (c < best) best = c;
            }
            dcur[x] = best;
        }
    }
}

// GD of every entry as the smaller of its two directions, then
// E = exp(-GD^2 / s2) with s2 = 2 sigma^2
__global__ __launch_bounds__(256) void k_bf_finish(int32_t n, const int64_t* __restrict__ prp,
                                                   const uint32_t* __restrict__ ch,
                                                   const double* __restrict__ gd, double s2,
                                                   double* __restrict__ E) {
#pragma clang fp contract(off)
    const int lane = __lane_id();
    const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const int64_t nw = (int64_t)gridDim.x * blockDim.x / WAVE;
    for (int64_t i = w0; i < n; i += nw) {
        for (int64_t x = prp[i] + lane; x < prp[i + 1]; x += WAVE) {
            const int32_t j = (int32_t)(ch[x] & COL_MASK);
            const int64_t y = row_find(ch, prp[j], prp[j + 1], (int32_t)i);
            const double a = gd[x], b = gd[y];
            const double m = a < b ? a : b;
            const double q = m * m;
            E[x] = exp_neg_ieee(-(q / s2));
        }
    }
}

// Z_i = sum of the row's E in entry order (one thread per row)
__global__ void k_weighted_z(int32_t n, const int64_t* __restrict__ prp,
                             const double* __restrict__ E, double* __restrict__ invZ,
                             float* __restrict__ invZf, float* __restrict__ invZlo) {
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double z = 0.0;
    for (int64_t x = prp[i]; x < prp[i + 1]; ++x) z = z + E[x];
    const double iz = prp[i + 1] > prp[i] ? 1.0 / z : 0.0;
    invZ[i] = iz;
    const float hi = (float)iz;
    invZf[i] = hi;
    invZlo[i] = (float)(iz - (double)hi);
}

// P~_ij = ((1/Z_i + 1/Z_j) e_d) / 2 (E_ij in place of e_d for a weighted
// graph), or with node-wise sigma (A non-NULL)
// (A_i[d] + A_j[d]) / 2.  Per row: W_i = sum_j trunc(P~_ij 2^32)
// (exact integer), qt_i = sum_j P~_ij (FP64: lane l of the G lanes sums
// entries l, l+G, ... in order, then a butterfly over the group).
__device__ __forceinline__ void row_weights_row(int64_t i, int lane, int G,
                                                const int64_t* __restrict__ prp,
                                                const uint32_t* __restrict__ ch,
                                                const double* __restrict__ invZ, const ECoef& ec,
                                                const double* __restrict__ A,
                                                const double* __restrict__ Ex,
                                                uint64_t* __restrict__ W, double* __restrict__ qt,
                                                float* __restrict__ qtf) {
#pragma clang fp contract(off)
    const double izi = invZ[i];
    unsigned long long ws = 0;
    double qs = 0.0;
    int64_t x = prp[i] + lane;
    const int64_t re = prp[i + 1];
    if (!A && !Ex) {
        // one global sigma: four entries' loads and gathers in flight, the
        // terms still added in entry order
        constexpr int U = 4;
        for (; x + (int64_t)(U - 1) * G < re; x += (int64_t)U * G) {
            uint32_t e[U];
            double zj[U];
#pragma unroll
            for (int q = 0; q < U; ++q) e[q] = ch[x + (int64_t)q * G];
#pragma unroll
            for (int q = 0; q < U; ++q) zj[q] = invZ[e[q] & COL_MASK];
#pragma unroll
            for (int q = 0; q < U; ++q) {
                const double s = izi + zj[q];
                const double t = pick_e(ec.e, e[q] >> 30) * s;
                const double p = t * 0.5;
                ws += (unsigned long long)(p * 4294967296.0);
                qs = qs + p;
            }
        }
    }
    for (; x < re; x += G) {
        const uint32_t e = ch[x];
        double p;
        if (A) {
            const double s = A[4 * i + (e >> 30)] + A[4 * (int64_t)(e & COL_MASK) + (e >> 30)];
            p = s * 0.5;
        } else {
            const double s = izi + invZ[e & COL_MASK];
            const double t = (Ex ? Ex[x] : pick_e(ec.e, e >> 30)) * s;
            p = t * 0.5;
        }
        ws += (unsigned long long)(p * 4294967296.0);
        qs = qs + p;
    }
    ws = group_sum_rt(ws, G);
    qs = group_sum_rt(qs, G);
    if (lane == 0) {
        W[i] = ws;
        qt[i] = qs;
        qtf[i] = (float)qs;
    }
}

template <int G>
__global__ __launch_bounds__(256) void k_row_weights(int32_t n, const int64_t* __restrict__ prp,
                                                     const uint32_t* __restrict__ ch,
                                                     const double* __restrict__ invZ, ECoef ec,
                                                     const double* __restrict__ A,
                                                     const double* __restrict__ Ex,
                                                     uint64_t* __restrict__ W,
                                                     double* __restrict__ qt,
                                                     float* __restrict__ qtf) {
    const int lane = threadIdx.x % G;
    const int64_t grp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    const int64_t ngrp = (int64_t)gridDim.x * blockDim.x / G;
    for (int64_t i = grp; i < n; i += ngrp)
        row_weights_row(i, lane, G, prp, ch, invZ, ec, A, Ex, W, qt, qtf);
}

// Union of graphs: every graph keeps the group size its own single-graph
// build picks, so its weights come out bit for bit the same.  Graph c owns
// waves woff[c] .. woff[c+1]-1, each wave 64/G consecutive rows of it.
__global__ __launch_bounds__(256) void k_row_weights_union(int32_t count,
                                                           const int32_t* __restrict__ woff,
                                                           const int4* __restrict__ gtab,
                                                           const int64_t* __restrict__ prp,
                                                           const uint32_t* __restrict__ ch,
                                                           const double* __restrict__ invZ,
                                                           ECoef ec, uint64_t* __restrict__ W,
                                                           double* __restrict__ qt,
                                                           float* __restrict__ qtf) {
    const int32_t total = woff[count];
    const int32_t nwaves = (int32_t)(gridDim.x * (blockDim.x / WAVE));
    for (int32_t gw = __builtin_amdgcn_readfirstlane((int32_t)(blockIdx.x * (blockDim.x / WAVE) +
                                                               threadIdx.x / WAVE));
         gw < total; gw += nwaves) {
        int32_t lo = 0, hi = count - 1;  // last c with woff[c] <= gw
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (woff[mid] <= gw)
                lo = mid;
            else
                hi = mid - 1;
        }
        const int4 t = gtab[lo];  // (base, n, G, -)
        const int G = t.z;
        const int32_t r = (gw - woff[lo]) * (WAVE / G) + (int32_t)(__lane_id() / G);
        if (r < t.y)
            row_weights_row((int64_t)t.x + r, __lane_id() % G, G, prp, ch, invZ, ec, nullptr,
                            nullptr, W, qt, qtf);
    }
}

// guide[b] = draw result for the smallest word of bucket b (top gbits bits);
// guide[2^gbits] = draw result for the largest word.
__global__ void k_guide(int32_t n, const uint64_t* __restrict__ C, int gbits,
                        int32_t* __restrict__ guide) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nb = (int64_t)1 << gbits;
    if (b > nb) return;
    const uint64_t S = C[n];
    if (S == 0) {
        guide[b] = 0;
        return;
    }
    const uint64_t r = b < nb ? __umul64hi((uint64_t)b << (64 - gbits), S) : S - 1;
    int32_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        if (C[mid + 1] > r)
            hi = mid;
        else
            lo = mid + 1;
    }
    guide[b] = lo;
}

// P~ of entry e of row i, as row_weights_row computes it
__device__ __forceinline__ double entry_p(int64_t i, int64_t x, uint32_t e,
                                          const double* __restrict__ invZ, const ECoef& ec,
                                          const double* __restrict__ A,
                                          const double* __restrict__ Ex) {
#pragma clang fp contract(off)
    if (A) {
        const double s = A[4 * i + (e >> 30)] + A[4 * (int64_t)(e & COL_MASK) + (e >> 30)];
        return s * 0.5;
    }
    const double s = invZ[i] + invZ[e & COL_MASK];
    const double t = (Ex ? Ex[x] : pick_e(ec.e, e >> 30)) * s;
    return t * 0.5;
}

__global__ void k_materialise_P(int32_t n, const int64_t* __restrict__ prp,
                                const uint32_t* __restrict__ ch, const double* __restrict__ invZ,
                                ECoef ec, const double* __restrict__ A,
                                const double* __restrict__ Ex, double* __restrict__ P) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int64_t x = prp[i]; x < prp[i + 1]; ++x) P[x] = entry_p(i, x, ch[x], invZ, ec, A, Ex);
}

// P~ of the entries x0 .. x1-1 of row i (same operations as k_materialise_P)
__global__ void k_materialise_row(int32_t i, int64_t x0, int64_t x1,
                                  const uint32_t* __restrict__ ch, const double* __restrict__ invZ,
                                  ECoef ec, const double* __restrict__ A,
                                  const double* __restrict__ Ex, double* __restrict__ P) {
    const int64_t x = x0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= x1) return;
    P[x - x0] = entry_p(i, x, ch[x], invZ, ec, A, Ex);
}

static int pick_group(double mean_len) {
    if (mean_len <= 4) return 4;
    if (mean_len <= 8) return 8;
    if (mean_len <= 16) return 16;
    if (mean_len <= 32) return 32;
    return 64;
}

template <int G>
static void launch_row_weights(drg_ctx* ctx, drg_sim* s, const ECoef& ec) {
    const int64_t groups = s->n;
    const int grid = (int)std::min<int64_t>((groups * G + 255) / 256, 1 << 20);
    hipLaunchKernelGGL(k_row_weights<G>, dim3(std::max(grid, 1)), dim3(256), 0, ctx->stream, s->n,
                       s->row_ptr.get(), s->colhop.get(), s->invZ.get(), ec, s->A.get(),
                       s->Ex.get(), s->W.get(), s->qt.get(), s->qtf.get());
    DRG_LAUNCH_CHECK();
}

__global__ void k_gather_rowptr(int32_t m, const int32_t* __restrict__ at,
                                const int64_t* __restrict__ prp, int64_t* __restrict__ out) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < m) out[c] = prp[at[c]];
}

// Row weights of a union, graph by graph (see k_row_weights_union).
static void union_row_weights(drg_ctx* ctx, drg_sim* s, const ECoef& ec, UnionInfo* u) {
    hipStream_t st = ctx->stream;
    const int32_t m = u->count + 1;
    DevBuf<int32_t> at(m);
    DevBuf<int64_t> rpv(m);
    DRG_HIP(hipMemcpyAsync(at.get(), u->base.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice,
                           st));
    hipLaunchKernelGGL(k_gather_rowptr, dim3(ceil_div(m, 256)), dim3(256), 0, st, m, at.get(),
                       s->row_ptr.get(), rpv.get());
    DRG_LAUNCH_CHECK();
    std::vector<int64_t> h(m);
    DRG_HIP(hipMemcpyAsync(h.data(), rpv.get(), sizeof(int64_t) * m, hipMemcpyDeviceToHost, st));
    DRG_HIP(hipStreamSynchronize(st));
    u->nnz.assign(u->count, 0);
    std::vector<int4> tab(u->count);
    std::vector<int32_t> woff(u->count + 1, 0);
    for (int32_t c = 0; c < u->count; ++c) {
        const int32_t nc = u->base[c + 1] - u->base[c];
        u->nnz[c] = h[c + 1] - h[c];
        const int G = pick_group((double)u->nnz[c] / (double)nc);
        tab[c] = make_int4(u->base[c], nc, G, 0);
        const int64_t w = ((int64_t)nc + WAVE / G - 1) / (WAVE / G);
        if ((int64_t)woff[c] + w >= ((int64_t)1 << 31))
            throw Error(DRG_E_INVALID, "union too large");
        woff[c + 1] = woff[c] + (int32_t)w;
    }
    DevBuf<int4> dtab(u->count);
    DevBuf<int32_t> dwoff(m);
    DRG_HIP(hipMemcpyAsync(dtab.get(), tab.data(), sizeof(int4) * u->count, hipMemcpyHostToDevice,
                           st));
    DRG_HIP(hipMemcpyAsync(dwoff.get(), woff.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice,
                           st));
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((woff[u->count] + 3) / 4,
                                                                  (int64_t)ctx->num_cu * 64));
    hipLaunchKernelGGL(k_row_weights_union, dim3((unsigned)blocks), dim3(256), 0, st, u->count,
                       dwoff.get(), dtab.get(), s->row_ptr.get(), s->colhop.get(), s->invZ.get(),
                       ec, s->W.get(), s->qt.get(), s->qtf.get());
    DRG_LAUNCH_CHECK();
    DRG_HIP(hipStreamSynchronize(st));
}

drg_sim* build_similarity(drg_ctx* ctx, const drg_csr* g, int k, double sigma, uint32_t flags,
                          UnionInfo* u, double perplexity, const double* lengths) {
    if (!g) throw Error(DRG_E_INVALID, "graph is NULL");
    if (k < 1 || k > 4) throw Error(DRG_E_INVALID, "k must be in 1..4");
    const bool nodewise = perplexity != 0.0;
    if (nodewise) {
        if (!(perplexity >= 1.0) || !(perplexity < 1e300))
            throw Error(DRG_E_INVALID, "perplexity must be >= 1 and finite");
        if (u) throw Error(DRG_E_UNSUPPORTED, "batched layout: one global sigma only");
        if (lengths) throw Error(DRG_E_UNSUPPORTED, "node-wise sigma of a weighted graph");
        sigma = 1.0;  // not used
    }
    if (lengths && u) throw Error(DRG_E_UNSUPPORTED, "batched layout: unweighted graphs only");
    if (!(sigma > 0.0) || !std::isfinite(sigma)) throw Error(DRG_E_INVALID, "sigma must be > 0");
    if (g->n <= 0 || g->n >= (1 << 30)) throw Error(DRG_E_INVALID, "n must be in 1..2^30-1");
    if (g->nnz < 0 || !g->row_ptr || (g->nnz > 0 && !g->col))
        throw Error(DRG_E_INVALID, "bad CSR pointers or nnz");
    // a weighted build looks up reverse entries: the structure is always checked
    validate_csr_impl(ctx, g, lengths != nullptr || (flags & DRG_VALIDATE) != 0);
    hipStream_t st = ctx->stream;
    const int32_t n = g->n;
    if (lengths && g->nnz > 0) {
        DevBuf<int> bad(1);
        DRG_HIP(hipMemsetAsync(bad.get(), 0, sizeof(int), st));
        hipLaunchKernelGGL(k_check_lengths, dim3(ceil_div(n, 256)), dim3(256), 0, st, n,
                           g->row_ptr, g->col, lengths, bad.get());
        DRG_LAUNCH_CHECK();
        const int f = read_flag(bad, st);
        if (f & 32) throw Error(DRG_E_INVALID, "edge lengths must be positive and finite");
        if (f & 64) throw Error(DRG_E_INVALID, "edge lengths are not symmetric");
    }
    auto s = std::make_unique<drg_sim>();
    s->device = ctx->device;
    s->n = n;
    s->k = k;
    s->sigma = nodewise ? 0.0 : sigma;
    s->perplexity = nodewise ? perplexity : 0.0;
    ECoef ec{};
    for (int d = 1; d <= 4; ++d) {
        ec.e[d - 1] = (d <= k && !nodewise)
                          ? std::exp(-(double)(d * d) / (2.0 * sigma * sigma)) : 0.0;
        s->e[d - 1] = ec.e[d - 1];
    }
    DevBuf<int32_t> cnt((int64_t)n * k);
    s->row_ptr.alloc((int64_t)n + 1);
    if (k == 1) {
        hipLaunchKernelGGL(k_deg_counts, dim3(ceil_div((int64_t)n + 1, 256)), dim3(256), 0, st, n,
                           g->row_ptr, cnt.get(), s->row_ptr.get());
        DRG_LAUNCH_CHECK();
        s->nnz = g->nnz;
        s->colhop.alloc(s->nnz);
        if (s->nnz > 0) {
            hipLaunchKernelGGL(k_copy_cols, dim3(ceil_div(s->nnz, 256)), dim3(256), 0, st, g->nnz,
                               g->col, s->colhop.get());
            DRG_LAUNCH_CHECK();
        }
    } else {
        // launch shape: LDS bitmap when it fits, global bitmaps otherwise; in a
        // batch the bitmap spans the largest graph only
        const int32_t span = u ? u->max_comp : n;
        const int nwords = (span + 31) / 32;
        const size_t lds = (size_t)nwords * 4;
        const bool in_lds = lds + 512 <= (size_t)ctx->max_lds;
        DevBuf<unsigned long long> d2(1);
        DRG_HIP(hipMemsetAsync(d2.get(), 0, sizeof(unsigned long long), st));
        hipLaunchKernelGGL(k_sum_deg2, dim3(ceil_div(n, 256)), dim3(256), 0, st, n, g->row_ptr,
                           d2.get());
        DRG_LAUNCH_CHECK();
        unsigned long long sdeg2 = 0;
        DRG_HIP(hipMemcpyAsync(&sdeg2, d2.get(), sizeof(sdeg2), hipMemcpyDeviceToHost, st));
        DRG_HIP(hipStreamSynchronize(st));
        const double visit_deg = g->nnz > 0 ? (double)sdeg2 / (double)g->nnz : 1.0;
        const int G = pick_group(visit_deg);
        int per_cu = in_lds ? std::max(1, (int)(ctx->max_lds / (lds + 512))) : 4;
        per_cu = std::min(per_cu, 8);
        const int grid = std::max(1, std::min<int>(ctx->num_cu * per_cu, n));
        DevBuf<int32_t> queue;
        int64_t qcap = 0;
        if (k >= 3) {
            qcap = span;
            queue.alloc((int64_t)grid * qcap);
        }
        DevBuf<uint32_t> gbm;
        if (!in_lds) gbm.alloc((int64_t)grid * nwords);
        DevBuf<int32_t> work(1);
        BfsArgs a{};
        a.n = n;
        a.k = k;
        a.nwords = nwords;
        a.rp = g->row_ptr;
        a.col = g->col;
        a.cnt = cnt.get();
        a.queue = queue.get();
        a.qcap = qcap;
        a.gbm = gbm.get();
        a.work = work.get();
        a.node_base = u ? u->node_base : nullptr;
        DRG_HIP(hipMemsetAsync(work.get(), 0, sizeof(int32_t), st));
        if (in_lds)
            launch_khop<false, true>(ctx, a, G, grid, lds);
        else
            launch_khop<false, false>(ctx, a, G, grid, 0);
        DevBuf<int64_t> len(n);
        hipLaunchKernelGGL(k_row_len, dim3(ceil_div(n, 256)), dim3(256), 0, st, n, k, cnt.get(),
                           len.get());
        DRG_LAUNCH_CHECK();
        exclusive_scan<int64_t>(len.get(), s->row_ptr.get(), n, st);
        int64_t nnz = 0;
        DRG_HIP(hipMemcpyAsync(&nnz, s->row_ptr.get() + n, sizeof(int64_t),
                               hipMemcpyDeviceToHost, st));
        DRG_HIP(hipStreamSynchronize(st));
        s->nnz = nnz;
        s->colhop.alloc(nnz);
        a.prp = s->row_ptr.get();
        a.colhop = s->colhop.get();
        DRG_HIP(hipMemsetAsync(work.get(), 0, sizeof(int32_t), st));
        if (in_lds)
            launch_khop<true, true>(ctx, a, G, grid, lds);
        else
            launch_khop<true, false>(ctx, a, G, grid, 0);
        DRG_HIP(hipStreamSynchronize(st));
    }
    s->invZ.alloc(n);
    s->invZf.alloc(n);
    s->invZlo.alloc(n);
    s->qt.alloc(n);
    s->qtf.alloc(n);
    s->W.alloc(n);
    s->C.alloc((int64_t)n + 1);
    if (lengths) {
        // GD by k Bellman-Ford rounds (ping-pong between two distance arrays),
        // then E per entry and Z per row
        const int64_t nnz = s->nnz;
        s->Ex.alloc(std::max<int64_t>(nnz, 1));
        if (nnz > 0) {
            DevBuf<double> da(nnz), db(nnz);
            hipLaunchKernelGGL(k_fill_inf, dim3(ceil_div(nnz, 256)), dim3(256), 0, st, nnz,
                               da.get());
            DRG_LAUNCH_CHECK();
            const int grid = (int)std::max<int64_t>(
                1, std::min<int64_t>(ceil_div((int64_t)n * WAVE, 256), (int64_t)ctx->num_cu * 32));
            double* dp = da.get();
            double* dc = db.get();
            for (int r = 1; r <= k; ++r) {
                hipLaunchKernelGGL(k_bf_round, dim3(grid), dim3(256), 0, st, n,
                                   s->row_ptr.get(), s->colhop.get(), g->row_ptr, g->col,
                                   lengths, dp, dc);
                DRG_LAUNCH_CHECK();
                std::swap(dp, dc);
            }
            hipLaunchKernelGGL(k_bf_finish, dim3(grid), dim3(256), 0, st, n, s->row_ptr.get(),
                               s->colhop.get(), dp, 2.0 * sigma * sigma, s->Ex.get());
            DRG_LAUNCH_CHECK();
            DRG_HIP(hipStreamSynchronize(st));
        }
        hipLaunchKernelGGL(k_weighted_z, dim3(ceil_div(n, 256)), dim3(256), 0, st, n,
                           s->row_ptr.get(), s->Ex.get(), s->invZ.get(), s->invZf.get(),
                           s->invZlo.get());
    } else if (nodewise) {
        s->A.alloc(4 * (int64_t)n);
        s->tnode.alloc(n);
        hipLaunchKernelGGL(k_calibrate, dim3(ceil_div(n, 256)), dim3(256), 0, st, n, k,
                           cnt.get(), perplexity, s->tnode.get(), s->A.get(),
                           s->invZ.get(), s->invZf.get(), s->invZlo.get());
    } else {
        hipLaunchKernelGGL(k_normalise, dim3(ceil_div(n, 256)), dim3(256), 0, st, n, k, cnt.get(),
                           ec, s->invZ.get(), s->invZf.get(), s->invZlo.get());
    }
    DRG_LAUNCH_CHECK();
    const double mean_len = (double)s->nnz / (double)n;
    if (u) {
        union_row_weights(ctx, s.get(), ec, u);
    } else {
        switch (pick_group(mean_len)) {
            case 4: launch_row_weights<4>(ctx, s.get(), ec); break;
            case 8: launch_row_weights<8>(ctx, s.get(), ec); break;
            case 16: launch_row_weights<16>(ctx, s.get(), ec); break;
            case 32: launch_row_weights<32>(ctx, s.get(), ec); break;
            default: launch_row_weights<64>(ctx, s.get(), ec); break;
        }
    }
    exclusive_scan<uint64_t>(s->W.get(), s->C.get(), n, st);
    DRG_HIP(hipMemcpyAsync(&s->S, s->C.get() + n, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    DRG_HIP(hipStreamSynchronize(st));
    s->n_active = (int32_t)count_nonempty_rows<int64_t>(s->row_ptr.get(), n, st);
    if (!u && s->nnz > 0) {
        DevBuf<unsigned long long> l2(1);
        sum_len2_by_group(s->row_ptr.get(), nullptr, n, l2.get(), 1, st);
        unsigned long long h = 0;
        DRG_HIP(hipMemcpyAsync(&h, l2.get(), sizeof(h), hipMemcpyDeviceToHost, st));
        DRG_HIP(hipStreamSynchronize(st));
        s->len_wmean = (double)h / (double)s->nnz;
    }
    s->rec.alloc(n);
    s->g.alloc(n);
    if (u) {  // per-graph guides belong to the batch
        s->gbits = 0;
        DRG_HIP(hipStreamSynchronize(st));
        return s.release();
    }
    int gbits = 1;
    while (gbits < 30 && ((int64_t)1 << gbits) < n) ++gbits;
    s->gbits = gbits;
    s->guide.alloc(((int64_t)1 << gbits) + 1);
    hipLaunchKernelGGL(k_guide, dim3(ceil_div(((int64_t)1 << gbits) + 1, 256)), dim3(256), 0, st,
                       n, s->C.get(), gbits, s->guide.get());
    DRG_LAUNCH_CHECK();
    DRG_HIP(hipStreamSynchronize(st));
    // the column-blocked sweep carries one 1/Z per record and a hop per entry:
    // unweighted graphs with one global sigma only
    if (!nodewise && !lengths && blocked_wanted(ctx, s.get())) build_blocked(ctx, s.get());
    return s.release();
}

void sim_export_rows(const drg_sim* s, int32_t nrows, const int32_t* rows, int64_t cap,
                     int64_t* row_len, int32_t* col, uint8_t* hop, double* P, double* qt,
                     uint64_t* W, double* invZ) {
    if (nrows < 0 || (nrows > 0 && !rows)) throw Error(DRG_E_INVALID, "rows");
    DRG_HIP(hipSetDevice(s->device));
    DRG_HIP(hipDeviceSynchronize());
    std::vector<int64_t> a(nrows), b(nrows);
    int64_t total = 0;
    for (int32_t r = 0; r < nrows; ++r) {
        const int32_t i = rows[r];
        if (i < 0 || i >= s->n) throw Error(DRG_E_INVALID, "row index out of range");
        int64_t se[2];
        DRG_HIP(hipMemcpy(se, s->row_ptr.get() + i, sizeof(se), hipMemcpyDeviceToHost));
        a[r] = se[0];
        b[r] = se[1];
        total += se[1] - se[0];
    }
    if (row_len)
        for (int32_t r = 0; r < nrows; ++r) row_len[r] = b[r] - a[r];
    if ((col || hop || P) && total > cap)
        throw Error(DRG_E_INVALID, "the rows hold more entries than cap");
    ECoef ec{};
    for (int d = 0; d < 4; ++d) ec.e[d] = s->e[d];
    int64_t o = 0;
    for (int32_t r = 0; r < nrows; ++r) {
        const int32_t i = rows[r];
        const int64_t len = b[r] - a[r];
        if (len > 0 && (col || hop)) {
            std::vector<uint32_t> ch(len);
            DRG_HIP(hipMemcpy(ch.data(), s->colhop.get() + a[r], sizeof(uint32_t) * len,
                              hipMemcpyDeviceToHost));
            for (int64_t x = 0; x < len; ++x) {
                if (col) col[o + x] = (int32_t)(ch[x] & COL_MASK);
                if (hop) hop[o + x] = (uint8_t)((ch[x] >> 30) + 1);
            }
        }
        if (len > 0 && P) {
            DevBuf<double> dP(len);
            hipLaunchKernelGGL(k_materialise_row, dim3(ceil_div(len, 256)), dim3(256), 0, nullptr,
                               i, a[r], b[r], s->colhop.get(), s->invZ.get(), ec, s->A.get(),
                               s->Ex.get(), dP.get());
            DRG_LAUNCH_CHECK();
            DRG_HIP(hipMemcpy(P + o, dP.get(), sizeof(double) * len, hipMemcpyDeviceToHost));
        }
        if (qt) DRG_HIP(hipMemcpy(qt + r, s->qt.get() + i, sizeof(double), hipMemcpyDeviceToHost));
        if (W) DRG_HIP(hipMemcpy(W + r, s->W.get() + i, sizeof(uint64_t), hipMemcpyDeviceToHost));
        if (invZ)
            DRG_HIP(hipMemcpy(invZ + r, s->invZ.get() + i, sizeof(double), hipMemcpyDeviceToHost));
        o += len;
    }
}

void sim_export(const drg_sim* s, int64_t* row_ptr, int32_t* col, uint8_t* hop, double* P,
                double* qt, uint64_t* W, double* e, double* invZ) {
    const int32_t n = s->n;
    const int64_t nnz = s->nnz;
    DRG_HIP(hipSetDevice(s->device));
    DRG_HIP(hipDeviceSynchronize());
    if (row_ptr)
        DRG_HIP(hipMemcpy(row_ptr, s->row_ptr.get(), sizeof(int64_t) * (n + 1),
                          hipMemcpyDeviceToHost));
    if ((col || hop) && nnz > 0) {
        std::vector<uint32_t> ch(nnz);
        DRG_HIP(hipMemcpy(ch.data(), s->colhop.get(), sizeof(uint32_t) * nnz,
                          hipMemcpyDeviceToHost));
        for (int64_t x = 0; x < nnz; ++x) {
            if (col) col[x] = (int32_t)(ch[x] & COL_MASK);
            if (hop) hop[x] = (uint8_t)((ch[x] >> 30) + 1);
        }
    }
    if (P && nnz > 0) {
        DevBuf<double> dP(nnz);
        ECoef ec{};
        for (int d = 0; d < 4; ++d) ec.e[d] = s->e[d];
        hipLaunchKernelGGL(k_materialise_P, dim3(ceil_div(n, 256)), dim3(256), 0, nullptr, n,
                           s->row_ptr.get(), s->colhop.get(), s->invZ.get(), ec, s->A.get(),
                           s->Ex.get(), dP.get());
        DRG_LAUNCH_CHECK();
        DRG_HIP(hipMemcpy(P, dP.get(), sizeof(double) * nnz, hipMemcpyDeviceToHost));
    }
    if (qt) DRG_HIP(hipMemcpy(qt, s->qt.get(), sizeof(double) * n, hipMemcpyDeviceToHost));
    if (W) DRG_HIP(hipMemcpy(W, s->W.get(), sizeof(uint64_t) * n, hipMemcpyDeviceToHost));
    if (invZ) DRG_HIP(hipMemcpy(invZ, s->invZ.get(), sizeof(double) * n, hipMemcpyDeviceToHost));
    if (e)
        for (int d = 0; d < s->k; ++d) e[d] = s->e[d];
}

void sim_node_sigma(const drg_sim* s, double* sigma) {
    if (!sigma) throw Error(DRG_E_INVALID, "sigma is NULL");
    DRG_HIP(hipSetDevice(s->device));
    DRG_HIP(hipDeviceSynchronize());
    const int32_t n = s->n;
    std::vector<int64_t> rp((size_t)n + 1);
    DRG_HIP(hipMemcpy(rp.data(), s->row_ptr.get(), sizeof(int64_t) * (n + 1),
                      hipMemcpyDeviceToHost));
    std::vector<double> t;
    if (s->tnode.get()) {
        t.resize(n);
        DRG_HIP(hipMemcpy(t.data(), s->tnode.get(), sizeof(double) * n, hipMemcpyDeviceToHost));
    }
    for (int32_t i = 0; i < n; ++i) {
        if (rp[i + 1] == rp[i]) {
            sigma[i] = 0.0;
        } else if (t.empty()) {
            sigma[i] = s->sigma;
        } else {
            const double lt = std::log(t[i]);
            sigma[i] = lt < 0.0 ? std::sqrt(-0.5 / lt) : HUGE_VAL;
        }
    }
}

}  // namespace drg
