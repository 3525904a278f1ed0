// blocked.hip -- column-blocked copy of P~ and the LDS-staged sweep.
//
// The attraction sweep reads one record (y_c(j), 1/Z_j) per stored pair.
// On a large graph the records do not fit an L2 slice, and a random 16-byte
// gather drags a whole cache line through the memory hierarchy.  Here the
// columns are cut into blocks of BW = 2^bits nodes: a workgroup copies one
// block's records into LDS (BW x 16 bytes, one contiguous read) and sweeps,
// for a range of rows, the entries whose column falls in that block.  Those
// entries are stored per block in row order as 16-bit words (block-local
// column in the low 13 bits, hop-1 above), so the HBM stream is 2 bytes per
// pair and every neighbour gather is an LDS read.  Each (block, row) pair
// leaves a partial attraction; a second kernel adds the partials of a row in
// block order (deterministic), draws the row's negatives and applies the step.
#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "drg_blocked.hpp"
#include "drg_internal.hpp"

namespace drg {

// cnt[b*n + i] = number of entries of row i whose column lies in block b
// (columns are counted from col_base: a graph inside a union)
__global__ void k_blk_count(int32_t n, int32_t nb, int bits, const int64_t* __restrict__ prp,
                            const uint32_t* __restrict__ ch, uint32_t col_base,
                            int32_t* __restrict__ cnt) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * nb) return;
    const int32_t i = (int32_t)(t % n);
    const int32_t b = (int32_t)(t / n);
    auto lb = [&](int64_t lo, int64_t hi, uint32_t key) {
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if ((ch[mid] & COL_MASK) - col_base < key)
                lo = mid + 1;
            else
                hi = mid;
        }
        return lo;
    };
    const int64_t rs = prp[i], re = prp[i + 1];
    const int64_t s = lb(rs, re, (uint32_t)b << bits);
    const int64_t e = lb(s, re, (uint32_t)(b + 1) << bits);
    cnt[t] = (int32_t)(e - s);
}

__global__ void k_widen(int64_t m, const int32_t* __restrict__ a, int64_t* __restrict__ b) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < m) b[t] = a[t];
}

// off[b*(n+1) + i] = flat[b*n + i] - flat[b*n] for i <= n
__global__ void k_blk_offsets(int32_t n, int32_t nb, const int64_t* __restrict__ flat,
                              int64_t* __restrict__ base, int32_t* __restrict__ off) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)(n + 1) * nb) return;
    const int32_t b = (int32_t)(t / (n + 1));
    const int32_t i = (int32_t)(t % (n + 1));
    const int64_t b0 = flat[(int64_t)b * n];
    off[t] = (int32_t)(flat[(int64_t)b * n + i] - b0);
    if (i == 0) base[b] = b0;
    if (t == 0) base[nb] = flat[(int64_t)nb * n];
}

// one wave per row: for each block, copy the row's segment (coalesced)
__global__ __launch_bounds__(256) void k_blk_fill(int32_t n, int32_t nb, int bits,
                                                  const int64_t* __restrict__ prp,
                                                  const uint32_t* __restrict__ ch,
                                                  uint32_t col_base,
                                                  const int64_t* __restrict__ base,
                                                  const int32_t* __restrict__ off,
                                                  uint16_t* __restrict__ ent) {
    const int lane = __lane_id();
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    if (row >= n) return;
    const int32_t i = (int32_t)row;
    const int64_t rs = prp[i], re = prp[i + 1];
    const uint32_t mask = (1u << bits) - 1u;
    int64_t s = rs;
    for (int32_t b = 0; b < nb && s < re; ++b) {
        const int64_t dst = base[b] + off[(int64_t)b * (n + 1) + i];
        const int32_t len = off[(int64_t)b * (n + 1) + i + 1] - off[(int64_t)b * (n + 1) + i];
        for (int32_t x = lane; x < len; x += WAVE) {
            const uint32_t e = ch[s + x];
            ent[dst + x] =
                (uint16_t)((((e & COL_MASK) - col_base) & mask) | ((e >> 30) << BLK_HOP_SHIFT));
        }
        s += len;
    }
}

// Work items: block b's rows cut where the running cost (entries + rc per
// row) crosses multiples of `chunk`; rc >= chunk / ROWCAP keeps every item
// within ROWCAP rows.  item_first[b] = index of b's first item.

__global__ void k_blk_items(int32_t n, int32_t nb, const int32_t* __restrict__ off,
                            const int32_t* __restrict__ item_first, int64_t chunk, int64_t rc,
                            int4* __restrict__ items) {
    const int32_t b = blockIdx.y;
    const int32_t first = item_first[b], cnt = item_first[b + 1] - first;
    const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cnt) return;
    const int32_t* O = off + (int64_t)b * (n + 1);
    auto row_at = [&](int64_t target) {  // first row i with O[i] + rc i >= target
        int32_t lo = 0, hi = n;
        while (lo < hi) {
            const int32_t mid = lo + ((hi - lo) >> 1);
            if ((int64_t)O[mid] + rc * (int64_t)mid < target)
                lo = mid + 1;
            else
                hi = mid;
        }
        return lo;
    };
    const int32_t r0 = c == 0 ? 0 : row_at((int64_t)c * chunk);
    const int32_t r1 = c == cnt - 1 ? n : row_at((int64_t)(c + 1) * chunk);
    items[first + c] = make_int4(b, r0, r1, 0);
}

template <int B, int NH, int F>
__global__ __launch_bounds__(STREAM_BLOCK) void k_sweep_blocked(BlockedArgs a) {
    extern __shared__ float4 s_dyn[];
    const int4 it = a.items[blockIdx.x];
    blk_layout_item<B, NH, F>(a, s_dyn, it.x, it.y, it.z);
}

// The objective's attraction terms over the blocked layout (flat form): the
// row value (KIND 0) or the row's attraction gradient (KIND 1) per block.
template <int B, int NH, int KIND>
__global__ __launch_bounds__(STREAM_BLOCK) void k_obj_blocked(BlockedArgs a) {
    extern __shared__ float4 s_dyn[];
    const int32_t bw = 1 << a.bits;
    float4* s_rec = s_dyn;
    int32_t* s_off = reinterpret_cast<int32_t*>(s_dyn + bw);
    WaveFrag* s_frag = reinterpret_cast<WaveFrag*>(s_dyn + bw + (ROWCAP + 4) / 4);
    const int4 it = a.items[blockIdx.x];
    const int32_t b = it.x, r0 = it.y, r1 = it.z;
    blk_stage_rec(a, s_rec, b);
    blk_stage_off(a, s_off, b, r0, r1);
    if constexpr (KIND == 0)
        blk_flat<2>(a, ObjValOp<B, NH>{hop_weights(a)}, s_rec, s_off, s_frag, b, r0, r1);
    else
        blk_flat<2>(a, ObjGradOp<B, NH>{hop_weights(a)}, s_rec, s_off, s_frag, b, r0, r1);
}

__global__ void k_stage_y(int32_t n, const float2* __restrict__ y, const float* __restrict__ invZ,
                          float4* __restrict__ rec) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) rec[j] = make_float4(y[j].x, y[j].y, invZ[j], 0.0f);
}

struct FinishArgs {
    int32_t n0, nb, M;
    const int64_t* prp;
    const float2* partial;
    const float4* rec;
    const float* qt;
    const uint64_t* C;
    const int32_t* guide;
    int32_t gbits;
    uint64_t S;
    float gamma, clip;
    uint64_t seed, iter;
    float2* g;   // one-sided steps
};

// One thread per finest node: partials in block order, M negatives.
template <int B>
__global__ __launch_bounds__(256) void k_finish(FinishArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n0) return;
    float2 gi = make_float2(0.0f, 0.0f);
    if (a.prp[i + 1] > a.prp[i])
        gi = blk_finish_row<B>(a.partial, a.nb, a.n0, (int32_t)i, a.rec, a.rec[i], a.M, a.seed,
                               a.iter, (int32_t)i,
                               [&](uint64_t w) { return draw_node(w, a.C, a.guide, a.gbits, a.S); },
                               a.gamma * a.qt[i], a.clip);
    a.g[i] = gi;
}

// ------------------------------------------------------------------ Hogwild form
// Asynchronous iteration on the blocked layout.  The rows are cut into
// windows of ASYNC_WIN rows; the work items are launched in window order
// (every item of window w before any item whose first row lies in a later
// window), and each window counts the items that touch it.  The workgroup
// whose item completes a window finishes that window's rows on the spot:
// partials summed in block order, negatives drawn from the live records,
// and the step applied in place to the coordinates and to the records that
// items launched later stage into LDS.  Later windows thus see the earlier
// windows' new positions within the same iteration (Gauss-Seidel across
// windows, Hogwild within one: which updates a workgroup sees depends on
// timing, so runs are not repeatable).
constexpr int32_t ASYNC_WIN = ROWCAP;  // an item spans at most two windows

struct AsyncArgs {
    const int32_t* order;      // launch slot -> item
    uint32_t* wcnt;            // per window: items counted so far (0 between launches)
    const uint32_t* wneed;     // per window: items that touch it
    int32_t nb, M;
    const int64_t* prp;
    float4* rec;               // live records (x, y, 1/Z, 1/Z low part)
    const float* qt;
    const uint64_t* C;
    const int32_t* guide;
    int32_t gbits;
    uint64_t S;
    float gamma, clip, eta;
    uint64_t seed, iter;
    float2* y;                 // level coordinates, updated in place
    const int32_t* cmap;       // finest node -> level node (NULL at level 0)
    const float* w;            // anchor weight of each level node
};

template <int B>
__device__ void blk_async_window(const BlockedArgs& a, const AsyncArgs& h, int32_t win) {
    __threadfence();  // acquire: the other items' partials of this window
    const int32_t r0 = win * ASYNC_WIN, r1 = min(a.n0, r0 + ASYNC_WIN);
    auto draw = [&](uint64_t w) { return draw_node(w, h.C, h.guide, h.gbits, h.S); };
    for (int32_t i = r0 + (int32_t)threadIdx.x; i < r1; i += STREAM_BLOCK) {
        if (h.prp[i + 1] == h.prp[i]) continue;  // isolated: never moves
        const float4 ri = h.rec[i];
        const float2 gi = blk_finish_row<B>(a.partial, h.nb, a.n0, i, h.rec, ri, h.M, h.seed,
                                            h.iter, i, draw, h.gamma * h.qt[i], h.clip);
        if (!h.cmap) {
            const float wi = h.qt[i];
            const float nx = ri.x + h.eta * (gi.x / wi), ny = ri.y + h.eta * (gi.y / wi);
            h.y[i] = make_float2(nx, ny);
            h.rec[i] = make_float4(nx, ny, ri.z, ri.w);
        } else {
            const int32_t c = h.cmap[i];
            const float wc = h.w[c];
            if (wc > 0.0f) {
                atomicAdd(&h.y[c].x, h.eta * (gi.x / wc));
                atomicAdd(&h.y[c].y, h.eta * (gi.y / wc));
            }
        }
    }
    if (h.cmap) {
        // the window's records follow their level nodes as they stand now
        __syncthreads();
        __threadfence();
        for (int32_t i = r0 + (int32_t)threadIdx.x; i < r1; i += STREAM_BLOCK) {
            const float4 ri = h.rec[i];
            const float2 p = h.y[h.cmap[i]];
            h.rec[i] = make_float4(p.x, p.y, ri.z, ri.w);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) h.wcnt[win] = 0u;  // ready for the next launch
}

template <int B, int NH, int F>
__global__ __launch_bounds__(STREAM_BLOCK) void k_sweep_blocked_async(BlockedArgs a, AsyncArgs h) {
    extern __shared__ float4 s_dyn[];
    __shared__ int32_t s_fin[2];
    const int4 it = a.items[h.order[blockIdx.x]];
    blk_layout_item<B, NH, F>(a, s_dyn, it.x, it.y, it.z);
    __syncthreads();
    if (threadIdx.x == 0) {
        s_fin[0] = -1;
        s_fin[1] = -1;
        if (it.z > it.y) {
            __threadfence();  // release this item's partials
            const int32_t w0 = it.y / ASYNC_WIN, w1 = (it.z - 1) / ASYNC_WIN;
            for (int32_t w = w0; w <= w1; ++w)
                if (atomicAdd(&h.wcnt[w], 1u) + 1u == h.wneed[w]) s_fin[w - w0] = w;
        }
    }
    __syncthreads();
    for (int q = 0; q < 2; ++q)
        if (s_fin[q] >= 0) blk_async_window<B>(a, h, s_fin[q]);
}

// ------------------------------------------------------------------ host
static int env_int(const char* name, int dflt) {
    const char* v = std::getenv(name);
    return v && *v ? std::atoi(v) : dflt;
}

static int block_bits() { return std::min(13, std::max(6, env_int("DRG_BLOCK_BITS", 13))); }

bool blocked_wanted_for(drg_ctx* ctx, int32_t n, int64_t nnz) {
    const int force = env_int("DRG_SWEEP_BLOCKED", -1);  // 1 force on, 0 force off
    if (force == 0) return false;
    const int bits = block_bits();
    if (blk_lds_bytes(bits) > (size_t)ctx->max_lds) return false;
    if (force == 1) return nnz > 0;
    const int64_t nb = ((int64_t)n + (1 << bits) - 1) >> bits;
    // records of at least half an L2 slice or a pattern of 2^22 entries
    // (env DRG_BLK_MIN_BITS), and rows long enough to amortise the
    // per-block partials
    const int64_t min_nnz = (int64_t)1 << env_int("DRG_BLK_MIN_BITS", 22);
    const bool big = (int64_t)n * 16 >= ((int64_t)2 << 20) || nnz >= min_nnz;
    return big && nnz > 32 * nb * (int64_t)n;
}

bool blocked_wanted(drg_ctx* ctx, const drg_sim* s) { return blocked_wanted_for(ctx, s->n, s->nnz); }

void build_blocked_core(drg_ctx* ctx, int32_t n, int64_t nnz, const int64_t* prp,
                        const uint32_t* colhop, int32_t col_base, BlkLayout& L) {
    hipStream_t st = ctx->stream;
    const int bits = block_bits();
    const int32_t nb = (int32_t)(((int64_t)n + (1 << bits) - 1) >> bits);
    if ((int64_t)n * nb >= ((int64_t)1 << 40)) throw Error(DRG_E_UNSUPPORTED, "too many blocks");
    DevBuf<int32_t> cnt((int64_t)n * nb);
    hipLaunchKernelGGL(k_blk_count, dim3(ceil_div((int64_t)n * nb, 256)), dim3(256), 0, st, n, nb,
                       bits, prp, colhop, (uint32_t)col_base, cnt.get());
    DRG_LAUNCH_CHECK();
    // per-block entry counts must fit 32-bit offsets
    DevBuf<int64_t> flat((int64_t)n * nb + 1);
    {
        DevBuf<int64_t> cnt64((int64_t)n * nb);
        hipLaunchKernelGGL(k_widen, dim3(ceil_div((int64_t)n * nb, 256)), dim3(256), 0, st,
                           (int64_t)n * nb, cnt.get(), cnt64.get());
        DRG_LAUNCH_CHECK();
        exclusive_scan<int64_t>(cnt64.get(), flat.get(), (int64_t)n * nb, st);
    }
    cnt.reset();
    L.base.alloc(nb + 1);
    L.off.alloc((int64_t)(n + 1) * nb);
    hipLaunchKernelGGL(k_blk_offsets, dim3(ceil_div((int64_t)(n + 1) * nb, 256)), dim3(256), 0, st,
                       n, nb, flat.get(), L.base.get(), L.off.get());
    DRG_LAUNCH_CHECK();
    std::vector<int64_t> base(nb + 1);
    DRG_HIP(hipMemcpyAsync(base.data(), L.base.get(), sizeof(int64_t) * (nb + 1),
                           hipMemcpyDeviceToHost, st));
    DRG_HIP(hipStreamSynchronize(st));
    flat.reset();
    for (int32_t b = 0; b < nb; ++b)
        if (base[b + 1] - base[b] >= ((int64_t)1 << 31))
            throw Error(DRG_E_UNSUPPORTED, "column block too large for 32-bit offsets");
    L.ent.alloc(nnz + 8);  // 16-byte chunk reads may run 7 entries past the end
    DRG_HIP(hipMemsetAsync(L.ent.get(), 0, sizeof(uint16_t) * (nnz + 8), st));
    hipLaunchKernelGGL(k_blk_fill, dim3(ceil_div((int64_t)n * WAVE, 256)), dim3(256), 0, st, n,
                       nb, bits, prp, colhop, (uint32_t)col_base, L.base.get(), L.off.get(),
                       L.ent.get());
    DRG_LAUNCH_CHECK();
    // work items: about `chunk` units of work each (entries + rc per row),
    // at most ROWCAP rows each: at least 2^18 entries (env
    // DRG_BLK_CHUNK_BITS), which keeps the per-item setup small against the
    // sweep; a large pattern gets items of 1/16 of a CU's share.  The rule
    // depends only on the graph, so a graph gets the same items alone and
    // in a batch.  (Smaller items would let a small graph alone use more of
    // the device, at the cost of batches of such graphs.)
    const int64_t floor_chunk = (int64_t)1 << std::min(24, std::max(10, env_int("DRG_BLK_CHUNK_BITS", 18)));
    const int64_t want_items = std::max<int64_t>((int64_t)ctx->num_cu * 16, nb);
    const int64_t chunk = std::max<int64_t>(floor_chunk, (nnz + 16 * (int64_t)n * nb) / want_items);
    const int64_t rc = std::max<int64_t>(16, (chunk + ROWCAP - 1) / ROWCAP);
    std::vector<int32_t> first(nb + 1);
    first[0] = 0;
    for (int32_t b = 0; b < nb; ++b) {
        const int64_t cost = (base[b + 1] - base[b]) + rc * (int64_t)n;
        first[b + 1] = first[b] + (int32_t)std::max<int64_t>(1, (cost + chunk - 1) / chunk);
    }
    DevBuf<int32_t> dfirst(nb + 1);
    DRG_HIP(hipMemcpyAsync(dfirst.get(), first.data(), sizeof(int32_t) * (nb + 1),
                           hipMemcpyHostToDevice, st));
    L.items.alloc(first[nb]);
    int32_t maxcnt = 0;
    for (int32_t b = 0; b < nb; ++b) maxcnt = std::max(maxcnt, first[b + 1] - first[b]);
    hipLaunchKernelGGL(k_blk_items, dim3(ceil_div(maxcnt, 64), nb), dim3(64), 0, st, n, nb,
                       L.off.get(), dfirst.get(), chunk, rc, L.items.get());
    DRG_LAUNCH_CHECK();
    {
        std::vector<int4> hitems(first[nb]);
        DRG_HIP(hipMemcpyAsync(hitems.data(), L.items.get(), sizeof(int4) * first[nb],
                               hipMemcpyDeviceToHost, st));
        DRG_HIP(hipStreamSynchronize(st));
        for (const int4& it : hitems)
            if (it.z - it.y > ROWCAP || it.y < 0 || it.z > n || it.z < it.y)
                throw Error(DRG_E_DEVICE, "blocked sweep: work item outside its row window");
    }
    L.partial.alloc((int64_t)n * nb);
    // the flat sweep writes only rows with entries in a block; the others stay 0
    DRG_HIP(hipMemsetAsync(L.partial.get(), 0, sizeof(float2) * (int64_t)n * nb, st));
    L.nb = nb;
    L.bits = bits;
    L.nitems = first[nb];
    L.chunk = chunk;
    DRG_HIP(hipStreamSynchronize(st));
}

void build_blocked(drg_ctx* ctx, drg_sim* s) {
    BlkLayout L;
    build_blocked_core(ctx, s->n, s->nnz, s->row_ptr.get(), s->colhop.get(), 0, L);
    s->blk_base = std::move(L.base);
    s->blk_off = std::move(L.off);
    s->blk_ent = std::move(L.ent);
    s->blk_items = std::move(L.items);
    s->blk_partial = std::move(L.partial);
    s->blk_nb = L.nb;
    s->blk_bits = L.bits;
    s->blk_nitems = L.nitems;
}

int blk_lanes() {
    const int l = env_int("DRG_BLK_LANES", 0);  // force 16, 32 or 64 lanes per segment
    return (l == 16 || l == 32 || l == 64) ? l : 0;
}

int blk_flat_cpl() {
    const int f = env_int("DRG_BLK_FLAT", 4);
    return (f == 2 || f == 4) ? f : 0;
}

// True when the per-pair clip of the attraction can never bind: for an
// offset of length d the clipped quantity is at most
// 2b d^{2b-1} / (1 + d^{2b}) in magnitude, whose maximum over d (at
// d^{2b} = 2b - 1) is (2b-1)^{(2b-1)/(2b)}.  A 1% margin covers the
// rounding of the coefficient and of d^2.
bool attract_clip_free(int b, double clip) {
    const double m = std::pow(2.0 * b - 1.0, (2.0 * b - 1.0) / (2.0 * b));
    return clip >= 1.01 * m;
}

template <int B, int NH>
static void launch_blocked_b(drg_ctx* ctx, const BlockedArgs& a, int nitems) {
    const size_t lds = blk_lds_bytes(a.bits);
    const int form = blk_form(a.flat);
    auto fn = form == 4   ? k_sweep_blocked<B, NH, 4>
              : form == 2 ? k_sweep_blocked<B, NH, 2>
                          : k_sweep_blocked<B, NH, 0>;
    DRG_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds));
    hipLaunchKernelGGL(fn, dim3(nitems), dim3(STREAM_BLOCK), lds, ctx->stream, a);
    DRG_LAUNCH_CHECK();
}

template <int B, int NH, int KIND>
static void launch_obj_blocked(drg_ctx* ctx, const BlockedArgs& a, int nitems) {
    const size_t lds = blk_lds_bytes(a.bits);
    auto fn = k_obj_blocked<B, NH, KIND>;
    DRG_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds));
    hipLaunchKernelGGL(fn, dim3(nitems), dim3(STREAM_BLOCK), lds, ctx->stream, a);
    DRG_LAUNCH_CHECK();
}

void sweep_blocked_objective(drg_ctx* ctx, drg_sim* s, int b, const float* y, int kind) {
    hipLaunchKernelGGL(k_stage_y, dim3(ceil_div(s->n, 256)), dim3(256), 0, ctx->stream, s->n,
                       reinterpret_cast<const float2*>(y), s->invZf.get(), s->rec.get());
    DRG_LAUNCH_CHECK();
    BlockedArgs a{};
    a.n0 = s->n;
    a.bits = s->blk_bits;
    a.items = s->blk_items.get();
    a.ent = s->blk_ent.get();
    a.base = s->blk_base.get();
    a.off = s->blk_off.get();
    a.rec = s->rec.get();
    a.partial = s->blk_partial.get();
    a.eh0 = (float)(0.5 * s->e[0]);
    a.eh1 = (float)(0.5 * s->e[1]);
    a.eh2 = (float)(0.5 * s->e[2]);
    a.eh3 = (float)(0.5 * s->e[3]);
    const int nh = s->k == 1 ? 1 : (s->k == 2 ? 2 : 4);
#define DRG_OBJ(BB, NN)                                                                  \
    if (b == BB && nh == NN) {                                                           \
        if (kind == 0) launch_obj_blocked<BB, NN, 0>(ctx, a, s->blk_nitems);             \
        else launch_obj_blocked<BB, NN, 1>(ctx, a, s->blk_nitems);                       \
        return;                                                                          \
    }
    DRG_OBJ(1, 1) DRG_OBJ(1, 2) DRG_OBJ(1, 4)
    DRG_OBJ(2, 1) DRG_OBJ(2, 2) DRG_OBJ(2, 4)
    DRG_OBJ(3, 1) DRG_OBJ(3, 2) DRG_OBJ(3, 4)
#undef DRG_OBJ
    throw Error(DRG_E_INVALID, "objective: b in 1..3");
}

// Launch order and window counts of the Hogwild form, built on first use:
// items sorted by (window of their first row, block, first row).
static void build_async_order(drg_ctx* ctx, drg_sim* s) {
    std::vector<int4> items(s->blk_nitems);
    DRG_HIP(hipMemcpyAsync(items.data(), s->blk_items.get(), sizeof(int4) * items.size(),
                           hipMemcpyDeviceToHost, ctx->stream));
    DRG_HIP(hipStreamSynchronize(ctx->stream));
    const int32_t nwin = ceil_div(s->n, ASYNC_WIN);
    std::vector<int32_t> order(items.size());
    for (size_t t = 0; t < order.size(); ++t) order[t] = (int32_t)t;
    auto win_of = [&](const int4& it) { return it.y / ASYNC_WIN; };
    std::stable_sort(order.begin(), order.end(), [&](int32_t p, int32_t q) {
        const int4 &A = items[p], &Bq = items[q];
        if (win_of(A) != win_of(Bq)) return win_of(A) < win_of(Bq);
        if (A.x != Bq.x) return A.x < Bq.x;
        return A.y < Bq.y;
    });
    std::vector<uint32_t> need(nwin, 0u);
    for (const int4& it : items) {
        if (it.z <= it.y) continue;
        const int32_t w1 = (it.z - 1) / ASYNC_WIN;
        if (w1 - it.y / ASYNC_WIN > 1) throw Error(DRG_E_DEVICE, "async sweep: item spans > 2 windows");
        for (int32_t w = it.y / ASYNC_WIN; w <= w1; ++w) ++need[w];
    }
    s->blk_async_order.alloc((int64_t)order.size());
    s->blk_wneed.alloc(nwin);
    s->blk_wcnt.alloc(nwin);
    DRG_HIP(hipMemcpyAsync(s->blk_async_order.get(), order.data(), sizeof(int32_t) * order.size(),
                           hipMemcpyHostToDevice, ctx->stream));
    DRG_HIP(hipMemcpyAsync(s->blk_wneed.get(), need.data(), sizeof(uint32_t) * nwin,
                           hipMemcpyHostToDevice, ctx->stream));
    DRG_HIP(hipMemsetAsync(s->blk_wcnt.get(), 0, sizeof(uint32_t) * nwin, ctx->stream));
    DRG_HIP(hipStreamSynchronize(ctx->stream));
    s->blk_nwin = nwin;
}

template <int B, int NH>
static void launch_blocked_async_b(drg_ctx* ctx, const BlockedArgs& a, const AsyncArgs& h,
                                   int nitems) {
    const size_t lds = blk_lds_bytes(a.bits);
    const int form = blk_form(a.flat);
    auto fn = form == 4   ? k_sweep_blocked_async<B, NH, 4>
              : form == 2 ? k_sweep_blocked_async<B, NH, 2>
                          : k_sweep_blocked_async<B, NH, 0>;
    DRG_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds));
    hipLaunchKernelGGL(fn, dim3(nitems), dim3(STREAM_BLOCK), lds, ctx->stream, a, h);
    DRG_LAUNCH_CHECK();
}

// The sweep and finish of one synchronous FP32 iteration on the blocked
// layout.  `g` non-null: write the steps (coarse level); else update y.
static BlockedArgs layout_args(drg_sim* s, int b, float clip) {
    BlockedArgs a{};
    a.n0 = s->n;
    a.bits = s->blk_bits;
    a.items = s->blk_items.get();
    a.ent = s->blk_ent.get();
    a.base = s->blk_base.get();
    a.off = s->blk_off.get();
    a.rec = s->rec.get();
    a.partial = s->blk_partial.get();
    a.eh0 = (float)(-b * s->e[0]);
    a.eh1 = (float)(-b * s->e[1]);
    a.eh2 = (float)(-b * s->e[2]);
    a.eh3 = (float)(-b * s->e[3]);
    a.clip = clip / (float)(2 * b);
    a.noclip = attract_clip_free(b, clip) ? 1 : 0;
    a.lanes = blk_lanes();
    a.flat = blk_flat_cpl();
    return a;
}

// One Hogwild iteration on the blocked layout (records already staged from
// y): the sweep finishes every window in place, no further launch.
void sweep_blocked_async(drg_ctx* ctx, drg_sim* s, int b, int M, float gamma, float clip,
                         float eta, uint64_t seed, uint64_t iter, float* y, const int32_t* cmap,
                         const float* w, hipEvent_t e0, hipEvent_t e1) {
    if (s->blk_nwin == 0) build_async_order(ctx, s);
    const BlockedArgs a = layout_args(s, b, clip);
    AsyncArgs h{};
    h.order = s->blk_async_order.get();
    h.wcnt = s->blk_wcnt.get();
    h.wneed = s->blk_wneed.get();
    h.nb = s->blk_nb;
    h.M = s->S > 0 ? M : 0;
    h.prp = s->row_ptr.get();
    h.rec = s->rec.get();
    h.qt = s->qtf.get();
    h.C = s->C.get();
    h.guide = s->guide.get();
    h.gbits = s->gbits;
    h.S = s->S;
    h.gamma = gamma;
    h.clip = clip;
    h.eta = eta;
    h.seed = seed;
    h.iter = iter;
    h.y = reinterpret_cast<float2*>(y);
    h.cmap = cmap;
    h.w = w;
    if (e0) DRG_HIP(hipEventRecord(e0, ctx->stream));
#define DRG_BLKA(BB)                                                                   \
    case BB:                                                                           \
        if (s->k == 1) launch_blocked_async_b<BB, 1>(ctx, a, h, s->blk_nitems);        \
        else if (s->k == 2) launch_blocked_async_b<BB, 2>(ctx, a, h, s->blk_nitems);   \
        else launch_blocked_async_b<BB, 4>(ctx, a, h, s->blk_nitems);                  \
        break;
    switch (b) {
        DRG_BLKA(1)
        DRG_BLKA(2)
        default:
        DRG_BLKA(3)
    }
#undef DRG_BLKA
    if (e1) DRG_HIP(hipEventRecord(e1, ctx->stream));
}

void sweep_blocked(drg_ctx* ctx, drg_sim* s, int b, int M, float gamma, float clip,
                   uint64_t seed, uint64_t iter, float2* g, hipEvent_t e0, hipEvent_t e1) {
    const BlockedArgs a = layout_args(s, b, clip);
    if (e0) DRG_HIP(hipEventRecord(e0, ctx->stream));
#define DRG_BLK(BB)                                                                \
    case BB:                                                                       \
        if (s->k == 1) launch_blocked_b<BB, 1>(ctx, a, s->blk_nitems);             \
        else if (s->k == 2) launch_blocked_b<BB, 2>(ctx, a, s->blk_nitems);        \
        else launch_blocked_b<BB, 4>(ctx, a, s->blk_nitems);                       \
        break;
    switch (b) {
        DRG_BLK(1)
        DRG_BLK(2)
        default:
        DRG_BLK(3)
    }
#undef DRG_BLK
    if (e1) DRG_HIP(hipEventRecord(e1, ctx->stream));
    FinishArgs f{};
    f.n0 = s->n;
    f.nb = s->blk_nb;
    f.M = s->S > 0 ? M : 0;
    f.prp = s->row_ptr.get();
    f.partial = s->blk_partial.get();
    f.rec = s->rec.get();
    f.qt = s->qtf.get();
    f.C = s->C.get();
    f.guide = s->guide.get();
    f.gbits = s->gbits;
    f.S = s->S;
    f.gamma = gamma;
    f.clip = clip;
    f.seed = seed;
    f.iter = iter;
    f.g = g;
    switch (b) {
        case 1: hipLaunchKernelGGL(k_finish<1>, dim3(ceil_div(s->n, 256)), dim3(256), 0, ctx->stream, f); break;
        case 2: hipLaunchKernelGGL(k_finish<2>, dim3(ceil_div(s->n, 256)), dim3(256), 0, ctx->stream, f); break;
        default: hipLaunchKernelGGL(k_finish<3>, dim3(ceil_div(s->n, 256)), dim3(256), 0, ctx->stream, f); break;
    }
    DRG_LAUNCH_CHECK();
}

}  // namespace drg
