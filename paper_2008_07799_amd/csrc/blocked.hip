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

// ------------------------------------------------------------------ asynchronous form
// Asynchronous iteration on the blocked layout.  The rows are cut into
// ASYNC_STAGES equal ranges; the work items run stage by stage (an item
// belongs to the stage of its first row), and after the items of stage s
// the rows of stage s are finished and moved at once: their partials are
// complete (every item that holds part of them belongs to stage s or an
// earlier one), the negatives are gathered from the live records, and the
// new positions go straight into the coordinates and into the records that
// the following stages stage into LDS.  Later stages therefore see the
// moves of earlier ones within the same iteration, and the rows finished
// together read and write each other's records without order (Hogwild).
// Finishing per work item instead needs a device-wide cache write-back
// and invalidate per item to pass partials between XCDs, which cost more
// than half an iteration on R-MAT 2^20.
struct FinishInPlaceArgs {
    FinishArgs f;
    int32_t r0, r1;            // rows of the stage
    float4* rec;               // live records (x, y, 1/Z, 1/Z low part)
    float2* y;                 // level coordinates, updated in place
    const int32_t* cmap;       // finest node -> level node (NULL at level 0)
    const float* w;            // anchor weight of each level node
    float eta;
};

template <int B>
__global__ __launch_bounds__(256) void k_finish_inplace(FinishInPlaceArgs a) {
    const int64_t i = (int64_t)a.r0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.r1 || a.f.prp[i + 1] == a.f.prp[i]) return;  // isolated: never moves
    const FinishArgs& f = a.f;
    const float4 ri = a.rec[i];
    const float2 gi =
        blk_finish_row<B>(f.partial, f.nb, f.n0, (int32_t)i, a.rec, ri, f.M, f.seed, f.iter,
                          (int32_t)i,
                          [&](uint64_t w) { return draw_node(w, f.C, f.guide, f.gbits, f.S); },
                          f.gamma * f.qt[i], f.clip);
    if (!a.cmap) {
        const float wi = f.qt[i];
        const float nx = ri.x + a.eta * (gi.x / wi), ny = ri.y + a.eta * (gi.y / wi);
        a.y[i] = make_float2(nx, ny);
        a.rec[i] = make_float4(nx, ny, ri.z, ri.w);
    } else {
        const int32_t c = a.cmap[i];
        const float wc = a.w[c];
        if (wc > 0.0f) {
            atomicAdd(&a.y[c].x, a.eta * (gi.x / wc));
            atomicAdd(&a.y[c].y, a.eta * (gi.y / wc));
        }
    }
}

// records of every finest node from its level node's current position
__global__ void k_restage_xy(int32_t n0, const int32_t* __restrict__ cmap,
                             const float2* __restrict__ y, float4* __restrict__ rec) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n0) return;
    const float2 p = y[cmap[j]];
    const float4 r = rec[j];
    rec[j] = make_float4(p.x, p.y, r.z, r.w);
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
bool attract_clip_free(double b, double clip) {
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

// Work items of the asynchronous form, built on first use: the items
// sorted by (stage of their first row, block, first row), and where each
// stage's items begin.
static int async_stages() { return std::min(64, std::max(1, env_int("DRG_ASYNC_STAGES", 4))); }

static void build_async_order(drg_ctx* ctx, drg_sim* s) {
    const int S = async_stages();
    std::vector<int4> items(s->blk_nitems);
    DRG_HIP(hipMemcpyAsync(items.data(), s->blk_items.get(), sizeof(int4) * items.size(),
                           hipMemcpyDeviceToHost, ctx->stream));
    DRG_HIP(hipStreamSynchronize(ctx->stream));
    auto stage_of = [&](int32_t row) { return (int32_t)(((int64_t)row * S) / s->n); };
    std::stable_sort(items.begin(), items.end(), [&](const int4& p, const int4& q) {
        const int32_t sp = stage_of(p.y), sq = stage_of(q.y);
        if (sp != sq) return sp < sq;
        if (p.x != q.x) return p.x < q.x;
        return p.y < q.y;
    });
    s->blk_stage_first.assign(S + 1, 0);
    for (const int4& it : items) ++s->blk_stage_first[stage_of(it.y) + 1];
    for (int t = 0; t < S; ++t) s->blk_stage_first[t + 1] += s->blk_stage_first[t];
    s->blk_items_async.alloc((int64_t)items.size());
    DRG_HIP(hipMemcpyAsync(s->blk_items_async.get(), items.data(), sizeof(int4) * items.size(),
                           hipMemcpyHostToDevice, ctx->stream));
    DRG_HIP(hipStreamSynchronize(ctx->stream));
    s->blk_stages = S;
}

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

// One asynchronous iteration on the blocked layout (records already staged
// from y): per stage, the sweep of its work items, then its rows finished
// and moved in place; at a coarse level the records of all finest nodes then
// follow their level nodes.
void sweep_blocked_async(drg_ctx* ctx, drg_sim* s, int b, int M, float gamma, float clip,
                         float eta, uint64_t seed, uint64_t iter, float* y, const int32_t* cmap,
                         const float* w, hipEvent_t e0, hipEvent_t e1) {
    if (s->blk_stages == 0) build_async_order(ctx, s);
    BlockedArgs a = layout_args(s, b, clip);
    FinishInPlaceArgs fa{};
    fa.f.n0 = s->n;
    fa.f.nb = s->blk_nb;
    fa.f.M = s->S > 0 ? M : 0;
    fa.f.prp = s->row_ptr.get();
    fa.f.partial = s->blk_partial.get();
    fa.f.rec = s->rec.get();
    fa.f.qt = s->qtf.get();
    fa.f.C = s->C.get();
    fa.f.guide = s->guide.get();
    fa.f.gbits = s->gbits;
    fa.f.S = s->S;
    fa.f.gamma = gamma;
    fa.f.clip = clip;
    fa.f.seed = seed;
    fa.f.iter = iter;
    fa.rec = s->rec.get();
    fa.y = reinterpret_cast<float2*>(y);
    fa.cmap = cmap;
    fa.w = w;
    fa.eta = eta;
    const int S = s->blk_stages;
    if (e0) DRG_HIP(hipEventRecord(e0, ctx->stream));
    for (int t = 0; t < S; ++t) {
        const int32_t i0 = s->blk_stage_first[t], i1 = s->blk_stage_first[t + 1];
        a.items = s->blk_items_async.get() + i0;
        if (i1 > i0) {
#define DRG_BLK(BB)                                                                    \
    case BB:                                                                           \
        if (s->k == 1) launch_blocked_b<BB, 1>(ctx, a, i1 - i0);                       \
        else if (s->k == 2) launch_blocked_b<BB, 2>(ctx, a, i1 - i0);                  \
        else launch_blocked_b<BB, 4>(ctx, a, i1 - i0);                                 \
        break;
            switch (b) {
                DRG_BLK(1)
                DRG_BLK(2)
                default:
                DRG_BLK(3)
            }
#undef DRG_BLK
        }
        fa.r0 = (int32_t)(((int64_t)t * s->n) / S);
        fa.r1 = (int32_t)(((int64_t)(t + 1) * s->n) / S);
        if (fa.r1 > fa.r0) {
            const dim3 grid(ceil_div(fa.r1 - fa.r0, 256));
            switch (b) {
                case 1: hipLaunchKernelGGL(k_finish_inplace<1>, grid, dim3(256), 0, ctx->stream, fa); break;
                case 2: hipLaunchKernelGGL(k_finish_inplace<2>, grid, dim3(256), 0, ctx->stream, fa); break;
                default: hipLaunchKernelGGL(k_finish_inplace<3>, grid, dim3(256), 0, ctx->stream, fa); break;
            }
            DRG_LAUNCH_CHECK();
        }
        if (cmap && t + 1 < S) {
            hipLaunchKernelGGL(k_restage_xy, dim3(ceil_div(s->n, 256)), dim3(256), 0, ctx->stream,
                               s->n, cmap, fa.y, s->rec.get());
            DRG_LAUNCH_CHECK();
        }
    }
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
