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
#include <cstdlib>

#include "drg_internal.hpp"

namespace drg {

constexpr int BLK_HOP_SHIFT = 13;

// cnt[b*n + i] = number of entries of row i whose column lies in block b
__global__ void k_blk_count(int32_t n, int32_t nb, int bits, const int64_t* __restrict__ prp,
                            const uint32_t* __restrict__ ch, int32_t* __restrict__ cnt) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * nb) return;
    const int32_t i = (int32_t)(t % n);
    const int32_t b = (int32_t)(t / n);
    auto lb = [&](int64_t lo, int64_t hi, uint32_t key) {
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if ((ch[mid] & COL_MASK) < key)
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
            ent[dst + x] = (uint16_t)((e & mask) | ((e >> 30) << BLK_HOP_SHIFT));
        }
        s += len;
    }
}

// Work items: block b's rows cut where the running cost (entries + rc per
// row) crosses multiples of `chunk`; rc >= chunk / ROWCAP keeps every item
// within ROWCAP rows.  item_first[b] = index of b's first item.
constexpr int ROWCAP = 4096;

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

struct BlockedArgs {
    int32_t n0;
    int32_t bits;
    const int4* items;
    const uint16_t* ent;
    const int64_t* base;
    const int32_t* off;
    const float4* rec;
    float2* partial;
    float eh0, eh1, eh2, eh3;   // -2b * e_d / 2 per hop
    float clip;                 // clip / (2b)
    int32_t lanes;              // lanes per row segment (16, 32, 64; 0: per item)
    int32_t flat;               // chunks per lane of the flat (merge-path) form; 0: row form
};

template <int B>
__device__ __forceinline__ float blk_attract_coef(float d2) {
    return -2.0f * (float)B * powi<B - 1>(d2) / (1.0f + powi<B>(d2));
}
template <int B>
__device__ __forceinline__ float blk_repel_coef(float d2) {
    return 2.0f * (float)B * rcp_fast(d2 * (1.0f + powi<B>(d2)));
}

// Attraction of one stored pair, scaled by `valid` (0 or 1) so a lane can
// run all eight entries of its chunk without branching.  With the -2b factor
// folded into the weight, -2b clip(p dx, c/(2b)) = clip(-2b p dx, c) because
// the clip is odd.  A zero offset gives a zero force through dx = dy = 0.
struct HopW {  // -2b e_d / 2 per hop, held in vector registers inside the loops
    float e0, e1, e2, e3;
};

__device__ __forceinline__ HopW hop_weights(const BlockedArgs& a) {
    HopW h{a.eh0, a.eh1, a.eh2, a.eh3};
    // vector copies made once: selecting between two scalar operands would
    // otherwise copy both into vector registers at every pair
    asm volatile("" : "+v"(h.e0), "+v"(h.e1), "+v"(h.e2), "+v"(h.e3));
    return h;
}

template <int B, int NH>
__device__ __forceinline__ void blk_pair(const BlockedArgs& a, const HopW& hw, const float4& ri,
                                         const float4* s_rec, uint32_t u, uint32_t lmask,
                                         bool valid, float& ax, float& ay) {
    const float4 rj = s_rec[u & lmask];
    const float dx = ri.x - rj.x, dy = ri.y - rj.y;
    const float d2 = dx * dx + dy * dy;
    float eh;
    if constexpr (NH == 1) {
        eh = hw.e0;
    } else if constexpr (NH == 2) {
        eh = (u >> BLK_HOP_SHIFT) ? hw.e1 : hw.e0;
    } else {
        const uint32_t h = u >> BLK_HOP_SHIFT;
        eh = (h & 2u) ? ((h & 1u) ? hw.e3 : hw.e2) : ((h & 1u) ? hw.e1 : hw.e0);
    }
    const float p = powi<B - 1>(d2) * rcp_fast(1.0f + powi<B>(d2));
    const float w = valid ? eh * (ri.z + rj.z) : 0.0f;
    ax += w * clampf(p * dx, a.clip);
    ay += w * clampf(p * dy, a.clip);
}

// Pair operators of the flat sweep: what one stored pair (record rj, entry u)
// adds to the lane's partial of its row.  `valid` = 0 masks a slot.
template <int NH>
__device__ __forceinline__ float hop_weight(const HopW& hw, uint32_t u) {
    if constexpr (NH == 1) {
        return hw.e0;
    } else if constexpr (NH == 2) {
        return (u >> BLK_HOP_SHIFT) ? hw.e1 : hw.e0;
    } else {
        const uint32_t h = u >> BLK_HOP_SHIFT;
        return (h & 2u) ? ((h & 1u) ? hw.e3 : hw.e2) : ((h & 1u) ? hw.e1 : hw.e0);
    }
}

// the layout step: clipped attraction (weights carry -2b)
template <int B, int NH>
struct LayoutOp {
    const BlockedArgs* a;
    HopW hw;
    __device__ __forceinline__ void operator()(const float4& ri, const float4* s_rec, uint32_t u,
                                               uint32_t lmask, bool valid, float& ax,
                                               float& ay) const {
        blk_pair<B, NH>(*a, hw, ri, s_rec, u, lmask, valid, ax, ay);
    }
};

// the objective: P~_ij log w_ij = -P~_ij log1p(d^{2b}) (weights are e_d / 2)
template <int B, int NH>
struct ObjValOp {
    HopW hw;
    __device__ __forceinline__ void operator()(const float4& ri, const float4* s_rec, uint32_t u,
                                               uint32_t lmask, bool valid, float& ax,
                                               float& ay) const {
        const float4 rj = s_rec[u & lmask];
        const float dx = ri.x - rj.x, dy = ri.y - rj.y;
        const float d2 = dx * dx + dy * dy;
        const float pw = valid ? hop_weight<NH>(hw, u) * (ri.z + rj.z) : 0.0f;
        ax += pw * (-log1pf(powi<B>(d2)));
        (void)ay;
    }
};

// its gradient's attraction (unclipped): P~_ij (-2b d^{2b-2} / (1 + d^{2b})) (y_i - y_j)
template <int B, int NH>
struct ObjGradOp {
    HopW hw;
    __device__ __forceinline__ void operator()(const float4& ri, const float4* s_rec, uint32_t u,
                                               uint32_t lmask, bool valid, float& ax,
                                               float& ay) const {
        const float4 rj = s_rec[u & lmask];
        const float dx = ri.x - rj.x, dy = ri.y - rj.y;
        const float d2 = dx * dx + dy * dy;
        const float pw = valid ? hop_weight<NH>(hw, u) * (ri.z + rj.z) : 0.0f;
        const float k = pw * (float)(-2 * B) * powi<B - 1>(d2) / (1.0f + powi<B>(d2));
        ax += k * dx;
        ay += k * dy;
    }
};

// Workgroups of 1024 threads; an entry chunk is 16 bytes (eight 16-bit words).
constexpr int STREAM_BLOCK = 1024;
constexpr int STREAM_WAVES = STREAM_BLOCK / WAVE;

__device__ __forceinline__ uint32_t half16(const uint4& v, int q) {
    const uint32_t w = q < 2 ? v.x : (q < 4 ? v.y : (q < 6 ? v.z : v.w));
    return (q & 1) ? (w >> 16) : (w & 0xFFFFu);
}

// The rows of an item, S lanes per row segment (64/S rows per wave at a
// time): lane l of a group reads the aligned 16-byte chunk c0 + l of its
// segment, so a group covers 8 S entries per step; short segments use small
// groups so fewer lanes idle.  The first chunk of a group's next row is
// requested before the current row is processed.
template <int B, int NH, int S>
__device__ __forceinline__ void blk_rows(const BlockedArgs& a, const float4* s_rec,
                                         const int32_t* s_off, int32_t b, int32_t r0, int32_t r1) {
    constexpr int R = WAVE / S;
    const int lane = __lane_id();
    const int sl = lane % S, sub = lane / S;
    const int32_t wid = threadIdx.x / WAVE;
    const int64_t bbase = a.base[b];
    const uint4* E4 = reinterpret_cast<const uint4*>(a.ent);
    float2* P = a.partial + (int64_t)b * a.n0;
    const uint32_t lmask = (1u << a.bits) - 1u;
    const HopW hw = hop_weights(a);
    // chunk of row r for this lane (first window), zero when outside
    auto fetch = [&](int32_t r, int64_t& As, int64_t& Ae, uint4& v) {
        As = bbase + s_off[r - r0];
        Ae = bbase + s_off[r - r0 + 1];
        const int64_t c = (As >> 3) + sl;
        v = (As < Ae && c * 8 < Ae) ? E4[c] : make_uint4(0, 0, 0, 0);
    };
    const int32_t rstep = STREAM_WAVES * R;
    int32_t r = r0 + wid * R + sub;
    int64_t As = 0, Ae = 0;
    uint4 v = make_uint4(0, 0, 0, 0);
    if (r < r1) fetch(r, As, Ae, v);
    for (; r < r1; r += rstep) {
        // request the next row's first chunk now
        const int32_t rn = r + rstep;
        int64_t Asn = 0, Aen = 0;
        uint4 vn = make_uint4(0, 0, 0, 0);
        if (rn < r1) fetch(rn, Asn, Aen, vn);
        float ax = 0.0f, ay = 0.0f;
        if (As < Ae) {
            const float4 ri = a.rec[r];
            const int32_t len = (int32_t)(Ae - As);
            // rel: position of this lane's chunk start relative to the segment
            int32_t rel = (int32_t)(((As >> 3) << 3) - As) + 8 * sl;
            uint4 cur = v;
            while (true) {
                // the next window's chunk is requested before this one is used
                const int32_t reln = rel + 8 * S;
                const bool more = reln - 8 * sl < len;  // group-uniform
                const uint4 nxt = (more && reln < len) ? E4[((As + reln) >> 3)]
                                                       : make_uint4(0, 0, 0, 0);
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const bool valid = (uint32_t)(rel + q) < (uint32_t)len;
                    blk_pair<B, NH>(a, hw, ri, s_rec, half16(cur, q), lmask, valid, ax, ay);
                }
                if (!more) break;
                rel = reln;
                cur = nxt;
            }
            ax = group_sum<S>(ax);
            ay = group_sum<S>(ay);
        }
        if (sl == 0) P[r] = make_float2(ax, ay);
        As = Asn;
        Ae = Aen;
        v = vn;
    }
}

// ------------------------------------------------------------------ flat form
// The entries of an item (rows r0..r1 of block b) are contiguous, so the
// item is swept as one stream regardless of row boundaries: wave w takes a
// contiguous range of its 16-byte chunks, lane l the chunk w0 + l of each
// 64-chunk window; every lane walks its 8 entries, tracking the row through
// the LDS row offsets.  A row that starts and ends inside one lane is
// complete there.  A row that crosses lanes is summed by a keyed segmented
// scan over the lanes' last-row partials (in lane order), a row that crosses
// windows is carried by the wave, and a row that crosses waves is closed by
// one thread after the workgroup barrier, in wave order.  All of it depends
// only on the layout of the data, so the result is repeatable.
struct WaveFrag {
    int32_t hrow, trow, same, pad;  // open head row, open tail row (-1: none)
    float hx, hy, tx, ty;
};

// largest i in [lo, hi] with off[i] <= p
__device__ __forceinline__ int32_t row_of(const int32_t* off, int32_t lo, int32_t hi, int32_t p) {
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (off[mid] <= p)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// largest i in [lo, hi] with off[i] <= p, given off[lo] <= p: doubling steps
// from lo, then bisection (cheap when the answer is near lo)
__device__ __forceinline__ int32_t row_from(const int32_t* off, int32_t lo, int32_t hi, int32_t p) {
    int32_t step = 1;
    while (lo + step <= hi && off[lo + step] <= p) {
        lo += step;
        step <<= 1;
    }
    return row_of(off, lo, min(lo + step - 1, hi), p);
}

template <int CPL, typename Op>
__device__ __forceinline__ void blk_flat(const BlockedArgs& a, const Op& op, const float4* s_rec,
                                         const int32_t* s_off, WaveFrag* s_frag, int32_t b,
                                         int32_t r0, int32_t r1) {
    constexpr int EPL = 8 * CPL;          // entries per lane per window
    constexpr int WCH = WAVE * CPL;       // chunks per window
    const int lane = __lane_id();
    const int wid = threadIdx.x / WAVE;
    const int32_t nr = r1 - r0;
    const int64_t bbase = a.base[b];
    const int32_t e0 = s_off[0], e1 = s_off[nr];
    float2* P = a.partial + (int64_t)b * a.n0 + r0;
    const float4* R = a.rec + r0;
    const uint4* E4 = reinterpret_cast<const uint4*>(a.ent);
    const uint32_t lmask = (1u << a.bits) - 1u;
    const int64_t cA = (bbase + e0) >> 3;
    const int64_t nch = e1 > e0 ? ((bbase + e1 + 7) >> 3) - cA : 0;
    const int64_t per = (nch + STREAM_WAVES - 1) / STREAM_WAVES;
    const int64_t wc0 = cA + min(nch, per * wid), wc1 = cA + min(nch, per * (wid + 1));
    // the wave's first row and whether it started before the wave's range
    int32_t w_first = -1;
    bool w_open = false;
    if (wc0 < wc1) {
        const int32_t fp = max((int32_t)(8 * wc0 - bbase), e0);
        w_first = row_of(s_off, 0, nr - 1, fp);
        w_open = s_off[w_first] < fp;
    }
    if (lane == 0) {
        s_frag[wid].hrow = -1;
        s_frag[wid].trow = -1;
        s_frag[wid].same = 0;
    }
    // a complete row: written, unless it is the wave's open first row
    auto close_row = [&](int32_t row, float x, float y) {
        if (row == w_first && w_open) {
            s_frag[wid].hrow = row;
            s_frag[wid].hx = x;
            s_frag[wid].hy = y;
        } else {
            P[row] = make_float2(x, y);
        }
    };
    int32_t c_row = -1;  // row carried from the previous window (wave-uniform)
    float c_x = 0.0f, c_y = 0.0f;
    int32_t ilo = max(w_first, 0);
    // chunk loads are unconditional, clamped to the wave's last chunk (slots
    // past the range are masked), so the counters of outstanding loads stay
    // exact and a wait for one load does not drain the prefetches
    const int64_t clast = max(wc1 - 1, wc0);
    uint4 vn[CPL];
#pragma unroll
    for (int k = 0; k < CPL; ++k) vn[k] = E4[min(wc0 + (int64_t)lane * CPL + k, clast)];
    for (int64_t w0 = wc0; w0 < wc1; w0 += WCH) {
        const int64_t c = w0 + (int64_t)lane * CPL;  // the lane's first chunk
        const int32_t nl = (int32_t)min((int64_t)WAVE, (wc1 - w0 + CPL - 1) / CPL);
        const bool has = lane < nl;
        const int32_t pbase = (int32_t)(8 * c - bbase);
        const int32_t pf = max(pbase, e0);                                  // first valid slot
        const int32_t pl = min(min(pbase + EPL, (int32_t)(8 * wc1 - bbase)), e1);  // end of valid slots
        // the same bounds relative to the lane's first slot (none valid without a chunk)
        const int32_t qlo = pf - pbase, qhi = has ? pl - pbase : 0;
        // rows spanned by the window, then the lane's first row
        const int32_t wp0 = max((int32_t)(8 * w0 - bbase), e0);
        const int32_t wp1 = min((int32_t)(8 * min(w0 + WCH, wc1) - bbase), e1) - 1;
        const int32_t i0 = row_from(s_off, ilo, nr - 1, wp0);
        const int32_t i1 = row_from(s_off, i0, nr - 1, wp1);
        int32_t i = has ? row_of(s_off, i0, i1, pf) : i1;
        int32_t nxt = s_off[i + 1];
        // the row record is requested before the next window's chunks, so
        // waiting for it does not wait for them
        float4 ri = R[i];
        uint4 v[CPL];
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            v[k] = vn[k];
            vn[k] = E4[min(c + WCH + k, clast)];
        }
        float ax = 0.0f, ay = 0.0f, hx = 0.0f, hy = 0.0f;
        const int32_t hrow = i;
        bool hopen = true;  // still on the lane's first row
        int32_t qn = nxt - pbase;  // slot where the current row ends
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                constexpr int32_t Q0 = 0;
                const int32_t Q = Q0 + 8 * k + q;
                const bool valid = Q >= qlo && Q < qhi;
                if (valid && Q >= qn) {  // the row ends before this slot
                    const int32_t p = pbase + Q;
                    if (hopen) {
                        hx = ax;
                        hy = ay;
                        hopen = false;
                    } else {
                        close_row(i, ax, ay);  // started and ended inside this lane
                    }
                    do {
                        ++i;
                        nxt = s_off[i + 1];
                    } while (p >= nxt);
                    qn = nxt - pbase;
                    float4 rt = R[i];
                    // keeps the reload on this (rare) path: otherwise the load is
                    // moved past the branch and every entry waits for it
                    asm volatile("" : "+v"(rt.x), "+v"(rt.y), "+v"(rt.z));
                    ri = rt;
                    ax = 0.0f;
                    ay = 0.0f;
                }
                op(ri, s_rec, half16(v[k], q), lmask, valid, ax, ay);
            }
        }
        // the window's carried row continues into lane 0
        if (lane == 0 && hrow == c_row) {
            if (hopen) {
                ax = c_x + ax;
                ay = c_y + ay;
            } else {
                hx = c_x + hx;
                hy = c_y + hy;
            }
        }
        // keyed inclusive scan of the lanes' last-row partials
        const int32_t tk = has ? i : -2 - lane;
        float sx = ax, sy = ay;
#pragma unroll
        for (int d = 1; d < WAVE; d <<= 1) {
            const float ox = __shfl_up(sx, d), oy = __shfl_up(sy, d);
            const int32_t ok = __shfl_up(tk, d);
            if (lane >= d && ok == tk) {
                sx = ox + sx;
                sy = oy + sy;
            }
        }
        // a first row that ended inside the lane: add what earlier lanes hold
        const float px = __shfl_up(sx, 1), py = __shfl_up(sy, 1);
        const int32_t pk = __shfl_up(tk, 1);
        if (has && !hopen) {
            const bool cin = lane > 0 && pk == hrow;
            close_row(hrow, cin ? px + hx : hx, cin ? py + hy : hy);
        }
        // the last row: complete unless it goes on past this lane (into the
        // next lane, the next window or the next wave)
        const bool cont = has && nxt > pl;
        if (has && !cont) close_row(i, sx, sy);
        // carry of the window's last lane
        const int32_t L = nl - 1;
        const bool lcont = __shfl(cont ? 1 : 0, L) != 0;
        const int32_t lrow = __shfl(i, L);
        const float lx = __shfl(sx, L), ly = __shfl(sy, L);
        c_row = lcont ? lrow : -1;
        c_x = lcont ? lx : 0.0f;
        c_y = lcont ? ly : 0.0f;
        ilo = i1;
    }
    // the wave's open tail (its last row goes on into the next wave)
    if (c_row >= 0 && lane == 0) {
        s_frag[wid].trow = c_row;
        s_frag[wid].tx = c_x;
        s_frag[wid].ty = c_y;
        s_frag[wid].same = (c_row == w_first && w_open) ? 1 : 0;
    }
    __syncthreads();
    // rows across waves, in wave order: an open tail runs on through waves
    // that lie inside it and is closed by the next wave's open head
    if (threadIdx.x == 0) {
        float x = 0.0f, y = 0.0f;
        for (int w = 0; w < STREAM_WAVES; ++w) {
            const WaveFrag f = s_frag[w];
            if (f.same) {
                x = x + f.tx;
                y = y + f.ty;
                continue;
            }
            if (f.hrow >= 0) P[f.hrow] = make_float2(x + f.hx, y + f.hy);
            x = f.trow >= 0 ? f.tx : 0.0f;
            y = f.trow >= 0 ? f.ty : 0.0f;
        }
    }
}

// One workgroup per item (block b, rows r0..r1): the block's records and the
// item's row offsets go to LDS, then the rows are swept with the lanes per
// segment that suit the item's mean segment length.  Lane sums run in a
// fixed order and the group reductions are fixed, so the result is
// repeatable.
// Stages block b's records and the item's row offsets into LDS.
__device__ __forceinline__ void blk_stage(const BlockedArgs& a, float4* s_rec, int32_t* s_off,
                                          int32_t b, int32_t r0, int32_t r1) {
    const int32_t bw = 1 << a.bits;
    const int32_t j0 = b * bw;
    const int32_t cnt = min(bw, a.n0 - j0);
    const int32_t* O = a.off + (int64_t)b * (a.n0 + 1);
    for (int32_t t = threadIdx.x; t < bw; t += STREAM_BLOCK)
        s_rec[t] = t < cnt ? a.rec[j0 + t] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    for (int32_t t = threadIdx.x; t <= r1 - r0; t += STREAM_BLOCK) s_off[t] = O[r0 + t];
    __syncthreads();
}

template <int B, int NH>
__global__ __launch_bounds__(STREAM_BLOCK) void k_sweep_blocked(BlockedArgs a) {
    extern __shared__ float4 s_dyn[];
    const int32_t bw = 1 << a.bits;
    float4* s_rec = s_dyn;
    int32_t* s_off = reinterpret_cast<int32_t*>(s_dyn + bw);
    WaveFrag* s_frag = reinterpret_cast<WaveFrag*>(s_dyn + bw + (ROWCAP + 4) / 4);
    const int4 it = a.items[blockIdx.x];
    const int32_t b = it.x, r0 = it.y, r1 = it.z;
    blk_stage(a, s_rec, s_off, b, r0, r1);
    const LayoutOp<B, NH> op{&a, hop_weights(a)};
    if (a.flat == 1) {
        blk_flat<1>(a, op, s_rec, s_off, s_frag, b, r0, r1);
        return;
    }
    if (a.flat == 2) {
        blk_flat<2>(a, op, s_rec, s_off, s_frag, b, r0, r1);
        return;
    }
    if (a.flat == 4) {
        blk_flat<4>(a, op, s_rec, s_off, s_frag, b, r0, r1);
        return;
    }
    if (a.flat == 8) {
        blk_flat<8>(a, op, s_rec, s_off, s_frag, b, r0, r1);
        return;
    }
    int S = a.lanes;
    if (S == 0) {
        const int32_t rows = max(1, r1 - r0);
        const int32_t mean = (s_off[r1 - r0] - s_off[0]) / rows;
        S = mean >= 320 ? 64 : (mean >= 96 ? 32 : 16);
    }
    if (S == 16)
        blk_rows<B, NH, 16>(a, s_rec, s_off, b, r0, r1);
    else if (S == 32)
        blk_rows<B, NH, 32>(a, s_rec, s_off, b, r0, r1);
    else
        blk_rows<B, NH, 64>(a, s_rec, s_off, b, r0, r1);
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
    blk_stage(a, s_rec, s_off, b, r0, r1);
    if constexpr (KIND == 0)
        blk_flat<4>(a, ObjValOp<B, NH>{hop_weights(a)}, s_rec, s_off, s_frag, b, r0, r1);
    else
        blk_flat<4>(a, ObjGradOp<B, NH>{hop_weights(a)}, s_rec, s_off, s_frag, b, r0, r1);
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
    float gamma, clip, eta;
    uint64_t seed, iter;
    float2* g;   // coarse levels: one-sided steps
    float2* y;   // level 0: coordinates, updated in place
};

// One thread per finest node: partials in block order, M negatives, step.
template <int B>
__global__ __launch_bounds__(256) void k_finish(FinishArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n0) return;
    float gx = 0.0f, gy = 0.0f;
    const bool active = a.prp[i + 1] > a.prp[i];
    if (active) {
        float ax = 0.0f, ay = 0.0f;
        for (int32_t b = 0; b < a.nb; ++b) {
            const float2 p = a.partial[(int64_t)b * a.n0 + i];
            ax += p.x;
            ay += p.y;
        }
        const float4 ri = a.rec[i];
        float rx = 0.0f, ry = 0.0f;
        for (int m = 0; m < a.M; ++m) {
            const uint64_t w = neg_word(a.seed, a.iter, (int32_t)i, m);
            const int32_t v = draw_node(w, a.C, a.guide, a.gbits, a.S);
            const float4 rv = a.rec[v];
            const float dx = ri.x - rv.x, dy = ri.y - rv.y;
            const float d2 = dx * dx + dy * dy;
            if (d2 > 0.0f) {
                const float k = blk_repel_coef<B>(d2);
                rx += repel_component(k, dx, a.clip);
                ry += repel_component(k, dy, a.clip);
            }
        }
        const float gq = a.gamma * a.qt[i];
        gx = ax + gq * rx;
        gy = ay + gq * ry;
    }
    if (a.g) {
        a.g[i] = make_float2(gx, gy);
    } else if (active) {
        const float w = a.qt[i];
        float2 p = a.y[i];
        p.x += a.eta * (gx / w);
        p.y += a.eta * (gy / w);
        a.y[i] = p;
    }
}

// ------------------------------------------------------------------ host
static int env_int(const char* name, int dflt) {
    const char* v = std::getenv(name);
    return v && *v ? std::atoi(v) : dflt;
}

bool blocked_wanted(drg_ctx* ctx, const drg_sim* s) {
    const int force = env_int("DRG_SWEEP_BLOCKED", -1);  // 1 force on, 0 force off
    if (force == 0) return false;
    const int bits = std::min(13, std::max(6, env_int("DRG_BLOCK_BITS", 13)));
    if ((int64_t)(16u << bits) + 4 * (ROWCAP + 1) + 1024 > (int64_t)ctx->max_lds) return false;
    if (force == 1) return s->nnz > 0;
    const int64_t nb = ((int64_t)s->n + (1 << bits) - 1) >> bits;
    // records of at least half an L2 slice, and rows long enough to amortise
    // the per-block partials
    return (int64_t)s->n * 16 >= ((int64_t)2 << 20) && s->nnz > 32 * nb * (int64_t)s->n;
}

void build_blocked(drg_ctx* ctx, drg_sim* s) {
    hipStream_t st = ctx->stream;
    const int bits = std::min(13, std::max(6, env_int("DRG_BLOCK_BITS", 13)));
    const int32_t n = s->n;
    const int32_t nb = (int32_t)(((int64_t)n + (1 << bits) - 1) >> bits);
    if ((int64_t)n * nb >= ((int64_t)1 << 40)) throw Error(DRG_E_UNSUPPORTED, "too many blocks");
    DevBuf<int32_t> cnt((int64_t)n * nb);
    hipLaunchKernelGGL(k_blk_count, dim3(ceil_div((int64_t)n * nb, 256)), dim3(256), 0, st, n, nb,
                       bits, s->row_ptr.get(), s->colhop.get(), cnt.get());
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
    s->blk_base.alloc(nb + 1);
    s->blk_off.alloc((int64_t)(n + 1) * nb);
    hipLaunchKernelGGL(k_blk_offsets, dim3(ceil_div((int64_t)(n + 1) * nb, 256)), dim3(256), 0, st,
                       n, nb, flat.get(), s->blk_base.get(), s->blk_off.get());
    DRG_LAUNCH_CHECK();
    std::vector<int64_t> base(nb + 1);
    DRG_HIP(hipMemcpyAsync(base.data(), s->blk_base.get(), sizeof(int64_t) * (nb + 1),
                           hipMemcpyDeviceToHost, st));
    DRG_HIP(hipStreamSynchronize(st));
    flat.reset();
    for (int32_t b = 0; b < nb; ++b)
        if (base[b + 1] - base[b] >= ((int64_t)1 << 31))
            throw Error(DRG_E_UNSUPPORTED, "column block too large for 32-bit offsets");
    s->blk_ent.alloc(s->nnz + 8);  // 16-byte chunk reads may run 7 entries past the end
    DRG_HIP(hipMemsetAsync(s->blk_ent.get(), 0, sizeof(uint16_t) * (s->nnz + 8), st));
    hipLaunchKernelGGL(k_blk_fill, dim3(ceil_div((int64_t)n * WAVE, 256)), dim3(256), 0, st, n,
                       nb, bits, s->row_ptr.get(), s->colhop.get(), s->blk_base.get(),
                       s->blk_off.get(), s->blk_ent.get());
    DRG_LAUNCH_CHECK();
    // work items: about `chunk` units of work each (entries + rc per row),
    // at most ROWCAP rows each
    const int64_t want_items = std::max<int64_t>((int64_t)ctx->num_cu * 16, nb);
    const int64_t chunk =
        std::max<int64_t>(1 << 16, (s->nnz + 16 * (int64_t)n * nb) / want_items);
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
    s->blk_items.alloc(first[nb]);
    int32_t maxcnt = 0;
    for (int32_t b = 0; b < nb; ++b) maxcnt = std::max(maxcnt, first[b + 1] - first[b]);
    hipLaunchKernelGGL(k_blk_items, dim3(ceil_div(maxcnt, 64), nb), dim3(64), 0, st, n, nb,
                       s->blk_off.get(), dfirst.get(), chunk, rc, s->blk_items.get());
    DRG_LAUNCH_CHECK();
    {
        std::vector<int4> hitems(first[nb]);
        DRG_HIP(hipMemcpyAsync(hitems.data(), s->blk_items.get(), sizeof(int4) * first[nb],
                               hipMemcpyDeviceToHost, st));
        DRG_HIP(hipStreamSynchronize(st));
        for (const int4& it : hitems)
            if (it.z - it.y > ROWCAP || it.y < 0 || it.z > n || it.z < it.y)
                throw Error(DRG_E_DEVICE, "blocked sweep: work item outside its row window");
    }
    s->blk_partial.alloc((int64_t)n * nb);
    // the flat sweep writes only rows with entries in a block; the others stay 0
    DRG_HIP(hipMemsetAsync(s->blk_partial.get(), 0, sizeof(float2) * (int64_t)n * nb, st));
    s->blk_nb = nb;
    s->blk_bits = bits;
    s->blk_nitems = first[nb];
    DRG_HIP(hipStreamSynchronize(st));
}

template <int B, int NH>
static void launch_blocked_b(drg_ctx* ctx, const BlockedArgs& a, int nitems) {
    const size_t lds = ((size_t)16 << a.bits) + 16 * ((ROWCAP + 4) / 4) +
                       sizeof(WaveFrag) * STREAM_WAVES;
    auto fn = k_sweep_blocked<B, NH>;
    DRG_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds));
    hipLaunchKernelGGL(fn, dim3(nitems), dim3(STREAM_BLOCK), lds, ctx->stream, a);
    DRG_LAUNCH_CHECK();
}

template <int B, int NH, int KIND>
static void launch_obj_blocked(drg_ctx* ctx, const BlockedArgs& a, int nitems) {
    const size_t lds = ((size_t)16 << a.bits) + 16 * ((ROWCAP + 4) / 4) +
                       sizeof(WaveFrag) * STREAM_WAVES;
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

// The sweep and finish of one synchronous FP32 iteration on the blocked
// layout.  `g` non-null: write the steps (coarse level); else update y.
void sweep_blocked(drg_ctx* ctx, drg_sim* s, int b, int M, float gamma, float clip, float eta,
                   uint64_t seed, uint64_t iter, float2* g, float2* y, hipEvent_t e0,
                   hipEvent_t e1) {
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
    {
        const int l = env_int("DRG_BLK_LANES", 0);  // force 16, 32 or 64 lanes per segment
        a.lanes = (l == 16 || l == 32 || l == 64) ? l : 0;
        const int f = env_int("DRG_BLK_FLAT", 4);
        a.flat = (f == 1 || f == 2 || f == 4 || f == 8) ? f : 0;
    }
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
    f.eta = eta;
    f.seed = seed;
    f.iter = iter;
    f.g = g;
    f.y = y;
    switch (b) {
        case 1: hipLaunchKernelGGL(k_finish<1>, dim3(ceil_div(s->n, 256)), dim3(256), 0, ctx->stream, f); break;
        case 2: hipLaunchKernelGGL(k_finish<2>, dim3(ceil_div(s->n, 256)), dim3(256), 0, ctx->stream, f); break;
        default: hipLaunchKernelGGL(k_finish<3>, dim3(ceil_div(s->n, 256)), dim3(256), 0, ctx->stream, f); break;
    }
    DRG_LAUNCH_CHECK();
}

}  // namespace drg
