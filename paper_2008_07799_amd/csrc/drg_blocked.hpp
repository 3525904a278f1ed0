// drg_blocked.hpp -- device side of the LDS-staged sweep over the
// column-blocked copy of P~ (see blocked.hip): staging, pair operators and
// the two sweep forms, shared by the single-graph and batched kernels.
#pragma once
#include <type_traits>

#include "drg_forces.hpp"

namespace drg {

constexpr int BLK_HOP_SHIFT = 13;

constexpr int ROWCAP = 4096;  // rows per work item

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
    int32_t flat;               // chunks per lane and batch of the flat (merge-path) form (2, 4); 0: row form
    int32_t noclip;             // 1: the clip cannot bind (attract_clip_free), flat form skips it
};

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

// The hop weight of entry u by bit masks: m = the hop bit sign-extended
// (v_bfe_i32), then one bit-field insert (v_bfi_b32) per select.  Written
// as plain selects, a chain over four values is turned into an indexed load
// from a private copy of the table, and a single select into a compare and
// a conditional move.
__device__ __forceinline__ float mask_pick(int32_t m, float if_set, float if_clear) {
    float r;
    asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(r) : "v"(m), "v"(if_set), "v"(if_clear));
    return r;
}

template <int NH>
__device__ __forceinline__ float hop_weight(const HopW& hw, uint32_t u) {
    if constexpr (NH == 1) {
        return hw.e0;
    } else {
        const int32_t m0 = __builtin_amdgcn_sbfe((int32_t)u, BLK_HOP_SHIFT, 1);  // hop bit 0
        if constexpr (NH == 2) {
            return mask_pick(m0, hw.e1, hw.e0);
        } else {
            const int32_t m1 = __builtin_amdgcn_sbfe((int32_t)u, BLK_HOP_SHIFT + 1, 1);  // hop bit 1
            return mask_pick(m1, mask_pick(m0, hw.e3, hw.e2), mask_pick(m0, hw.e1, hw.e0));
        }
    }
}

template <int B, int NH>
__device__ __forceinline__ void blk_pair(const BlockedArgs& a, const HopW& hw, const float4& ri,
                                         const float4* s_rec, uint32_t u, uint32_t lmask,
                                         bool valid, float& ax, float& ay) {
    const float4 rj = s_rec[u & lmask];
    const float dx = ri.x - rj.x, dy = ri.y - rj.y;
    const float d2 = dx * dx + dy * dy;
    const float eh = hop_weight<NH>(hw, u);
    const float p = powi<B - 1>(d2) * rcp_fast(1.0f + powi<B>(d2));
    const float w = valid ? eh * (ri.z + rj.z) : 0.0f;
    ax += w * clampf(p * dx, a.clip);
    ay += w * clampf(p * dy, a.clip);
}

// Pair operators of the flat sweep: what one stored pair (row record ri,
// column record rj, entry u) adds to the lane's partial of its row.
// `valid` = 0 masks a slot.
//
// The layout step: clipped attraction (weights carry -2b).  CLIP = false
// when the clip cannot bind (|p dx| stays below it for every d, see
// attract_clip_free): the clamp would return its argument, so it is left out and
// the weight is folded into p first (one rounding moved, two clamps and a
// multiply fewer per pair).
template <int B, int NH, bool CLIP>
struct LayoutOp {
    const BlockedArgs* a;
    HopW hw;
    __device__ __forceinline__ void operator()(const float4& ri, const float4& rj, uint32_t u,
                                               bool valid, float& ax, float& ay) const {
        const float dx = ri.x - rj.x, dy = ri.y - rj.y;
        float p;
        if constexpr (B == 1) {
            // 1 + d^2 as two FMAs: d^2 alone is not needed
            p = rcp_fast(fmaf(dx, dx, fmaf(dy, dy, 1.0f)));
        } else {
            const float d2 = dx * dx + dy * dy;
            p = powi<B - 1>(d2) * rcp_fast(1.0f + powi<B>(d2));
        }
        const float w = valid ? hop_weight<NH>(hw, u) * (ri.z + rj.z) : 0.0f;
        if constexpr (CLIP) {
            ax += w * clampf(p * dx, a->clip);
            ay += w * clampf(p * dy, a->clip);
        } else {
            const float k = w * p;
            ax += k * dx;
            ay += k * dy;
        }
    }
};

// the objective: P~_ij log w_ij = -P~_ij log1p(d^{2b}) (weights are e_d / 2)
template <int B, int NH>
struct ObjValOp {
    HopW hw;
    __device__ __forceinline__ void operator()(const float4& ri, const float4& rj, uint32_t u,
                                               bool valid, float& ax, float& ay) const {
        const float dx = ri.x - rj.x, dy = ri.y - rj.y;
        const float d2 = dx * dx + dy * dy;
        const float pw = valid ? hop_weight<NH>(hw, u) * (ri.z + rj.z) : 0.0f;
        ax += pw * (-log1p_fast(powi<B>(d2)));
        (void)ay;
    }
};

// its gradient's attraction (unclipped): P~_ij (-2b d^{2b-2} / (1 + d^{2b})) (y_i - y_j)
template <int B, int NH>
struct ObjGradOp {
    HopW hw;
    __device__ __forceinline__ void operator()(const float4& ri, const float4& rj, uint32_t u,
                                               bool valid, float& ax, float& ay) const {
        const float dx = ri.x - rj.x, dy = ri.y - rj.y;
        const float d2 = dx * dx + dy * dy;
        const float pw = valid ? hop_weight<NH>(hw, u) * (ri.z + rj.z) : 0.0f;
        const float k = pw * (float)(-2 * B) * powi<B - 1>(d2) * rcp_fast(1.0f + powi<B>(d2));
        ax += k * dx;
        ay += k * dy;
    }
};

// Workgroups of 1024 threads; an entry chunk is 16 bytes (eight 16-bit words).
constexpr int STREAM_BLOCK = 1024;
constexpr int STREAM_WAVES = STREAM_BLOCK / WAVE;
constexpr int ROW_CACHE = WAVE;  // row records per wave cached by the flat form

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

// Lane moves by DPP (register crossbar, no LDS): a lane reads the value of
// another lane of the wave; a lane with no source lane, or outside the rows
// enabled by RM, reads 0.
constexpr int DPP_ROW_SHR = 0x110;      // + d: lane - d of the same 16-lane row
constexpr int DPP_WAVE_SHR1 = 0x138;    // lane - 1 of the wave
constexpr int DPP_ROW_BCAST15 = 0x142;  // lane 15 of the previous row (rows 1, 3: RM 0xA)
constexpr int DPP_ROW_BCAST31 = 0x143;  // lane 31 (rows 2, 3: RM 0xC)

template <int CTRL, int RM>
__device__ __forceinline__ int32_t lane_dpp(int32_t v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, RM, 0xF, false);
}

template <int CTRL, int RM>
__device__ __forceinline__ float lane_dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, RM, 0xF, false));
}

// ------------------------------------------------------------------ flat form
// The entries of an item (rows r0..r1 of block b) are contiguous, so the
// item is swept as one stream regardless of row boundaries: wave w takes a
// contiguous range of its 16-byte chunks, lane l the chunks w0 + 2 CPL l ..
// w0 + 2 CPL (l+1) - 1 of each window of 128 CPL chunks; every lane walks
// its entries in order, tracking the row through the LDS row offsets.  A row
// that starts and ends inside one lane is
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

// largest i in [lo, hi] with off[i] <= p, given off[lo] <= p, for
// wave-uniform lo, hi, p (all lanes active): the wave tests the next 64
// offsets at once; as off is non-decreasing, those at most p form a prefix,
// so the answer is lo plus its length (one LDS read per 64 rows)
__device__ __forceinline__ int32_t row_from_wave(const int32_t* off, int32_t lo, int32_t hi,
                                                 int32_t p) {
    const int lane = __lane_id();
    while (true) {
        const int32_t j = lo + 1 + lane;
        const bool le = j <= hi && off[j] <= p;
        const int c = __popcll(__ballot(le));
        if (c < WAVE) return lo + c;
        lo += WAVE;
    }
}

// TOGETHER = false: the next window's second batch is requested only when
// it starts (no third buffer: for kernels short of registers).  The loads'
// timing does not change any result.
template <int CPL, typename Op, bool TOGETHER = true>
__device__ __forceinline__ void blk_flat(const BlockedArgs& a, const Op& op, const float4* s_rec,
                                         const int32_t* s_off, WaveFrag* s_frag, int32_t b,
                                         int32_t r0, int32_t r1) {
    // A lane takes 2 CPL consecutive chunks per window, held as two batches
    // of CPL: once this window's first batch is used, both batches of the
    // next window are requested together (so the two halves of a lane's
    // cache lines are fetched together, not a half window apart, when one
    // could be evicted in between), and the second batch waits in a third
    // buffer until this window's second batch is used.
    constexpr int CPW = 2 * CPL;          // chunks per lane per window
    constexpr int EPL = 8 * CPW;          // entries per lane per window
    constexpr int WCH = WAVE * CPW;       // chunks per window
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
    // rows [i0, i1] spanned by the window starting at chunk w (wave-uniform),
    // searched from row lo
    auto win_rows = [&](int64_t w, int32_t lo, int32_t& i0, int32_t& i1) {
        const int32_t wp0 = max((int32_t)(8 * w - bbase), e0);
        const int32_t wp1 = min((int32_t)(8 * min(w + WCH, wc1) - bbase), e1) - 1;
        i0 = row_from_wave(s_off, lo, nr - 1, wp0);
        i1 = row_from_wave(s_off, i0, nr - 1, wp1);
    };
    // The records of the first ROW_CACHE rows of a window sit in the wave's
    // LDS cache (x, y, z arrays), so a lane that moves on to the next row
    // reads its record there instead of waiting on a global load.  Each
    // window's records are requested one window ahead.
    float* cx = reinterpret_cast<float*>(s_frag + STREAM_WAVES) + wid * (3 * ROW_CACHE);
    float* cy = cx + ROW_CACHE;
    float* cz = cy + ROW_CACHE;
    auto row_rec = [&](int32_t i0, int32_t i1, float& x, float& y, float& z) {
        const int32_t r = i0 + lane;
        const float4 t = r <= i1 ? R[r] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        x = t.x;
        y = t.y;
        z = t.z;
    };
    int32_t ni0 = 0, ni1 = -1;  // rows of the next window
    float nx = 0.0f, ny = 0.0f, nz = 0.0f;
    if (wc0 < wc1) {
        win_rows(wc0, max(w_first, 0), ni0, ni1);
        row_rec(ni0, ni1, nx, ny, nz);
    }
    // chunk loads are unconditional, clamped to the wave's last chunk (slots
    // past the range are masked), so the counters of outstanding loads stay
    // exact and a wait for one load does not drain the prefetches
    const int64_t clast = max(wc1 - 1, wc0);
    uint4 va[CPL], vb[CPL], vn[TOGETHER ? CPL : 1];
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
        va[k] = E4[min(wc0 + (int64_t)lane * CPW + k, clast)];
        if constexpr (TOGETHER) vb[k] = E4[min(wc0 + (int64_t)lane * CPW + CPL + k, clast)];
    }
    for (int64_t w0 = wc0; w0 < wc1; w0 += WCH) {
        // this window's rows and their cached records
        const int32_t i0 = ni0, i1 = ni1;
        cx[lane] = nx;
        cy[lane] = ny;
        cz[lane] = nz;
        if (w0 + WCH < wc1) {
            win_rows(w0 + WCH, i1, ni0, ni1);
            row_rec(ni0, ni1, nx, ny, nz);
        }
        // record of row i of this window: cached, or from global memory
        auto load_row = [&](int32_t i) {
            const int32_t k = i - i0;
            float4 t;
            if (k < ROW_CACHE) {
                t = make_float4(cx[k], cy[k], cz[k], 0.0f);
            } else {
                t = R[i];
                // keeps the load on this (rare) path: otherwise it is moved
                // past the branch and every entry waits for it
                asm volatile("" : "+v"(t.x), "+v"(t.y), "+v"(t.z));
            }
            return t;
        };
        const int64_t c = w0 + (int64_t)lane * CPW;  // the lane's first chunk
        const int32_t nl = (int32_t)min((int64_t)WAVE, (wc1 - w0 + CPW - 1) / CPW);
        const bool has = lane < nl;
        const int32_t pbase = (int32_t)(8 * c - bbase);
        const int32_t pf = max(pbase, e0);                                  // first valid slot
        const int32_t pl = min(min(pbase + EPL, (int32_t)(8 * wc1 - bbase)), e1);  // end of valid slots
        // the same bounds relative to the lane's first slot (none valid without a chunk)
        const int32_t qlo = pf - pbase, qhi = has ? pl - pbase : 0;
        // the lane's first row
        int32_t i = has ? row_of(s_off, i0, i1, pf) : i1;
        int32_t nxt = s_off[i + 1];
        float4 ri = load_row(i);
        // FULL: every slot of every lane of the window is valid (all windows
        // but those at the ends of an item or of the wave's range)
        const bool full = __all(has && qlo == 0 && qhi == EPL);
        if constexpr (!TOGETHER) {
            if (full) {
#pragma unroll
                for (int k = 0; k < CPL; ++k) vb[k] = E4[min(c + CPL + k, clast)];
            }
        }
        float ax = 0.0f, ay = 0.0f, hx = 0.0f, hy = 0.0f;
        const int32_t hrow = i;
        bool hopen = true;  // still on the lane's first row
        int32_t qn = nxt - pbase;  // slot where the current row ends
        // If the first row ends inside the lane's slots, the row that follows
        // (the one holding position nxt) and its record are found now, by all
        // such lanes together, so that the first row change in the slots
        // below only moves registers (a later one, rare, searches itself).
        bool pre = has && nxt < pl;
        int32_t i2 = i, nxt2 = nxt;
        float4 r2 = ri;
        if (pre) {
            do {
                ++i2;
                nxt2 = s_off[i2 + 1];
            } while (nxt >= nxt2);
            r2 = load_row(i2);
        }
        // the pair of slot Q (entry u, column record rj), after closing the
        // rows that end before it
        auto slot = [&](int32_t Q, bool valid, uint32_t u, const float4& rj) {
            if (valid && Q >= qn) {  // the row ends before this slot
                if (hopen) {
                    hx = ax;
                    hy = ay;
                    hopen = false;
                } else {
                    // started and ended inside this lane, so it is not the
                    // wave's open first row: stored directly (32-bit offset)
                    *reinterpret_cast<float2*>(reinterpret_cast<char*>(P) +
                                               (uint32_t)i * (uint32_t)sizeof(float2)) =
                        make_float2(ax, ay);
                }
                if (pre) {
                    // valid slots are consecutive, so this slot is at
                    // position nxt: the row found above
                    i = i2;
                    nxt = nxt2;
                    ri = r2;
                    pre = false;
                } else {
                    const int32_t p = pbase + Q;
                    do {
                        ++i;
                        nxt = s_off[i + 1];
                    } while (p >= nxt);
                    ri = load_row(i);
                }
                qn = nxt - pbase;
                ax = 0.0f;
                ay = 0.0f;
            }
            op(ri, rj, u, valid, ax, ay);
        };
        if (full) {
            // the slots of one batch, chunks v[0..CPL) at slots Q0 .., unrolled
            auto batch = [&](auto q0_c, const uint4* v) {
                constexpr int32_t Q0 = decltype(q0_c)::value;
#pragma unroll
                for (int k = 0; k < CPL; ++k) {
#pragma unroll
                    for (int h = 0; h < 8; h += 4) {
                        // four column records requested before any is used
                        float4 rj[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q) rj[q] = s_rec[half16(v[k], h + q) & lmask];
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            slot(Q0 + 8 * k + h + q, true, half16(v[k], h + q), rj[q]);
                    }
                }
            };
            batch(std::integral_constant<int32_t, 0>{}, va);
            // the next window's batches
#pragma unroll
            for (int k = 0; k < CPL; ++k) {
                va[k] = E4[min(c + WCH + k, clast)];
                if constexpr (TOGETHER) vn[k] = E4[min(c + WCH + CPL + k, clast)];
            }
            batch(std::integral_constant<int32_t, 8 * CPL>{}, vb);
            if constexpr (TOGETHER) {
#pragma unroll
                for (int k = 0; k < CPL; ++k) vb[k] = vn[k];
            }
        } else {
            // a window at the end of the item or of the wave's range: the
            // chunks are read again one at a time (they are cached), every
            // slot tested
            for (int k = 0; k < CPW; ++k) {
                const uint4 ck = E4[min(c + k, clast)];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int32_t Q = 8 * k + q;
                    const uint32_t u = half16(ck, q);
                    slot(Q, Q >= qlo && Q < qhi, u, s_rec[u & lmask]);
                }
            }
#pragma unroll
            for (int k = 0; k < CPL; ++k) {
                va[k] = E4[min(c + WCH + k, clast)];
                if constexpr (TOGETHER) vb[k] = E4[min(c + WCH + CPL + k, clast)];
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
        // keyed inclusive scan of the lanes' last-row partials (keys are
        // row + 1, or a distinct negative value for a lane without entries;
        // never 0, the key a lane reads when it has no source lane)
        const int32_t tk = has ? i + 1 : -1 - lane;
        float sx = ax, sy = ay;
        auto scan_step = [&](auto ctrl_c, auto rows_c) {
            constexpr int C = decltype(ctrl_c)::value, RM = decltype(rows_c)::value;
            const int32_t ok = lane_dpp<C, RM>(tk);
            const float ox = lane_dpp<C, RM>(sx), oy = lane_dpp<C, RM>(sy);
            if (ok == tk) {
                sx = ox + sx;
                sy = oy + sy;
            }
        };
        scan_step(std::integral_constant<int, DPP_ROW_SHR + 1>{}, std::integral_constant<int, 0xF>{});
        scan_step(std::integral_constant<int, DPP_ROW_SHR + 2>{}, std::integral_constant<int, 0xF>{});
        scan_step(std::integral_constant<int, DPP_ROW_SHR + 4>{}, std::integral_constant<int, 0xF>{});
        scan_step(std::integral_constant<int, DPP_ROW_SHR + 8>{}, std::integral_constant<int, 0xF>{});
        scan_step(std::integral_constant<int, DPP_ROW_BCAST15>{}, std::integral_constant<int, 0xA>{});
        scan_step(std::integral_constant<int, DPP_ROW_BCAST31>{}, std::integral_constant<int, 0xC>{});
        // a first row that ended inside the lane: add what earlier lanes hold
        const float px = lane_dpp<DPP_WAVE_SHR1, 0xF>(sx), py = lane_dpp<DPP_WAVE_SHR1, 0xF>(sy);
        const int32_t pk = lane_dpp<DPP_WAVE_SHR1, 0xF>(tk);
        if (has && !hopen) {
            const bool cin = lane > 0 && pk == hrow + 1;
            close_row(hrow, cin ? px + hx : hx, cin ? py + hy : hy);
        }
        // the last row: complete unless it goes on past this lane (into the
        // next lane, the next window or the next wave)
        const bool cont = has && nxt > pl;
        if (has && !cont) close_row(i, sx, sy);
        // carry of the window's last lane
        const int32_t L = __builtin_amdgcn_readfirstlane(nl - 1);  // wave-uniform
        const bool lcont = __builtin_amdgcn_readlane(cont ? 1 : 0, L) != 0;
        const int32_t lrow = __builtin_amdgcn_readlane(i, L);
        const float lx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(sx), L));
        const float ly = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(sy), L));
        c_row = lcont ? lrow : -1;
        c_x = lcont ? lx : 0.0f;
        c_y = lcont ? ly : 0.0f;
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
// item's row offsets go to LDS, then the rows are swept.  Lane sums run in a
// fixed order and the group reductions are fixed, so the result is
// repeatable.
// Stages block b's records into LDS (callers synchronise before use).
// Each thread requests all its records before writing any, so the staging
// costs one memory round trip instead of one per record.
__device__ __forceinline__ void blk_stage_rec(const BlockedArgs& a, float4* s_rec, int32_t b) {
    constexpr int RU = 8;  // records per thread per pass (8192-record blocks: one pass)
    const int32_t bw = 1 << a.bits;
    const int32_t j0 = b * bw;
    const int32_t cnt = min(bw, a.n0 - j0);
    for (int32_t t0 = 0; t0 < bw; t0 += STREAM_BLOCK * RU) {
        float4 v[RU];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int32_t t = t0 + u * STREAM_BLOCK + (int32_t)threadIdx.x;
            v[u] = t < cnt ? a.rec[j0 + t] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int32_t t = t0 + u * STREAM_BLOCK + (int32_t)threadIdx.x;
            if (t < bw) s_rec[t] = v[u];
        }
    }
}

// Stages the row offsets of rows r0..r1 in block b (all requests first),
// then synchronises.
__device__ __forceinline__ void blk_stage_off(const BlockedArgs& a, int32_t* s_off, int32_t b,
                                              int32_t r0, int32_t r1) {
    constexpr int OU = (ROWCAP + STREAM_BLOCK) / STREAM_BLOCK;  // covers ROWCAP + 1 offsets
    const int32_t* O = a.off + (int64_t)b * (a.n0 + 1) + r0;
    const int32_t nr = r1 - r0;
    int32_t v[OU];
#pragma unroll
    for (int u = 0; u < OU; ++u) {
        const int32_t t = u * STREAM_BLOCK + (int32_t)threadIdx.x;
        v[u] = t <= nr ? O[t] : 0;
    }
#pragma unroll
    for (int u = 0; u < OU; ++u) {
        const int32_t t = u * STREAM_BLOCK + (int32_t)threadIdx.x;
        if (t <= nr) s_off[t] = v[u];
    }
    __syncthreads();
}

// The sweep of one work item (block b, rows r0..r1) once the block's records
// and the item's row offsets are in LDS: the flat form with F chunks per
// lane and batch (F = 2, 4), or for F = 0 the row form (a.lanes lanes per
// segment, 0: chosen from the item's mean segment length).  s_dyn is the
// workgroup's dynamic LDS (records, row offsets, wave fragments).
template <int B, int NH, int F, bool TOGETHER = true>
__device__ __forceinline__ void blk_sweep_staged(const BlockedArgs& a, float4* s_dyn, int32_t b,
                                                 int32_t r0, int32_t r1) {
    const int32_t bw = 1 << a.bits;
    float4* s_rec = s_dyn;
    int32_t* s_off = reinterpret_cast<int32_t*>(s_dyn + bw);
    WaveFrag* s_frag = reinterpret_cast<WaveFrag*>(s_dyn + bw + (ROWCAP + 4) / 4);
    if constexpr (F > 0) {
        if (a.noclip)
            blk_flat<F, LayoutOp<B, NH, false>, TOGETHER>(
                a, LayoutOp<B, NH, false>{&a, hop_weights(a)}, s_rec, s_off, s_frag, b, r0, r1);
        else
            blk_flat<F, LayoutOp<B, NH, true>, TOGETHER>(
                a, LayoutOp<B, NH, true>{&a, hop_weights(a)}, s_rec, s_off, s_frag, b, r0, r1);
    } else {
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
}

// One work item of the layout sweep: staging, then the sweep.
template <int B, int NH, int F>
__device__ __forceinline__ void blk_layout_item(const BlockedArgs& a, float4* s_dyn, int32_t b,
                                                int32_t r0, int32_t r1) {
    const int32_t bw = 1 << a.bits;
    blk_stage_rec(a, s_dyn, b);
    blk_stage_off(a, reinterpret_cast<int32_t*>(s_dyn + bw), b, r0, r1);
    blk_sweep_staged<B, NH, F>(a, s_dyn, b, r0, r1);
}

// Consecutive work items items[0..cnt) of one block b: the records are
// staged once, then every item is swept exactly as alone (its own row
// offsets, wave ranges and lane order), so the result is the same bit for
// bit as one workgroup per item (the next window's second batch is
// requested late: this loop leaves too few registers for a third buffer).
template <int B, int NH, int F>
__device__ __forceinline__ void blk_layout_items(const BlockedArgs& a, float4* s_dyn, int32_t b,
                                                 const int4* __restrict__ items, int32_t cnt) {
    const int32_t bw = 1 << a.bits;
    blk_stage_rec(a, s_dyn, b);
    for (int32_t k = 0; k < cnt; ++k) {
        const int4 it = items[k];
        __syncthreads();  // the previous item is done with the offsets and fragments
        blk_stage_off(a, reinterpret_cast<int32_t*>(s_dyn + bw), b, it.y, it.z);
        blk_sweep_staged<B, NH, F, false>(a, s_dyn, b, it.y, it.z);
    }
}

// sweep form as a template argument: the flat form's chunks per lane and batch, 0 for
// the row form
inline int blk_form(int flat) { return (flat == 2 || flat == 4) ? flat : 0; }

// dynamic LDS of a blocked-sweep workgroup: column records, row offsets,
// wave fragments, the flat form's row-record caches
inline size_t blk_lds_bytes(int bits) {
    return ((size_t)16 << bits) + 16 * ((ROWCAP + 4) / 4) + sizeof(WaveFrag) * STREAM_WAVES +
           sizeof(float) * 3 * ROW_CACHE * STREAM_WAVES;
}

// g_i of one finest node on the blocked layout: its block partials added in
// block order, plus its own M negatives (draw(w) gives the record index of
// the drawn node, key the node's own id for the negative words).
template <int B, typename Draw>
__device__ __forceinline__ float2 blk_finish_row(const float2* __restrict__ partial, int32_t nb,
                                                 int64_t stride, int32_t row,
                                                 const float4* __restrict__ rec, const float4& ri,
                                                 int M, uint64_t seed, uint64_t iter, int32_t key,
                                                 Draw draw, float gq, float clip) {
    float ax = 0.0f, ay = 0.0f;
    for (int32_t b = 0; b < nb; ++b) {
        const float2 p = partial[(int64_t)b * stride + row];
        ax += p.x;
        ay += p.y;
    }
    float rx = 0.0f, ry = 0.0f;
    for (int m = 0; m < M; ++m) {
        const float4 rv = rec[draw(neg_word(seed, iter, key, m))];
        const float dx = ri.x - rv.x, dy = ri.y - rv.y;
        const float d2 = dx * dx + dy * dy;
        if (d2 > 0.0f) {
            const float k = blk_repel_coef<B>(d2);
            rx += repel_component(k, dx, clip);
            ry += repel_component(k, dy, clip);
        }
    }
    return make_float2(ax + gq * rx, ay + gq * ry);
}

}  // namespace drg
