// drg_common.hpp -- shared device helpers of libdrgraph (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>

namespace drg {

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define DRG_HIP(call)                                                                 \
    do {                                                                              \
        hipError_t _e = (call);                                                       \
        if (_e != hipSuccess)                                                         \
            throw ::drg::Error(_e == hipErrorOutOfMemory ? -3 : -4,                   \
                               std::string(#call) + ": " + hipGetErrorString(_e));    \
    } while (0)

#define DRG_LAUNCH_CHECK() DRG_HIP(hipGetLastError())

// ---------------------------------------------------------------- constants
constexpr uint64_t TAG_INIT = 1, TAG_COARSEN = 2, TAG_NEG = 3;
constexpr uint32_t COL_MASK = 0x3FFFFFFFu;  // entry = col | (hop-1) << 30
constexpr int WAVE = 64;

// ---------------------------------------------------------------- Philox4x64-10
// Counter-based generator of Salmon et al. (SC'11): per round, the first and
// third counter words are multiplied by fixed odd constants; the high halves
// are XOR-ed with the other words and the round key, the low halves pass
// through.  The key advances by Weyl increments between rounds.
struct U64x4 {
    uint64_t w[4];
};

__device__ __forceinline__ U64x4 philox4x64(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                            uint64_t k0, uint64_t k1) {
    constexpr uint64_t MUL_A = 0xD2E7470EE14C6C93ULL, MUL_B = 0xCA5A826395121157ULL;
    constexpr uint64_t INC_A = 0x9E3779B97F4A7C15ULL, INC_B = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t pa_hi = __umul64hi(MUL_A, c0), pa_lo = MUL_A * c0;
        const uint64_t pb_hi = __umul64hi(MUL_B, c2), pb_lo = MUL_B * c2;
        const uint64_t n0 = pb_hi ^ c1 ^ k0;
        const uint64_t n2 = pa_hi ^ c3 ^ k1;
        c0 = n0;
        c1 = pb_lo;
        c2 = n2;
        c3 = pa_lo;
        k0 += INC_A;
        k1 += INC_B;
    }
    U64x4 r;
    r.w[0] = c0;
    r.w[1] = c1;
    r.w[2] = c2;
    r.w[3] = c3;
    return r;
}

__device__ __forceinline__ uint64_t pick4(const U64x4& r, int s) {
    return s == 0 ? r.w[0] : (s == 1 ? r.w[1] : (s == 2 ? r.w[2] : r.w[3]));
}

// Word for negative slot m of node i at iteration it: block (i, it, m/4).
__device__ __forceinline__ uint64_t neg_word(uint64_t seed, uint64_t it, int32_t i, int m) {
    U64x4 r = philox4x64((uint64_t)(uint32_t)i, it, (uint64_t)(m >> 2), 0, seed, TAG_NEG);
    return pick4(r, m & 3);
}

// Negative draw: the smallest v with C[v+1] > floor(w S / 2^64).  The guide
// table brackets the answer by the top gbits bits of w.
__device__ __forceinline__ int32_t draw_node(uint64_t w, const uint64_t* __restrict__ C,
                                             const int32_t* __restrict__ guide, int gbits,
                                             uint64_t S) {
    const uint64_t r = __umul64hi(w, S);
    const uint32_t bkt = (uint32_t)(w >> (64 - gbits));
    int32_t lo = guide[bkt], hi = guide[bkt + 1];
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (C[mid + 1] > r)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

// ---------------------------------------------------------------- wave / block
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int l = __lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
    return v;
}

// Butterfly sum over aligned groups of g lanes (g a power of two <= 64).
template <typename T>
__device__ __forceinline__ T group_sum_rt(T v, int g) {
    for (int off = g >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, g);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    const int l = __lane_id();
#pragma unroll
    for (int off = 1; off < WAVE; off <<= 1) {
        T t = __shfl_up(v, off, WAVE);
        if (l >= off) v += t;
    }
    return v;
}

// Exclusive block scan; sbuf is an LDS array of BLOCK/64 elements.  Ends with
// a barrier so sbuf may be reused right away.
template <int BLOCK, typename T>
__device__ __forceinline__ T block_excl_scan(T v, T* total, T* sbuf) {
    constexpr int NW = BLOCK / WAVE;
    const int wid = threadIdx.x / WAVE;
    T inc = wave_incl_scan(v);
    if (__lane_id() == WAVE - 1) sbuf[wid] = inc;
    __syncthreads();
    T off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        T t = sbuf[w];
        if (w < wid) off += t;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

// Block sum in a fixed order (deterministic for a given BLOCK).
template <int BLOCK, typename T>
__device__ __forceinline__ T block_sum(T v, T* sbuf) {
    constexpr int NW = BLOCK / WAVE;
    v = group_sum<WAVE>(v);
    if (__lane_id() == 0) sbuf[threadIdx.x / WAVE] = v;
    __syncthreads();
    T tot = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) tot += sbuf[w];
    __syncthreads();
    return tot;
}

// log(1 + x) for x >= 0 with one hardware logarithm: for u = fl(1 + x),
// log(u) * x / (u - 1) (Goldberg's correction: the rounding of u cancels to
// first order), and x itself where u rounds to 1.  Measured within 5 ulp of
// the correctly rounded value over [1e-12, 1e4] (the library log1pf: 1 ulp),
// at a fraction of its cost.
__device__ __forceinline__ float log1p_fast(float x) {
    const float u = 1.0f + x;
    if (u == 1.0f) return x;
    if (!(u <= 3.402823466e38f)) return u;  // infinity or NaN
    return __logf(u) * (x / (u - 1.0f));
}

__device__ __forceinline__ float clampf(float v, float c) {
    return __builtin_amdgcn_fmed3f(v, -c, c);  // one v_med3_f32
}

// 1/x with the hardware reciprocal (v_rcp_f32, 1 ulp).
__device__ __forceinline__ float rcp_fast(float x) { return __builtin_amdgcn_rcpf(x); }

// Clipped repulsion component k*d.  The coefficient can overflow to inf for
// a pair at an underflowing distance; a zero component then stays zero.
__device__ __forceinline__ float repel_component(float k, float d, float c) {
    return d == 0.0f ? 0.0f : clampf(k * d, c);
}

template <int B>
__device__ __forceinline__ float powi(float x) {
    if constexpr (B == 0) return 1.0f;
    else if constexpr (B == 1) return x;
    else if constexpr (B == 2) return x * x;
    else return x * x * x;
}

// Work index of block b of an nblocks-block launch.  Blocks go to the 8 XCDs
// round-robin (b % 8); this gives the blocks of one XCD a contiguous range of
// work, so each XCD's L2 serves a narrow slice of the data at a time.
__device__ __forceinline__ int32_t xcd_block(int32_t b, int32_t nblocks) {
    const int32_t x = b & 7, lb = b >> 3;
    const int32_t per = nblocks >> 3, rem = nblocks & 7;
    return x * per + min(x, rem) + lb;
}

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

}  // namespace drg
