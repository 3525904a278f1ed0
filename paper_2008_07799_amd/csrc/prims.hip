// prims.hip -- scans, stable radix sort and counts used by the build stages.
#include "drg_common.hpp"
#include "drg_prims.hpp"

namespace drg {

Allocator& thread_allocator() {
    static thread_local Allocator a;
    return a;
}

void* dev_alloc_bytes(int64_t bytes, const Allocator& al) {
    void* p = nullptr;
    if (al.alloc) {
        p = al.alloc((size_t)bytes, al.user);
        if (!p)
            throw Error(-3, "allocator returned NULL for " + std::to_string(bytes) + " bytes");
        return p;
    }
    hipError_t e = hipMalloc(&p, (size_t)bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error(e == hipErrorOutOfMemory ? -3 : -4,
                    "hipMalloc(" + std::to_string(bytes) + " bytes): " + hipGetErrorString(e));
    }
    return p;
}

// ------------------------------------------------------------------ scan
constexpr int SCAN_BLOCK = 256, SCAN_IPT = 8, SCAN_TILE = SCAN_BLOCK * SCAN_IPT;

template <typename T>
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_tiles(const T* __restrict__ in,
                                                           T* __restrict__ out, int64_t n,
                                                           T* __restrict__ partial) {
    __shared__ T sbuf[SCAN_BLOCK / WAVE];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_IPT;
    T v[SCAN_IPT];
    T s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_IPT; ++j) {
        const int64_t idx = base + j;
        v[j] = idx < n ? in[idx] : T(0);
        s += v[j];
    }
    T tot;
    T run = block_excl_scan<SCAN_BLOCK>(s, &tot, sbuf);
#pragma unroll
    for (int j = 0; j < SCAN_IPT; ++j) {
        const int64_t idx = base + j;
        if (idx < n) out[idx] = run;
        run += v[j];
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

template <typename T>
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_add(T* __restrict__ out, int64_t n,
                                                         const T* __restrict__ offs) {
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    const T add = offs[blockIdx.x];
    for (int j = threadIdx.x; j < SCAN_TILE; j += SCAN_BLOCK) {
        const int64_t idx = base + j;
        if (idx < n) out[idx] += add;
    }
}

template <typename T>
void exclusive_scan(const T* in, T* out, int64_t n, hipStream_t s) {
    const int64_t nb = n > 0 ? (n + SCAN_TILE - 1) / SCAN_TILE : 1;
    DevBuf<T> partial(nb + 1);
    if (n > 0) {
        hipLaunchKernelGGL(k_scan_tiles<T>, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, in, out,
                           n, partial.get());
        DRG_LAUNCH_CHECK();
    } else {
        DRG_HIP(hipMemsetAsync(partial.get(), 0, sizeof(T), s));
    }
    if (nb > 1) {
        DevBuf<T> offs(nb + 1);
        exclusive_scan<T>(partial.get(), offs.get(), nb, s);
        hipLaunchKernelGGL(k_scan_add<T>, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, out, n,
                           offs.get());
        DRG_LAUNCH_CHECK();
        DRG_HIP(hipMemcpyAsync(out + n, offs.get() + nb, sizeof(T), hipMemcpyDeviceToDevice, s));
        DRG_HIP(hipStreamSynchronize(s));
    } else {
        DRG_HIP(hipMemcpyAsync(out + n, partial.get(), sizeof(T), hipMemcpyDeviceToDevice, s));
        DRG_HIP(hipStreamSynchronize(s));
    }
}

template void exclusive_scan<int32_t>(const int32_t*, int32_t*, int64_t, hipStream_t);
template void exclusive_scan<uint32_t>(const uint32_t*, uint32_t*, int64_t, hipStream_t);
template void exclusive_scan<int64_t>(const int64_t*, int64_t*, int64_t, hipStream_t);
template void exclusive_scan<uint64_t>(const uint64_t*, uint64_t*, int64_t, hipStream_t);

// ------------------------------------------------------------------ radix sort
// LSD radix sort, 8-bit digits.  Per pass: a per-tile digit histogram laid out
// digit-major, an exclusive scan of it, then a stable scatter.  Inside a tile
// items are ranked in index order: per wave, lanes with equal digits are
// matched with eight ballots; per-wave digit counts in LDS order the waves.
constexpr int RS_BLOCK = 256, RS_IPT = 8, RS_TILE = RS_BLOCK * RS_IPT, RS_BINS = 256;
constexpr int RS_NW = RS_BLOCK / WAVE;

__global__ __launch_bounds__(RS_BLOCK) void k_rs_hist(const uint32_t* __restrict__ keys, int64_t n,
                                                      int shift, uint32_t* __restrict__ hist,
                                                      int64_t nblocks) {
    __shared__ uint32_t h[RS_BINS];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int j = threadIdx.x; j < RS_TILE; j += RS_BLOCK) {
        const int64_t idx = base + j;
        if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 0xFF], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(RS_BLOCK) void k_rs_scatter(
    const uint32_t* __restrict__ kin, const int32_t* __restrict__ vin, int64_t n, int shift,
    const uint32_t* __restrict__ offs, int64_t nblocks, uint32_t* __restrict__ kout,
    int32_t* __restrict__ vout) {
    __shared__ uint32_t run[RS_BINS];
    __shared__ uint32_t wcnt[RS_NW][RS_BINS];
    const int tid = threadIdx.x, wid = tid / WAVE;
    run[tid] = offs[(int64_t)tid * nblocks + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_IPT; ++r) {
#pragma unroll
        for (int w = 0; w < RS_NW; ++w) wcnt[w][tid] = 0;
        __syncthreads();
        const int64_t idx = base + (int64_t)r * RS_BLOCK + tid;
        const bool valid = idx < n;
        const uint32_t key = valid ? kin[idx] : 0u;
        const uint32_t dig = (key >> shift) & 0xFF;
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool on = (dig >> bit) & 1u;
            const uint64_t bm = __ballot(on);
            m &= on ? bm : ~bm;
        }
        const int rank = __popcll(m & lanemask_lt());
        if (valid && rank == 0) wcnt[wid][dig] = (uint32_t)__popcll(m);
        __syncthreads();
        {
            uint32_t acc = run[tid];
#pragma unroll
            for (int w = 0; w < RS_NW; ++w) {
                const uint32_t c = wcnt[w][tid];
                wcnt[w][tid] = acc;
                acc += c;
            }
            run[tid] = acc;
        }
        __syncthreads();
        if (valid) {
            const uint32_t pos = wcnt[wid][dig] + (uint32_t)rank;
            kout[pos] = key;
            vout[pos] = vin[idx];
        }
        __syncthreads();
    }
}

void radix_sort_pairs(uint32_t* keys, int32_t* vals, int64_t n, int key_bits, hipStream_t s) {
    if (n <= 1) return;
    if (n >= (int64_t)1 << 32) throw Error(-5, "radix_sort_pairs: too many items");
    const int64_t nb = (n + RS_TILE - 1) / RS_TILE;
    DevBuf<uint32_t> k2(n);
    DevBuf<int32_t> v2(n);
    DevBuf<uint32_t> hist(nb * RS_BINS + 1), offs(nb * RS_BINS + 1);
    uint32_t *ka = keys, *kb = k2.get();
    int32_t *va = vals, *vb = v2.get();
    const int passes = key_bits <= 0 ? 0 : (key_bits + 7) / 8;
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)nb), dim3(RS_BLOCK), 0, s, ka, n, shift,
                           hist.get(), nb);
        DRG_LAUNCH_CHECK();
        exclusive_scan<uint32_t>(hist.get(), offs.get(), nb * RS_BINS, s);
        hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)nb), dim3(RS_BLOCK), 0, s, ka, va, n,
                           shift, offs.get(), nb, kb, vb);
        DRG_LAUNCH_CHECK();
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (ka != keys) {
        DRG_HIP(hipMemcpyAsync(keys, ka, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
        DRG_HIP(hipMemcpyAsync(vals, va, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    }
    DRG_HIP(hipStreamSynchronize(s));
}

// ------------------------------------------------------------------ counts
template <typename T>
__global__ void k_count_nonempty(const T* __restrict__ rp, int64_t n,
                                 unsigned long long* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool ne = i < n && rp[i + 1] > rp[i];
    const uint64_t m = __ballot(ne);
    if (__lane_id() == 0 && m) atomicAdd(out, (unsigned long long)__popcll(m));
}

template <typename T>
int64_t count_nonempty_rows(const T* rp, int64_t n, hipStream_t s) {
    DevBuf<unsigned long long> c(1);
    DRG_HIP(hipMemsetAsync(c.get(), 0, sizeof(unsigned long long), s));
    if (n > 0) {
        hipLaunchKernelGGL(k_count_nonempty<T>, dim3(ceil_div(n, 256)), dim3(256), 0, s, rp, n,
                           c.get());
        DRG_LAUNCH_CHECK();
    }
    unsigned long long h = 0;
    DRG_HIP(hipMemcpyAsync(&h, c.get(), sizeof(h), hipMemcpyDeviceToHost, s));
    DRG_HIP(hipStreamSynchronize(s));
    return (int64_t)h;
}

template int64_t count_nonempty_rows<int32_t>(const int32_t*, int64_t, hipStream_t);
template int64_t count_nonempty_rows<int64_t>(const int64_t*, int64_t, hipStream_t);

// Lanes of a wave whose rows share a group id add their count with one
// atomic per run of equal ids (the ids of a union are sorted by graph, so a
// wave touches one or two counters instead of 64 atomics on one address).
template <typename T>
__global__ void k_count_nonempty_by_group(const T* __restrict__ rp, const int32_t* __restrict__ gid,
                                          int64_t n, int32_t* __restrict__ cnt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = (int)__lane_id();
    const bool in = i < n;
    const bool ne = in && rp[i + 1] > rp[i];
    const int32_t g = in ? gid[i] : -1;
    const int32_t gp = __shfl_up(g, 1);
    const bool head = in && (lane == 0 || gp != g);
    const uint64_t heads = __ballot(head);
    const uint64_t flags = __ballot(ne);
    if (head) {
        const uint64_t above = lane == 63 ? 0ull : heads & (~0ull << (lane + 1));
        const uint64_t upto = above ? (above & (0ull - above)) - 1ull : ~0ull;
        const int c = __popcll(flags & upto & (~0ull << lane));
        if (c) atomicAdd(&cnt[g], c);
    }
}

template <typename T>
void count_nonempty_by_group(const T* rp, const int32_t* gid, int64_t n, int32_t* cnt,
                             int32_t groups, hipStream_t s) {
    DRG_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t) * (size_t)std::max<int32_t>(groups, 0), s));
    if (n > 0) {
        hipLaunchKernelGGL(k_count_nonempty_by_group<T>, dim3(ceil_div(n, 256)), dim3(256), 0, s,
                           rp, gid, n, cnt);
        DRG_LAUNCH_CHECK();
    }
}

// out[g] = sum over the rows of group g of len^2 (gid NULL: one group).  A
// wave whose rows all belong to one group adds with one atomic.
__global__ void k_sum_len2(const int64_t* __restrict__ rp, const int32_t* __restrict__ gid,
                           int64_t n, unsigned long long* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = i < n;
    const unsigned long long l = in ? (unsigned long long)(rp[i + 1] - rp[i]) : 0ull;
    const unsigned long long v = l * l;
    const int32_t g = in ? (gid ? gid[i] : 0) : -1;
    const int32_t g0 = __builtin_amdgcn_readfirstlane(g);
    if (__all(g == g0 || !in)) {
        const unsigned long long t = group_sum<WAVE>(v);
        if (__lane_id() == 0 && t) atomicAdd(&out[g0], t);
    } else if (in && v) {
        atomicAdd(&out[g], v);
    }
}

void sum_len2_by_group(const int64_t* rp, const int32_t* gid, int64_t n, unsigned long long* out,
                       int32_t groups, hipStream_t s) {
    DRG_HIP(hipMemsetAsync(out, 0, sizeof(unsigned long long) * (size_t)std::max<int32_t>(groups, 1),
                           s));
    if (n > 0) {
        hipLaunchKernelGGL(k_sum_len2, dim3(ceil_div(n, 256)), dim3(256), 0, s, rp, gid, n, out);
        DRG_LAUNCH_CHECK();
    }
}

template void count_nonempty_by_group<int32_t>(const int32_t*, const int32_t*, int64_t, int32_t*,
                                               int32_t, hipStream_t);
template void count_nonempty_by_group<int64_t>(const int64_t*, const int32_t*, int64_t, int32_t*,
                                               int32_t, hipStream_t);

}  // namespace drg
