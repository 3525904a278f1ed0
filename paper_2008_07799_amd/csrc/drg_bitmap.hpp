// drg_bitmap.hpp -- "set of node ids in a bitmap -> sorted list" on a block.
#pragma once
#include "drg_common.hpp"

namespace drg {

// Reads and clears bm[0..nwords), skipping bit `skip` (-1: none), and calls
// emit(position, id) for every set bit in ascending id order, positions
// starting at `base`.  Each thread takes WPT consecutive words per chunk; a
// block prefix sum of the per-thread popcounts places them.  All threads of
// the block must call it; s_red holds BLOCK/64 ints of LDS.
template <int BLOCK, int WPT, typename Emit>
__device__ __forceinline__ int64_t bitmap_emit_clear(uint32_t* bm, int nwords, int skip,
                                                     int64_t base, int* s_red, Emit emit) {
    for (int w0 = 0; w0 < nwords; w0 += BLOCK * WPT) {
        const int wb = w0 + (int)threadIdx.x * WPT;
        uint32_t wv[WPT];
        int c = 0;
#pragma unroll
        for (int j = 0; j < WPT; ++j) {
            const int w = wb + j;
            uint32_t x = 0;
            if (w < nwords) {
                x = bm[w];
                if (x) bm[w] = 0;
                if (skip >= 0 && w == (skip >> 5)) x &= ~(1u << (skip & 31));
            }
            wv[j] = x;
            c += __popc(x);
        }
        int tot;
        const int ex = block_excl_scan<BLOCK>(c, &tot, s_red);
        int64_t o = base + ex;
#pragma unroll
        for (int j = 0; j < WPT; ++j) {
            uint32_t x = wv[j];
            while (x) {
                const int b = __ffs(x) - 1;
                x &= x - 1;
                emit(o++, ((uint32_t)(wb + j) << 5) | (uint32_t)b);
            }
        }
        base += tot;
    }
    return base;
}

// Reads and clears bm[0..nwords); returns the number of set bits (block-wide).
template <int BLOCK>
__device__ __forceinline__ int bitmap_count_clear(uint32_t* bm, int nwords, int* s_red) {
    int c = 0;
    for (int w = threadIdx.x; w < nwords; w += BLOCK) {
        const uint32_t x = bm[w];
        if (x) {
            c += __popc(x);
            bm[w] = 0;
        }
    }
    return block_sum<BLOCK>(c, s_red);
}

}  // namespace drg
