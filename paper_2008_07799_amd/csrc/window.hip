// window.hip -- work items of the windowed sweep: consecutive rows of one
// graph (as many as the groups of a workgroup hold) and the column window
// their pattern entries span.
#include <climits>
#include <cstdlib>

#include "drg_forces.hpp"
#include "drg_internal.hpp"

namespace drg {

// last c in [0, count) with off[c] <= x
__device__ __forceinline__ int32_t owner_of(const int32_t* __restrict__ off, int32_t count,
                                            int64_t x) {
    int32_t lo = 0, hi = count - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if ((int64_t)off[mid] <= x)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// item t of graph c: rows base[c] + (t - ibase[c]) * R[c] ..., empty window
__global__ void k_win_items(int32_t nitems, int32_t count, const int32_t* __restrict__ ibase,
                            const int32_t* __restrict__ base, const int32_t* __restrict__ R,
                            WinItem* __restrict__ items) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nitems) return;
    const int32_t c = owner_of(ibase, count, t);
    const int32_t r0 = base[c] + (int32_t)(t - ibase[c]) * R[c];
    WinItem it{};
    it.graph = c;
    it.r0 = r0;
    it.nrows = min(R[c], base[c + 1] - r0);
    it.c0 = INT_MAX;
    it.c1 = 0;
    items[t] = it;
}

// every non-empty row widens its item's window to its first and last column
__global__ void k_win_span(int32_t n, int32_t count, const int32_t* __restrict__ ibase,
                           const int32_t* __restrict__ base, const int32_t* __restrict__ R,
                           const int64_t* __restrict__ prp, const uint32_t* __restrict__ colhop,
                           WinItem* __restrict__ items) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int64_t rs = prp[r], re = prp[r + 1];
    if (rs >= re) return;
    const int32_t c = owner_of(base, count, r);
    WinItem* it = items + ibase[c] + ((int32_t)r - base[c]) / R[c];
    atomicMin(&it->c0, (int32_t)(colhop[rs] & COL_MASK));
    atomicMax(&it->c1, (int32_t)(colhop[re - 1] & COL_MASK) + 1);
}

__global__ void k_win_fix(int32_t nitems, WinItem* __restrict__ items) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nitems && items[t].c0 >= items[t].c1) {
        items[t].c0 = 0;
        items[t].c1 = 0;
    }
}

int32_t build_window_items(drg_ctx* ctx, const drg_sim* s, const std::vector<int32_t>& base,
                           const std::vector<int32_t>& rows_per_item, DevBuf<WinItem>& out) {
    hipStream_t st = ctx->stream;
    const int32_t count = (int32_t)rows_per_item.size();
    if ((int32_t)base.size() != count + 1 || base[count] != s->n)
        throw Error(DRG_E_INVALID, "window items: bad graph bases");
    std::vector<int32_t> ibase(count + 1, 0);
    for (int32_t c = 0; c < count; ++c) {
        const int32_t nc = base[c + 1] - base[c];
        const int64_t k = ((int64_t)nc + rows_per_item[c] - 1) / rows_per_item[c];
        if ((int64_t)ibase[c] + k >= ((int64_t)1 << 31)) throw Error(DRG_E_INVALID, "too many items");
        ibase[c + 1] = ibase[c] + (int32_t)k;
    }
    const int32_t nitems = ibase[count];
    DevBuf<int32_t> dib(count + 1), db(count + 1), dR(count);
    DRG_HIP(hipMemcpyAsync(dib.get(), ibase.data(), sizeof(int32_t) * (count + 1),
                           hipMemcpyHostToDevice, st));
    DRG_HIP(hipMemcpyAsync(db.get(), base.data(), sizeof(int32_t) * (count + 1),
                           hipMemcpyHostToDevice, st));
    DRG_HIP(hipMemcpyAsync(dR.get(), rows_per_item.data(), sizeof(int32_t) * count,
                           hipMemcpyHostToDevice, st));
    out.alloc(std::max(nitems, 1));
    if (nitems > 0) {
        hipLaunchKernelGGL(k_win_items, dim3(ceil_div(nitems, 256)), dim3(256), 0, st, nitems,
                           count, dib.get(), db.get(), dR.get(), out.get());
        DRG_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_win_span, dim3(ceil_div(s->n, 256)), dim3(256), 0, st, s->n, count,
                           dib.get(), db.get(), dR.get(), s->row_ptr.get(), s->colhop.get(),
                           out.get());
        DRG_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_win_fix, dim3(ceil_div(nitems, 256)), dim3(256), 0, st, nitems,
                           out.get());
        DRG_LAUNCH_CHECK();
    }
    DRG_HIP(hipStreamSynchronize(st));
    return nitems;
}

}  // namespace drg

namespace drg {
static int env_int(const char* name, int dflt) {
    const char* v = std::getenv(name);
    return v && *v ? std::atoi(v) : dflt;
}
int win_rpl() {
    const int r = env_int("DRG_WIN_RPL", 4);
    return r >= 8 ? 8 : (r >= 4 ? 4 : (r >= 2 ? 2 : 1));
}
int win_chunk(drg_ctx* ctx) {
    int ch = env_int("DRG_WIN_CH", 8192);
    ch = std::max(256, std::min(ch, (ctx->max_lds - 1024) / 16));
    return ch;
}
// A single graph's records stay in L2 while its rows are swept, where the row
// form gathers them faster than the windowed form stages them (measured on
// RGG, Barabasi-Albert, grid and R-MAT inputs), so the row form is the default.
bool window_wanted(const drg_sim* s) {
    const int f = env_int("DRG_SWEEP_WINDOW", 0);
    return f != 0 && s->nnz > 0;
}
}  // namespace drg
