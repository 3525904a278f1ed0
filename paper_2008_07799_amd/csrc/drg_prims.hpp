// drg_prims.hpp -- device-wide building blocks used by the build stages.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace drg {

// Where device memory comes from: a caller's allocator (set on the context,
// see drg_allocator) or, when alloc is NULL, hipMalloc / hipFree.
struct Allocator {
    void* (*alloc)(size_t bytes, void* user) = nullptr;
    void (*free)(void* ptr, void* user) = nullptr;
    void* user = nullptr;
};

// The allocator of the entry point running on this thread: the context's,
// for the duration of a call on a context; else the default.
Allocator& thread_allocator();

void* dev_alloc_bytes(int64_t bytes, const Allocator& al);

// RAII device buffer; freed with the allocator it came from.
template <typename T>
struct DevBuf {
    T* p = nullptr;
    int64_t n = 0;
    Allocator al;
    DevBuf() = default;
    explicit DevBuf(int64_t count) { alloc(count); }
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n), al(o.al) {
        o.p = nullptr;
        o.n = 0;
    }
    DevBuf& operator=(DevBuf&& o) noexcept {
        if (this != &o) {
            reset();
            p = o.p;
            n = o.n;
            al = o.al;
            o.p = nullptr;
            o.n = 0;
        }
        return *this;
    }
    ~DevBuf() { reset(); }
    void alloc(int64_t count);
    void reset() {
        if (p) {
            if (al.free)
                al.free(p, al.user);
            else
                (void)hipFree(p);
        }
        p = nullptr;
        n = 0;
    }
    T* get() const { return p; }
};

template <typename T>
void DevBuf<T>::alloc(int64_t count) {
    reset();
    const Allocator use = thread_allocator();
    p = static_cast<T*>(dev_alloc_bytes((count > 0 ? count : 1) * (int64_t)sizeof(T), use));
    al = use;
    n = count;
}

// out[0..n] = exclusive prefix sums of in[0..n), out[n] = total.  out may
// alias in only if it is a distinct buffer of n+1 elements (not in place).
template <typename T>
void exclusive_scan(const T* in, T* out, int64_t n, hipStream_t s);

// Stable sort of (key, value) pairs by the low key_bits bits of the key.
void radix_sort_pairs(uint32_t* keys, int32_t* vals, int64_t n, int key_bits, hipStream_t s);

// Number of i in [0, n) with rp[i+1] > rp[i].
template <typename T>
int64_t count_nonempty_rows(const T* rp, int64_t n, hipStream_t s);

// out[g] = sum of squared row lengths of group g (gid NULL: one group, out[0]).
// Enqueued on s, no wait.
void sum_len2_by_group(const int64_t* rp, const int32_t* gid, int64_t n, unsigned long long* out,
                       int32_t groups, hipStream_t s);
// cnt[c] = number of i in [0, n) with gid[i] == c and rp[i+1] > rp[i], for
// c in [0, groups); gid[i] must lie in [0, groups).  Enqueued on s, no wait.
template <typename T>
void count_nonempty_by_group(const T* rp, const int32_t* gid, int64_t n, int32_t* cnt,
                             int32_t groups, hipStream_t s);

}  // namespace drg
