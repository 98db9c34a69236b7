// Internal declarations of libig (HIP, gfx950).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <utility>

#include "../../include/ig.h"

namespace ig {

// ----------------------------------------------------------------- errors ----
struct Error : std::runtime_error {
    ig_status code;
    Error(ig_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define IG_HIP(call)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            throw ::ig::Error(IG_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define IG_REQUIRE(cond, code, msg)                                                      \
    do {                                                                                 \
        if (!(cond)) throw ::ig::Error((code), (msg));                                   \
    } while (0)

// ------------------------------------------------------------ device memory ----
// (memory.cpp) Stream-ordered scratch from a per-device block cache over the
// library's arena: a block freed on one stream is handed to a later allocation
// only after that allocation's stream has been made to wait for the freeing
// stream's work.  While a UserAllocScope with a caller allocator is alive on the
// thread, scratch comes from that allocator instead.
void *scratch_alloc(size_t bytes, hipStream_t s);
void scratch_free(void *p, hipStream_t s) noexcept;
// Long-lived buffers (models): from `user` when non-null, else the arena of the
// current device; device_free takes the device the buffer was allocated on.
void *device_alloc(size_t bytes, hipStream_t s, const ig_allocator *user);
void device_free(void *p, int dev, const ig_allocator *user) noexcept;
// The caller allocator of the running call (null: the library's arena).
struct UserAllocScope {
    const ig_allocator *prev;
    explicit UserAllocScope(const ig_allocator *a);
    ~UserAllocScope();
    UserAllocScope(const UserAllocScope &) = delete;
    UserAllocScope &operator=(const UserAllocScope &) = delete;
};
const ig_allocator *current_user_allocator();
// Cached scratch and wholly free arena chunks of the current device back to the
// runtime; the arena's sizes on the current device.
void release_memory();
void memory_stats(uint64_t *reserved, uint64_t *in_use, uint64_t *cached);
// bytes from host memory to device memory, queued on s (the host memory may be
// reused as soon as the call returns: small copies go through pinned staging)
void upload(void *dst, const void *src, size_t bytes, hipStream_t s);

template <class T>
struct Scratch {
    T *p = nullptr;
    size_t n = 0;
    hipStream_t s = nullptr;
    Scratch() = default;
    Scratch(size_t count, hipStream_t st) { reset(count, st); }
    void reset(size_t count, hipStream_t st) {
        release();
        s = st;
        n = count;
        p = count ? static_cast<T *>(scratch_alloc(count * sizeof(T), st)) : nullptr;
    }
    void release() {
        if (p) scratch_free(p, s);
        p = nullptr;
        n = 0;
    }
    ~Scratch() { scratch_free(p, s); }
    Scratch(const Scratch &) = delete;
    Scratch &operator=(const Scratch &) = delete;
    Scratch(Scratch &&o) noexcept : p(o.p), n(o.n), s(o.s) { o.p = nullptr; o.n = 0; }
    Scratch &operator=(Scratch &&o) noexcept {
        if (this != &o) { release(); p = o.p; n = o.n; s = o.s; o.p = nullptr; o.n = 0; }
        return *this;
    }
    T *get() const { return p; }
};

// ------------------------------------------------------------- word widths ----
// Kernels that hold bitsets in registers are compiled for a fixed storage width
// KS (64-bit words); a problem with K words uses the smallest KS >= K and zero
// padding (complemented rows pad with all-ones, so padding never matters).
int storage_words(int K);   // KS for K (1..64), or -1

// ------------------------------------------------------------ fit segments ----
// One (problem, class) of a fit.  All pointers are device pointers.
struct Seg {
    const uint64_t *X;     // class rows [n][KS] in input order
    const uint64_t *NX;    // complement of X
    const uint64_t *NXo;   // complement of the other class's rows [n_o][KS]
    uint32_t n, n_o;
    uint32_t KS, K;
    const uint32_t *cand;  // distinct candidate pair ids of the current chunk
    uint32_t *surv;        // coherent pair ids (appended)
    uint32_t *nsurv;       // device counter of surv
    unsigned long long *tests;  // device sum of t(b)
};

// Pair id q of a class with n records: q < n is record q itself, otherwise
// q - n indexes the pairs (i, j), i < j, in the order j = 1, 2, ...; i = 0..j-1.
__device__ __forceinline__ void decode_pair(uint64_t q, uint32_t n, uint32_t &i, uint32_t &j) {
    if (q < n) { i = j = (uint32_t)q; return; }
    uint64_t p = q - n;
    // a single-precision estimate (within one of the root for p < 2^40), then exact
    // integer correction
    uint64_t jj = (uint64_t)((1.0f + sqrtf(1.0f + 8.0f * (float)p)) * 0.5f);
    while (jj * (jj - 1) / 2 > p) --jj;
    while ((jj + 1) * jj / 2 <= p) ++jj;
    i = (uint32_t)(p - jj * (jj - 1) / 2);
    j = (uint32_t)jj;
}

// ----------------------------------------------------------- launch helpers ----
void launch_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s);
void launch_fill_u64(uint64_t *p, uint64_t v, size_t n, hipStream_t s);

// exclusive prefix sum of n u32 values (out may alias in); total written to *d_total if
// non-null.  ws: scan_ws_size(n) u32 of scratch, or null to allocate it on the stream.
size_t scan_ws_size(size_t n);
void scan_exclusive_u32(const uint32_t *in, uint32_t *out, size_t n, uint32_t *d_total, hipStream_t s,
                        uint32_t *ws = nullptr);

// Stable LSD radix sort of (u64 key, u32 val) pairs, 8 bits per pass.  Ping-pongs
// between (k0,v0) and (k1,v1); returns 0 when the result is in (k0,v0), 1 when in
// (k1,v1).  digit_mask bit p set = pass p (bits [8p, 8p+8)) runs; clear bits mark
// digits known to be constant.  ws: radix_ws_size(n) u32 of scratch, or null to
// allocate it on the stream (a captured sequence must pass it).
size_t radix_ws_size(size_t n);
int radix_sort_pairs(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, size_t n,
                     uint32_t digit_mask, hipStream_t s, uint32_t *ws = nullptr);

}  // namespace ig
