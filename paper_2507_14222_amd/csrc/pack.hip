// Packing of records into bitsets (Section 3.2, Eq. 5) and the class split
// (rows stacked by class, Section 3.2).  Token of feature f, bin c: off[f] + c;
// token j is bit j%64 of word j/64.
#include "common.h"
#include "kernels.h"

namespace ig {

// Every code must be below its feature's bin count; every label 0 or 1.
__global__ void k_validate_codes(const uint16_t *__restrict__ codes, size_t total, uint32_t d,
                                 const uint16_t *__restrict__ nbins, uint32_t *__restrict__ err) {
    size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    uint32_t bad = 0;
    for (; g < total; g += stride) {
        uint32_t f = (uint32_t)(g % d);
        bad |= codes[g] >= nbins[f];
    }
    if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(err, 1u);
}

// Stable split by label: pos[i] = rank of record i among records of its class.
// One workgroup of 1024 threads walks the records in order.
__global__ __launch_bounds__(1024) void k_split_labels(const uint8_t *__restrict__ labels, uint32_t n,
                                                      uint32_t *__restrict__ pos, uint32_t *__restrict__ counts,
                                                      uint32_t *__restrict__ err) {
    __shared__ uint32_t wsum[16];
    __shared__ uint32_t ones_run;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) ones_run = 0;
    __syncthreads();
    uint32_t bad = 0;
    for (uint32_t base = 0; base < n; base += 1024) {
        uint32_t g = base + threadIdx.x;
        uint32_t l = g < n ? labels[g] : 0u;
        bad |= (g < n) && (l > 1u);
        bool one = (g < n) && (l == 1u);
        uint64_t m = __ballot(one);
        uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
        uint32_t before_in_wave = (uint32_t)__popcll(m & lt);
        if (lane == 0) wsum[wave] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t before = ones_run + before_in_wave;
        for (int w = 0; w < wave; ++w) before += wsum[w];
        if (g < n) pos[g] = one ? before : g - before;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t t = 0;
            for (int w = 0; w < 16; ++w) t += wsum[w];
            ones_run += t;
        }
        __syncthreads();
    }
    if (__ballot(bad) && lane == 0) atomicOr(err, 2u);
    if (threadIdx.x == 0) {
        counts[1] = ones_run;
        counts[0] = n - ones_run;
    }
}

// One thread per (record, storage word).  meta = [off(d) | flo(KS) | fhi(KS)]:
// features [flo[k], fhi[k]) are the ones whose token range meets word k.
__global__ void k_pack_split(const uint16_t *__restrict__ codes, const uint8_t *__restrict__ labels, uint32_t n,
                             uint32_t d, uint32_t KS, const uint32_t *__restrict__ meta,
                             const uint32_t *__restrict__ pos, uint64_t *__restrict__ X0, uint64_t *__restrict__ X1,
                             uint64_t *__restrict__ NX0, uint64_t *__restrict__ NX1) {
    size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (size_t)n * KS) return;
    uint32_t i = (uint32_t)(g / KS), k = (uint32_t)(g % KS);
    const uint32_t *off = meta, *flo = meta + d, *fhi = meta + d + KS;
    uint64_t w = 0;
    for (uint32_t f = flo[k]; f < fhi[k]; ++f) {
        uint32_t bit = off[f] + codes[(size_t)i * d + f];
        if ((bit >> 6) == k) w |= 1ull << (bit & 63);
    }
    size_t r = (size_t)pos[i] * KS + k;
    if (labels[i]) { X1[r] = w; NX1[r] = ~w; }
    else { X0[r] = w; NX0[r] = ~w; }
}

// Class split of rows given already packed ([n][K] words, stored with width KS).
__global__ void k_split_packed(const uint64_t *__restrict__ words, const uint8_t *__restrict__ labels, uint32_t n,
                               uint32_t K, uint32_t KS, const uint32_t *__restrict__ pos, uint64_t *__restrict__ X0,
                               uint64_t *__restrict__ X1, uint64_t *__restrict__ NX0, uint64_t *__restrict__ NX1) {
    size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (size_t)n * KS) return;
    uint32_t i = (uint32_t)(g / KS), k = (uint32_t)(g % KS);
    uint64_t w = k < K ? words[(size_t)i * K + k] : 0ull;
    size_t r = (size_t)pos[i] * KS + k;
    if (labels[i]) { X1[r] = w; NX1[r] = ~w; }
    else { X0[r] = w; NX0[r] = ~w; }
}

// Pattern code rows (IG_ABSENT = feature not present) -> words [m][KS].
// err bit 1: a code out of range; bit 2: a pattern with no token.
__global__ void k_pack_patterns(const uint16_t *__restrict__ codes, uint32_t m, uint32_t d, uint32_t KS,
                                const uint32_t *__restrict__ meta, const uint16_t *__restrict__ nbins,
                                uint64_t *__restrict__ W, uint32_t *__restrict__ err) {
    size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (size_t)m) return;
    const uint32_t *off = meta, *flo = meta + d, *fhi = meta + d + KS;
    uint32_t bad = 0, any = 0;
    for (uint32_t k = 0; k < KS; ++k) {
        uint64_t w = 0;
        for (uint32_t f = flo[k]; f < fhi[k]; ++f) {
            uint32_t c = codes[g * d + f];
            if (c == IG_ABSENT) continue;
            if (c >= nbins[f]) { bad = 1; continue; }
            uint32_t bit = off[f] + c;
            if ((bit >> 6) == k) w |= 1ull << (bit & 63);
        }
        any |= w != 0;
        W[g * KS + k] = w;
    }
    if (bad) atomicOr(err, 1u);
    if (!any) atomicOr(err, 2u);
}

void launch_validate_codes(const uint16_t *codes, size_t total, uint32_t d, const uint16_t *nbins, uint32_t *err,
                           hipStream_t s) {
    if (!total) return;
    size_t g = (total + 255) / 256;
    if (g > 16384) g = 16384;
    hipLaunchKernelGGL(k_validate_codes, dim3((unsigned)g), dim3(256), 0, s, codes, total, d, nbins, err);
    IG_HIP(hipGetLastError());
}

void launch_split_labels(const uint8_t *labels, uint32_t n, uint32_t *pos, uint32_t *counts, uint32_t *err,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_split_labels, dim3(1), dim3(1024), 0, s, labels, n, pos, counts, err);
    IG_HIP(hipGetLastError());
}

void launch_pack_split(const uint16_t *codes, const uint8_t *labels, uint32_t n, uint32_t d, uint32_t KS,
                       const uint32_t *meta, const uint32_t *pos, uint64_t *X0, uint64_t *X1, uint64_t *NX0,
                       uint64_t *NX1, hipStream_t s) {
    size_t total = (size_t)n * KS;
    if (!total) return;
    hipLaunchKernelGGL(k_pack_split, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, codes, labels, n, d, KS,
                       meta, pos, X0, X1, NX0, NX1);
    IG_HIP(hipGetLastError());
}

void launch_split_packed(const uint64_t *words, const uint8_t *labels, uint32_t n, uint32_t K, uint32_t KS,
                         const uint32_t *pos, uint64_t *X0, uint64_t *X1, uint64_t *NX0, uint64_t *NX1,
                         hipStream_t s) {
    size_t total = (size_t)n * KS;
    if (!total) return;
    hipLaunchKernelGGL(k_split_packed, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, words, labels, n, K,
                       KS, pos, X0, X1, NX0, NX1);
    IG_HIP(hipGetLastError());
}

void launch_pack_patterns(const uint16_t *codes, uint32_t m, uint32_t d, uint32_t KS, const uint32_t *meta,
                          const uint16_t *nbins, uint64_t *W, uint32_t *err, hipStream_t s) {
    if (!m) return;
    hipLaunchKernelGGL(k_pack_patterns, dim3((m + 255) / 256), dim3(256), 0, s, codes, m, d, KS, meta, nbins, W, err);
    IG_HIP(hipGetLastError());
}

}  // namespace ig
