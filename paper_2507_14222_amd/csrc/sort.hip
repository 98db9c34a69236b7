// Device primitives of libig: fills, exclusive scan and a stable LSD radix sort of
// (u64 key, u32 value) pairs.  Used for candidate de-duplication (Eq. 1 defines
// B^c as a set) and for putting pattern sets in canonical order.
#include "common.h"

namespace ig {

// ------------------------------------------------------------------ fills ----
__global__ void k_fill_u32(uint32_t *p, uint32_t v, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}
__global__ void k_fill_u64(uint64_t *p, uint64_t v, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

static unsigned grid_for(size_t n, unsigned block) {
    size_t g = (n + block - 1) / block;
    if (g > 65535u * 8u) g = 65535u * 8u;
    return (unsigned)(g ? g : 1);
}

void launch_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s) {
    if (!n) return;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
    IG_HIP(hipGetLastError());
}
void launch_fill_u64(uint64_t *p, uint64_t v, size_t n, hipStream_t s) {
    if (!n) return;
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
    IG_HIP(hipGetLastError());
}

// ------------------------------------------------------------------- scan ----
constexpr int SCAN_T = 256;
constexpr int SCAN_I = 16;
constexpr int SCAN_TILE = SCAN_T * SCAN_I;   // 4096 values per workgroup

// inclusive scan of one value per thread across a 256-thread workgroup
__device__ __forceinline__ uint32_t block_incl_scan(uint32_t v, uint32_t *sh /*[4]*/, uint32_t &total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    if (lane == 63) sh[wave] = v;
    __syncthreads();
    uint32_t pre = 0;
    for (int w = 0; w < wave; ++w) pre += sh[w];
    total = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
    return v + pre;
}

// per-tile sums
__global__ __launch_bounds__(SCAN_T) void k_scan_reduce(const uint32_t *in, size_t n, uint32_t *sums) {
    __shared__ uint32_t sh[4];
    size_t base = (size_t)blockIdx.x * SCAN_TILE;
    uint32_t v = 0;
#pragma unroll
    for (int it = 0; it < SCAN_I; ++it) {
        size_t e = base + (size_t)it * SCAN_T + threadIdx.x;
        if (e < n) v += in[e];
    }
    uint32_t tot;
    block_incl_scan(v, sh, tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// exclusive scan of each tile, offset by the (already scanned) tile prefix
// vec: in and out are 16-byte aligned, so a thread's values move as 16-byte loads
// and stores (a quarter of the scattered accesses) wherever all SCAN_I are in range.
__global__ __launch_bounds__(SCAN_T) void k_scan_tiles(const uint32_t *in, uint32_t *out, size_t n,
                                                      const uint32_t *tile_prefix, uint32_t *d_total, bool vec) {
    __shared__ uint32_t sh[4];
    __shared__ uint32_t carry;
    size_t base = (size_t)blockIdx.x * SCAN_TILE;
    if (threadIdx.x == 0) carry = tile_prefix ? tile_prefix[blockIdx.x] : 0u;
    __syncthreads();
    // each thread owns SCAN_I consecutive values: thread-local sums, then one block scan
    static_assert(SCAN_I % 4 == 0, "whole 16-byte pieces per thread");
    uint32_t loc[SCAN_I];
    uint32_t s = 0;
    size_t tb = base + (size_t)threadIdx.x * SCAN_I;
    const bool full = vec && tb + SCAN_I <= n;
    if (full) {
        const uint4 *v4 = reinterpret_cast<const uint4 *>(in + tb);
#pragma unroll
        for (int q = 0; q < SCAN_I / 4; ++q) {
            const uint4 v = v4[q];
            loc[4 * q] = v.x;
            loc[4 * q + 1] = v.y;
            loc[4 * q + 2] = v.z;
            loc[4 * q + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int it = 0; it < SCAN_I; ++it) {
            size_t e = tb + it;
            loc[it] = (e < n) ? in[e] : 0u;
        }
    }
#pragma unroll
    for (int it = 0; it < SCAN_I; ++it) s += loc[it];
    uint32_t tot;
    uint32_t incl = block_incl_scan(s, sh, tot);
    uint32_t run = carry + incl - s;
    if (full) {
        uint4 *o4 = reinterpret_cast<uint4 *>(out + tb);
#pragma unroll
        for (int q = 0; q < SCAN_I / 4; ++q) {
            uint4 v;
            v.x = run;
            run += loc[4 * q];
            v.y = run;
            run += loc[4 * q + 1];
            v.z = run;
            run += loc[4 * q + 2];
            v.w = run;
            run += loc[4 * q + 3];
            o4[q] = v;
        }
    } else {
#pragma unroll
        for (int it = 0; it < SCAN_I; ++it) {
            size_t e = tb + it;
            uint32_t v = loc[it];
            if (e < n) out[e] = run;
            run += v;
        }
    }
    if (d_total && blockIdx.x == gridDim.x - 1 && threadIdx.x == SCAN_T - 1) *d_total = run;
}

static bool aligned16(const void *a, const void *b) {
    return (((uintptr_t)a | (uintptr_t)b) & 15u) == 0;
}

size_t scan_ws_size(size_t n) {
    size_t total = 0;
    while (n > (size_t)SCAN_TILE) {
        n = (n + SCAN_TILE - 1) / SCAN_TILE;
        total += n;
    }
    return total + 1;
}

static void scan_with_ws(const uint32_t *in, uint32_t *out, size_t n, uint32_t *d_total, uint32_t *ws,
                         hipStream_t s) {
    if (n == 0) {
        if (d_total) launch_fill_u32(d_total, 0, 1, s);
        return;
    }
    size_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (tiles == 1) {
        hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(SCAN_T), 0, s, in, out, n, (const uint32_t *)nullptr,
                           d_total, aligned16(in, out));
        IG_HIP(hipGetLastError());
        return;
    }
    uint32_t *sums = ws;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)tiles), dim3(SCAN_T), 0, s, in, n, sums);
    IG_HIP(hipGetLastError());
    scan_with_ws(sums, sums, tiles, nullptr, ws + tiles, s);
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)tiles), dim3(SCAN_T), 0, s, in, out, n, (const uint32_t *)sums,
                       d_total, aligned16(in, out));
    IG_HIP(hipGetLastError());
}

void scan_exclusive_u32(const uint32_t *in, uint32_t *out, size_t n, uint32_t *d_total, hipStream_t s,
                        uint32_t *ws) {
    if (ws) {
        scan_with_ws(in, out, n, d_total, ws, s);
        return;
    }
    Scratch<uint32_t> own(scan_ws_size(n), s);
    scan_with_ws(in, out, n, d_total, own.get(), s);
}

// ------------------------------------------------------------- radix sort ----
// Digit histograms per tile, laid out digit-major ([256][tiles]) so that one
// exclusive scan gives every tile its output offset for every digit; the scatter
// then ranks equal digits stably inside the tile (wave ballots + LDS counts).
constexpr int RS_T = 256;
constexpr int RS_I = 16;
constexpr int RS_TILE = RS_T * RS_I;

__global__ __launch_bounds__(RS_T) void k_rs_hist(const uint64_t *__restrict__ keys, size_t n, int shift,
                                                 uint32_t *__restrict__ hist, uint32_t tiles) {
    __shared__ uint32_t h[4][256];
    const int wave = threadIdx.x >> 6;
    for (int t = threadIdx.x; t < 4 * 256; t += RS_T) (&h[0][0])[t] = 0;
    __syncthreads();
    size_t base = (size_t)blockIdx.x * RS_TILE;
#pragma unroll 4
    for (int it = 0; it < RS_I; ++it) {
        size_t e = base + (size_t)it * RS_T + threadIdx.x;
        if (e < n) {
            uint32_t dg = (uint32_t)(keys[e] >> shift) & 255u;
            atomicAdd(&h[wave][dg], 1u);
        }
    }
    __syncthreads();
    const int t = threadIdx.x;
    hist[(size_t)t * tiles + blockIdx.x] = h[0][t] + h[1][t] + h[2][t] + h[3][t];
}

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int lane = threadIdx.x & 63;
    return lane ? (~0ull >> (64 - lane)) : 0ull;
}

// One tile per workgroup, in two phases.  Ranking: wave w takes elements
// [1024 w, 1024 w + 1024) of the tile, 64 at a time; lanes with equal digits find
// each other with eight ballots, and a per-wave running count per digit (LDS, only
// that wave touches its row) gives each element its stable rank among the wave's
// elements of its digit.  The tile's elements are then placed in LDS in digit order
// (wave-major inside a digit, so input order is kept) and written out from there:
// consecutive threads store consecutive positions of a digit's output run, so the
// stores coalesce instead of landing one element per bucket.  Keys and values pass
// through the same LDS buffer one after the other, which keeps a workgroup at
// 37 KB of LDS (four per CU).
__global__ __launch_bounds__(RS_T) void k_rs_scatter(const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin,
                                                    uint64_t *__restrict__ kout, uint32_t *__restrict__ vout,
                                                    size_t n, int shift, const uint32_t *__restrict__ offs,
                                                    uint32_t tiles) {
    __shared__ uint64_t skey[RS_TILE];   // keys, then the values (as uint32)
    __shared__ uint32_t wcnt[4][256];   // per-wave counts, then per-wave starts in the tile
    __shared__ uint32_t gmap[256];      // output position of tile slot 0 of each digit
    __shared__ uint32_t wsum[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, t = threadIdx.x;
    for (int i = t; i < 4 * 256; i += RS_T) (&wcnt[0][0])[i] = 0;
    __syncthreads();
    const size_t base = (size_t)blockIdx.x * RS_TILE;
    const uint32_t nt = n - base < (size_t)RS_TILE ? (uint32_t)(n - base) : (uint32_t)RS_TILE;
    uint64_t key[RS_I];
    uint32_t val[RS_I], dr[RS_I];   // dr: digit | rank in the wave << 8
#pragma unroll
    for (int it = 0; it < RS_I; ++it) {
        const uint32_t li = (uint32_t)wave * (RS_I * 64) + it * 64 + lane;
        const bool valid = li < nt;
        key[it] = valid ? kin[base + li] : 0ull;
        val[it] = valid ? vin[base + li] : 0u;
        const uint32_t dg = (uint32_t)(key[it] >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (dg >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t before = wcnt[wave][dg];
        const uint32_t rank = before + (uint32_t)__popcll(peers & lanemask_lt());
        // the wave reads its counts before the lowest lane of each digit moves them on
        if (valid && (peers & lanemask_lt()) == 0) wcnt[wave][dg] = before + (uint32_t)__popcll(peers);
        dr[it] = valid ? (dg | rank << 8) : 0xffffffffu;
    }
    __syncthreads();
    // digit t: counts of the four waves, their prefix, and the digit's start in the tile
    const uint32_t c0 = wcnt[0][t], c1 = wcnt[1][t], c2 = wcnt[2][t], c3 = wcnt[3][t];
    const uint32_t tot = c0 + c1 + c2 + c3;
    uint32_t incl = tot;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_up(incl, o, 64);
        if (lane >= o) incl += u;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint32_t start = incl - tot;
    for (int w = 0; w < wave; ++w) start += wsum[w];
    wcnt[0][t] = start;
    wcnt[1][t] = start + c0;
    wcnt[2][t] = start + c0 + c1;
    wcnt[3][t] = start + c0 + c1 + c2;
    gmap[t] = offs[(size_t)t * tiles + blockIdx.x] - start;
    __syncthreads();
    // keys through LDS, then the values through the same buffer
#pragma unroll
    for (int it = 0; it < RS_I; ++it) {
        if (dr[it] == 0xffffffffu) continue;
        skey[wcnt[wave][dr[it] & 255u] + (dr[it] >> 8)] = key[it];
    }
    __syncthreads();
    uint32_t dst[RS_I];
#pragma unroll
    for (int j = 0; j < RS_I; ++j) {
        const uint32_t i = t + j * RS_T;
        if (i < nt) {
            const uint64_t k = skey[i];
            dst[j] = gmap[(uint32_t)(k >> shift) & 255u] + i;
            kout[dst[j]] = k;
        }
    }
    __syncthreads();
    uint32_t *sv = reinterpret_cast<uint32_t *>(skey);
#pragma unroll
    for (int it = 0; it < RS_I; ++it) {
        if (dr[it] == 0xffffffffu) continue;
        sv[wcnt[wave][dr[it] & 255u] + (dr[it] >> 8)] = val[it];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < RS_I; ++j) {
        const uint32_t i = t + j * RS_T;
        if (i < nt) vout[dst[j]] = sv[i];
    }
}

size_t radix_ws_size(size_t n) {
    const size_t tiles = (n + RS_TILE - 1) / RS_TILE;
    return tiles * 256 + scan_ws_size(tiles * 256);
}

int radix_sort_pairs(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, size_t n, uint32_t digit_mask,
                     hipStream_t s, uint32_t *ws) {
    if (n <= 1 || digit_mask == 0) return 0;
    IG_REQUIRE(n < (1ull << 32), IG_E_UNSUPPORTED, "radix sort of more than 2^32 elements");
    const size_t tiles = (n + RS_TILE - 1) / RS_TILE;
    Scratch<uint32_t> own;
    if (!ws) {
        own.reset(radix_ws_size(n), s);
        ws = own.get();
    }
    uint32_t *hist = ws, *scan_ws = ws + tiles * 256;
    uint64_t *ka = k0, *kb = k1;
    uint32_t *va = v0, *vb = v1;
    int cur = 0;
    for (int pass = 0; pass < 8; ++pass) {
        if (!((digit_mask >> pass) & 1u)) continue;
        int shift = pass * 8;
        hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)tiles), dim3(RS_T), 0, s, ka, n, shift, hist, (uint32_t)tiles);
        IG_HIP(hipGetLastError());
        scan_exclusive_u32(hist, hist, tiles * 256, nullptr, s, scan_ws);
        hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)tiles), dim3(RS_T), 0, s, ka, va, kb, vb, n, shift,
                           (const uint32_t *)hist, (uint32_t)tiles);
        IG_HIP(hipGetLastError());
        std::swap(ka, kb);
        std::swap(va, vb);
        cur ^= 1;
    }
    return cur;
}

}  // namespace ig
