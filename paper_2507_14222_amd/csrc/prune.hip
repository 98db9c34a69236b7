// Exact pruning of the scoring contraction (Eq. 4) by token buckets.
//
// A pattern b adds its weight to A(t) or N(t) only when it lies inside the flow t,
// that is when t holds every token of b (Eq. 6).  Each pattern of a model is put
// into the bucket of one of its tokens (the one whose training frequency is
// lowest, so that few flows hold it); a flow is then tested only against the
// buckets of the d tokens it holds, one per feature, and every other pattern is
// known to lie outside it.  The sums are the same integers as the dense
// contraction's: no pattern inside a flow is ever skipped.
//
// Model side (once per model): k_token_counts, k_bucket_keys, k_bucket_first.
// Call side (per scoring call, in caller-provided or library scratch):
// k_prune_count -> k_prune_plan -> k_prune_scatter -> k_score_mfma_pruned.
//
// The fit's contractions are pruned the same way (Eq. 3 and Eq. 2 test whether a
// record contains a candidate, which needs every token of the candidate in the
// record): the records of the tested class are listed under each token they hold
// (k_bucket_records), a candidate goes to the bucket of its token held by the
// fewest of those records (k_cand_bucket_keys, k_bucket_place), and
// k_contain_mfma_pruned tests it against that bucket's records only.  Bucket L
// lists every record: it takes the candidates without a token (the empty set,
// which every record contains).
#include "common.h"
#include "kernels.h"

namespace ig {

constexpr uint32_t kMaxBuckets = 4096;   // L <= 4096 tokens

// cnt[u] += the records of X [n][KS] holding token u (bits of the first L tokens)
__global__ void k_token_counts(const uint64_t *__restrict__ X, uint32_t n, uint32_t KS, uint32_t L,
                               uint32_t *__restrict__ cnt) {
    __shared__ uint32_t h[kMaxBuckets];
    for (uint32_t u = threadIdx.x; u < L; u += blockDim.x) h[u] = 0;
    __syncthreads();
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        for (uint32_t k = 0; k < KS; ++k) {
            uint64_t w = X[(size_t)i * KS + k];
            while (w) {
                const uint32_t tok = 64 * k + (uint32_t)__builtin_ctzll(w);
                w &= w - 1;
                if (tok < L) atomicAdd(&h[tok], 1u);
            }
        }
    }
    __syncthreads();
    for (uint32_t u = threadIdx.x; u < L; u += blockDim.x)
        if (h[u]) atomicAdd(&cnt[u], h[u]);
}

// key[e] = the bucket token of pattern row e of W [m][KS]: its token with the
// smallest cost, the lowest such token on ties.  A row without a token below L
// (never produced: the empty set is not a pattern) sets *err.
__global__ void k_bucket_keys(const uint64_t *__restrict__ W, size_t m, uint32_t KS, uint32_t L,
                              const uint32_t *__restrict__ cost, uint64_t *__restrict__ key,
                              uint32_t *__restrict__ err) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    uint32_t best = ~0u, bc = ~0u;
    for (uint32_t k = 0; k < KS; ++k) {
        uint64_t w = W[e * KS + k];
        while (w) {
            const uint32_t tok = 64 * k + (uint32_t)__builtin_ctzll(w);
            w &= w - 1;
            if (tok >= L) break;
            const uint32_t c = cost[tok];
            if (c < bc) {   // tokens come in ascending order: ties keep the lowest
                bc = c;
                best = tok;
            }
        }
    }
    if (best == ~0u) {
        atomicOr(err, 1u);
        best = 0;
    }
    key[e] = best;
}

// first[u] = the first position of bucket u in the ascending keys (entries of empty
// buckets are left as preset)
__global__ void k_bucket_first(const uint64_t *__restrict__ key, size_t m, uint32_t *__restrict__ first) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    if (e == 0 || key[e] != key[e - 1]) first[key[e]] = (uint32_t)e;
}

void launch_token_counts(const uint64_t *X, uint32_t n, uint32_t KS, uint32_t L, uint32_t *cnt, hipStream_t s) {
    if (!n) return;
    IG_REQUIRE(L <= kMaxBuckets, IG_E_UNSUPPORTED, "more than 4096 tokens");
    const uint32_t blocks = std::min<uint32_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(k_token_counts, dim3(blocks), dim3(256), 0, s, X, n, KS, L, cnt);
    IG_HIP(hipGetLastError());
}

void launch_bucket_keys(const uint64_t *W, size_t m, uint32_t KS, uint32_t L, const uint32_t *cost, uint64_t *key,
                        uint32_t *err, hipStream_t s) {
    if (!m) return;
    hipLaunchKernelGGL(k_bucket_keys, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, W, m, KS, L, cost, key,
                       err);
    IG_HIP(hipGetLastError());
}

void launch_bucket_first(const uint64_t *key, size_t m, uint32_t *first, hipStream_t s) {
    if (!m) return;
    hipLaunchKernelGGL(k_bucket_first, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, key, m, first);
    IG_HIP(hipGetLastError());
}

// ---------------------------------------------------- fit contractions ----
// Elements are grouped by key with one histogram per workgroup of BK_T * iters elements
// (whist, key-major: [key][workgroup]), whose exclusive scan gives each
// (key, workgroup) its first output position; k_bucket_place then puts each
// workgroup's elements there (their order inside a key is not fixed, and no
// result depends on it).
constexpr uint32_t BK_T = 256;
// elements per thread: more for large inputs, so that there are fewer (key,
// workgroup) cells to write, scan and read back
static uint32_t bucket_iters(size_t m) { return m >= (1u << 22) ? 32u : 8u; }

__device__ __forceinline__ void bucket_hist_out(uint32_t *h, uint32_t L, uint32_t *whist, uint32_t nwg) {
    __syncthreads();
    for (uint32_t u = threadIdx.x; u <= L; u += BK_T) whist[(size_t)u * nwg + blockIdx.x] = h[u];
}

// Lanes of the wave whose key (< 2^13) equals this lane's, among the active ones:
// one ballot per key bit.
__device__ __forceinline__ uint64_t key_peers(uint32_t k, bool active) {
    uint64_t peers = __ballot(active);
#pragma unroll
    for (int b = 0; b < 13; ++b) {
        const bool bit = (k >> b) & 1u;
        const uint64_t m = __ballot(bit);
        peers &= bit ? m : ~m;
    }
    return peers;
}

__device__ __forceinline__ uint64_t lanes_below() {
    const int lane = threadIdx.x & 63;
    return lane ? (~0ull >> (64 - lane)) : 0ull;
}

// Adds this lane's element to h[k] with one LDS atomic per distinct key of the wave
// (the lowest lane of each key adds for all); returns the element's place among
// the workgroup's elements of key k.  Every lane of the wave calls it.
__device__ __forceinline__ uint32_t group_add(uint32_t *h, uint32_t k, bool active) {
    const uint64_t peers = key_peers(k, active);
    const uint64_t below = peers & lanes_below();
    const int leader = peers ? __builtin_ctzll(peers) : 0;
    uint32_t base = 0;
    if (active && !below) base = atomicAdd(&h[k], (uint32_t)__popcll(peers));
    base = (uint32_t)__shfl((int)base, leader, 64);
    return base + (uint32_t)__popcll(below);
}

// Xr [n][KSr] (zero at launch): bit rank[t] for each token t < L of record r of
// X [n][KS] -- the records' tokens renumbered so that a lower number is a token
// held by fewer records of the tested class.  One thread per (record, word).
__global__ void k_rank_rows(const uint64_t *__restrict__ X, uint32_t n, uint32_t KS, uint32_t L,
                            const uint16_t *__restrict__ rank, uint32_t KSr, unsigned long long *__restrict__ Xr) {
    const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (size_t)n * KS) return;
    const uint32_t r = (uint32_t)(g / KS), w = (uint32_t)(g % KS);
    uint64_t x = X[g];
    while (x) {
        const uint32_t t = 64 * w + (uint32_t)__builtin_ctzll(x);
        x &= x - 1;
        if (t >= L) break;
        const uint32_t q = rank[t];
        atomicOr(&Xr[(size_t)r * KSr + (q >> 6)], 1ull << (q & 63));
    }
}

// key[e] = the bucket of candidate e, the pair id ids[e] of records i, j: the
// token inv[q] of the lowest renumbered token q both hold in Xr (L when none: the
// empty set).  One thread per candidate (its loads wait on each other, so many
// candidates in flight hide them); the histogram is a pass of its own.
__global__ __launch_bounds__(256) void k_cand_keys_rank(const uint64_t *__restrict__ Xr, uint32_t n, uint32_t KSr,
                                                        const uint32_t *__restrict__ ids, size_t m, uint32_t L,
                                                        const uint16_t *__restrict__ inv, uint32_t *__restrict__ key) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    uint32_t i, j, best = L;
    decode_pair(ids[e], n, i, j);
    const uint64_t *xi = Xr + (size_t)i * KSr, *xj = Xr + (size_t)j * KSr;
    for (uint32_t w = 0; w < KSr; ++w) {
        const uint64_t x = xi[w] & xj[w];
        if (x) {
            best = inv[64 * w + (uint32_t)__builtin_ctzll(x)];
            break;
        }
    }
    key[e] = best;
}

// Per-workgroup histogram of the keys (key <= L) into whist.
__global__ __launch_bounds__(BK_T) void k_key_hist(const uint32_t *__restrict__ key, size_t m, uint32_t L,
                                                   uint32_t *__restrict__ whist, uint32_t nwg, uint32_t iters) {
    __shared__ uint32_t h[kMaxBuckets + 1];
    for (uint32_t u = threadIdx.x; u <= L; u += BK_T) h[u] = 0;
    __syncthreads();
    const size_t base = (size_t)blockIdx.x * BK_T * iters;
    for (uint32_t it = 0; it < iters; ++it) {
        const size_t e = base + (size_t)it * BK_T + threadIdx.x;
        const bool act = e < m;
        group_add(h, act ? key[e] : L, act);
    }
    bucket_hist_out(h, L, whist, nwg);
}

// The same from one-hot rows W [m][KS]: the row's token of the lowest rank.
__global__ __launch_bounds__(BK_T) void k_row_keys_rank(const uint64_t *__restrict__ W, size_t m, uint32_t KS,
                                                        uint32_t L, const uint16_t *__restrict__ rank,
                                                        const uint16_t *__restrict__ inv, uint32_t *__restrict__ key,
                                                        uint32_t *__restrict__ whist, uint32_t nwg, uint32_t iters) {
    __shared__ uint32_t h[kMaxBuckets + 1];
    __shared__ uint16_t rk[kMaxBuckets];
    for (uint32_t u = threadIdx.x; u <= L; u += BK_T) h[u] = 0;
    for (uint32_t u = threadIdx.x; u < L; u += BK_T) rk[u] = rank[u];
    __syncthreads();
    const size_t base = (size_t)blockIdx.x * BK_T * iters;
    for (uint32_t it = 0; it < iters; ++it) {
        const size_t e = base + (size_t)it * BK_T + threadIdx.x;
        const bool act = e < m;
        uint32_t best = L;
        if (act) {
            for (uint32_t k = 0; k < KS; ++k) {
                uint64_t w = W[e * KS + k];
                while (w) {
                    const uint32_t tok = 64 * k + (uint32_t)__builtin_ctzll(w);
                    w &= w - 1;
                    if (tok >= L) break;
                    best = min(best, (uint32_t)rk[tok]);
                }
            }
            if (best < L) best = inv[best];
            key[e] = best;
        }
        group_add(h, best, act);
    }
    bucket_hist_out(h, L, whist, nwg);
}

// key[r * d + k] = token k (ascending) of record r of X [n][KS], d per record;
// per-workgroup histogram in whist.
__global__ __launch_bounds__(BK_T) void k_record_keys(const uint64_t *__restrict__ X, uint32_t n, uint32_t KS,
                                                      uint32_t L, uint32_t d, uint32_t *__restrict__ key,
                                                      uint32_t *__restrict__ whist, uint32_t nwg, uint32_t iters) {
    __shared__ uint32_t h[kMaxBuckets + 1];
    for (uint32_t u = threadIdx.x; u <= L; u += BK_T) h[u] = 0;
    __syncthreads();
    const size_t base = (size_t)blockIdx.x * BK_T * iters, m = (size_t)n * d;
    for (uint32_t it = 0; it < iters; ++it) {
        const size_t e = base + (size_t)it * BK_T + threadIdx.x;
        if (e >= m) break;
        const uint32_t r = (uint32_t)(e / d), k = (uint32_t)(e % d);
        // the k-th set bit of the row
        uint32_t t = L, seen = 0;
        for (uint32_t w = 0; w < KS; ++w) {
            const uint64_t x = X[(size_t)r * KS + w];
            const uint32_t c = (uint32_t)__popcll(x);
            if (k < seen + c) {
                uint64_t y = x;
                for (uint32_t q = seen; q < k; ++q) y &= y - 1;
                t = 64 * w + (uint32_t)__builtin_ctzll(y);
                break;
            }
            seen += c;
        }
        if (t > L) t = L;
        key[e] = t;
        atomicAdd(&h[t], 1u);
    }
    bucket_hist_out(h, L, whist, nwg);
}

// out[pos[key][wg] + place] = e / div for the elements e of workgroup wg (pos:
// the exclusive scan of whist; out may be null), and out2 there = src[e] when src
// is given.  The
// workgroup's cursors start at its column of pos, so the place is the cursor.
__global__ __launch_bounds__(BK_T) void k_bucket_place(const uint32_t *__restrict__ key, size_t m, uint32_t L,
                                                       const uint32_t *__restrict__ pos, uint32_t nwg, uint32_t div,
                                                       uint32_t *__restrict__ out, const uint32_t *__restrict__ src,
                                                       uint32_t *__restrict__ out2, uint32_t iters) {
    __shared__ uint32_t h[kMaxBuckets + 1];
    for (uint32_t u = threadIdx.x; u <= L; u += BK_T) h[u] = pos[(size_t)u * nwg + blockIdx.x];
    __syncthreads();
    const size_t base = (size_t)blockIdx.x * BK_T * iters;
    for (uint32_t it = 0; it < iters; ++it) {
        const size_t e = base + (size_t)it * BK_T + threadIdx.x;
        const bool act = e < m;
        const uint32_t k = act ? key[e] : L;
        const uint32_t p = group_add(h, k, act);
        if (act) {
            if (out) out[p] = (uint32_t)(e / div);
            if (src) out2[p] = src[e];
        }
    }
}

// first[u] = pos[u * nwg] for u <= L, first[L + 1] = m: each key's first position.
__global__ void k_bucket_starts(const uint32_t *__restrict__ pos, uint32_t nwg, uint32_t L, uint32_t m,
                                uint32_t *__restrict__ first) {
    const uint32_t u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u <= L) first[u] = pos[(size_t)u * nwg];
    if (u == L + 1) first[u] = m;
}

uint32_t bucket_groups(size_t m) {
    const size_t e = (size_t)BK_T * bucket_iters(m);
    return (uint32_t)((m + e - 1) / e);
}

size_t bucket_ws_words(size_t m, uint32_t L) {
    const size_t cells = (size_t)(L + 1) * std::max<uint32_t>(bucket_groups(m), 1);
    return 2 * cells + scan_ws_size(cells);
}

// Groups the m keyed elements (whist filled by a key kernel over bucket_groups(m)
// workgroups): out[...] = e / div grouped by key, first [L + 2] = each key's first
// position.  ws: bucket_ws_words(m, L) u32.
static void bucket_group(const uint32_t *key, size_t m, uint32_t L, uint32_t *whist, uint32_t div, uint32_t *out,
                         uint32_t *first, uint32_t *ws, hipStream_t s, const uint32_t *src = nullptr,
                         uint32_t *out2 = nullptr) {
    const uint32_t nwg = std::max<uint32_t>(bucket_groups(m), 1);
    const size_t cells = (size_t)(L + 1) * nwg;
    uint32_t *pos = ws + cells;
    scan_exclusive_u32(whist, pos, cells, nullptr, s, ws + 2 * cells);
    hipLaunchKernelGGL(k_bucket_starts, dim3((L + 2 + 255) / 256), dim3(256), 0, s, pos, nwg, L, (uint32_t)m, first);
    IG_HIP(hipGetLastError());
    if (m)
        hipLaunchKernelGGL(k_bucket_place, dim3(nwg), dim3(BK_T), 0, s, key, m, L, pos, nwg, div, out, src, out2,
                           bucket_iters(m));
    IG_HIP(hipGetLastError());
}

void launch_rank_rows(const uint64_t *X, uint32_t n, uint32_t KS, uint32_t L, const uint16_t *rank, uint32_t KSr,
                      uint64_t *Xr, hipStream_t s) {
    IG_REQUIRE(L >= 1 && L <= kMaxBuckets && KSr * 64 >= L, IG_E_UNSUPPORTED, "token buckets need 1 to 4096 tokens");
    launch_fill_u64(Xr, 0ull, std::max<size_t>((size_t)n * KSr, 1), s);
    const size_t g = (size_t)n * KS;
    if (!g) return;
    hipLaunchKernelGGL(k_rank_rows, dim3((unsigned)((g + 255) / 256)), dim3(256), 0, s, X, n, KS, L, rank, KSr,
                       reinterpret_cast<unsigned long long *>(Xr));
    IG_HIP(hipGetLastError());
}

void launch_group_candidates(const uint64_t *Xr, uint32_t n, uint32_t KSr, const uint32_t *ids, const uint64_t *W,
                             uint32_t KS, size_t m, uint32_t L, const uint16_t *rank, const uint16_t *inv,
                             uint32_t *key, uint32_t *perm, uint32_t *first, uint32_t *ws, hipStream_t s,
                             uint32_t *ids_out) {
    IG_REQUIRE(L >= 1 && L <= kMaxBuckets, IG_E_UNSUPPORTED, "token buckets need 1 to 4096 tokens");
    IG_REQUIRE(inv && ((ids && Xr) || (!ids && W && rank)), IG_E_INVAL,
               "candidates need pair ids and ranked records, or rows");
    const uint32_t nwg = std::max<uint32_t>(bucket_groups(m), 1);
    uint32_t *whist = ws;
    if (!m) {
        launch_fill_u32(whist, 0u, (size_t)(L + 1) * nwg, s);
    } else if (ids) {
        hipLaunchKernelGGL(k_cand_keys_rank, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, Xr, n, KSr, ids, m,
                           L, inv, key);
        IG_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_key_hist, dim3(nwg), dim3(BK_T), 0, s, key, m, L, whist, nwg, bucket_iters(m));
    } else {
        hipLaunchKernelGGL(k_row_keys_rank, dim3(nwg), dim3(BK_T), 0, s, W, m, KS, L, rank, inv, key, whist, nwg,
                           bucket_iters(m));
    }
    IG_HIP(hipGetLastError());
    bucket_group(key, m, L, whist, 1, perm, first, ws, s, ids_out ? ids : nullptr, ids_out);
}

void launch_group_records(const uint64_t *X, uint32_t n, uint32_t KS, uint32_t L, uint32_t d, uint32_t *key,
                          uint32_t *list, uint32_t *first, uint32_t *ws, hipStream_t s) {
    IG_REQUIRE(L >= 1 && L <= kMaxBuckets && d >= 1, IG_E_UNSUPPORTED, "token buckets need 1 to 4096 tokens");
    const size_t m = (size_t)n * d;
    const uint32_t nwg = std::max<uint32_t>(bucket_groups(m), 1);
    uint32_t *whist = ws;
    if (!m) launch_fill_u32(whist, 0u, (size_t)(L + 1) * nwg, s);
    else
        hipLaunchKernelGGL(k_record_keys, dim3(nwg), dim3(BK_T), 0, s, X, n, KS, L, d, key, whist, nwg,
                           bucket_iters(m));
    IG_HIP(hipGetLastError());
    bucket_group(key, m, L, whist, d, list, first, ws, s);
}

// ------------------------------------------------------------ per call ----
// Whether every code of flow t is below its feature's bin count.
__device__ __forceinline__ bool flow_valid(const uint16_t *row, uint32_t d, const uint16_t *nbins) {
    bool ok = true;
    for (uint32_t f = 0; f < d; ++f) ok &= row[f] < nbins[f];
    return ok;
}

// out[t] = (0, 0) for a valid flow, (-1, -1) for one with a code out of range;
// cnt[u] += the valid flows holding token u.
__global__ __launch_bounds__(256) void k_prune_count(const uint16_t *__restrict__ codes, uint32_t n, uint32_t d,
                                                     const uint32_t *__restrict__ off,
                                                     const uint16_t *__restrict__ nbins, uint32_t L,
                                                     uint32_t *__restrict__ cnt, int64_t *__restrict__ out) {
    __shared__ uint32_t h[kMaxBuckets];
    for (uint32_t u = threadIdx.x; u < L; u += blockDim.x) h[u] = 0;
    __syncthreads();
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) {
        const uint16_t *row = codes + (size_t)t * d;
        const bool ok = flow_valid(row, d, nbins);
        out[2 * (size_t)t] = ok ? 0 : -1;
        out[2 * (size_t)t + 1] = ok ? 0 : -1;
        if (ok)
            for (uint32_t f = 0; f < d; ++f) atomicAdd(&h[off[f] + row[f]], 1u);
    }
    __syncthreads();
    for (uint32_t u = threadIdx.x; u < L; u += blockDim.x)
        if (h[u]) atomicAdd(&cnt[u], h[u]);
}

// Exclusive scan of v over the 1024 threads of the workgroup (sh: 1024 entries).
__device__ uint32_t block_excl_scan(uint32_t v, uint32_t *sh) {
    const uint32_t tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (uint32_t o = 1; o < 1024; o <<= 1) {
        const uint32_t add = tid >= o ? sh[tid - o] : 0u;
        __syncthreads();
        sh[tid] += add;
        __syncthreads();
    }
    const uint32_t incl = sh[tid];
    __syncthreads();
    return incl - v;
}

// Work units of a pruned contraction over nb buckets of grouped candidates (first
// [nb + 1]: bucket starts, bucket u holding first[u + 1] - first[u] of them):
// uoff[u] = the first unit of bucket u, an exclusive scan of ceil(count_u / cols)
// (uoff[nb] = the total); *tests += sum over u of count_u * nrec[u], the
// (candidate, record) pairs the contraction examines.  One workgroup of 1024.
__global__ __launch_bounds__(1024) void k_contain_plan(const uint32_t *__restrict__ first,
                                                       const uint32_t *__restrict__ nrec, uint32_t nb, uint32_t cols,
                                                       uint32_t *__restrict__ uoff,
                                                       unsigned long long *__restrict__ tests) {
    __shared__ uint32_t sh[1024];
    const uint32_t tid = threadIdx.x, per = (nb + 1023) / 1024, b = tid * per;
    auto units = [&](uint32_t u) { return (first[u + 1] - first[u] + cols - 1) / cols; };
    uint32_t sum = 0;
    unsigned long long t = 0;
    for (uint32_t u = b; u < b + per && u < nb; ++u) {
        sum += units(u);
        t += (unsigned long long)(first[u + 1] - first[u]) * nrec[u];
    }
    uint32_t run = block_excl_scan(sum, sh);
    for (uint32_t u = b; u < b + per && u < nb; ++u) {
        uoff[u] = run;
        run += units(u);
    }
    if (tid == 1023) uoff[nb] = run;   // the last thread's run ends at the total
    if (t) atomicAdd(tests, t);
}

// desc[2 unit], desc[2 unit + 1] = the work unit's candidates [c0, c1), tiles
// [t0, t1) and real records nrec, as (c0, c1, t0, t1), (nrec, 0, 0, 0); units at or
// past uoff[nb] get c0 = c1 = 0 (nothing to do).  One thread per unit of the bound.
__global__ void k_contain_units(const uint32_t *__restrict__ uoff, uint32_t nb, const uint32_t *__restrict__ first,
                                const uint32_t *__restrict__ bt, const uint32_t *__restrict__ nrec, uint32_t cols,
                                uint32_t bound, uint4 *__restrict__ desc) {
    const uint32_t unit = blockIdx.x * blockDim.x + threadIdx.x;
    if (unit >= bound) return;
    if (unit >= uoff[nb]) {
        desc[2 * (size_t)unit] = make_uint4(0, 0, 0, 0);
        desc[2 * (size_t)unit + 1] = make_uint4(0, 0, 0, 0);
        return;
    }
    uint32_t lo = 0, hi = nb;   // the last u with uoff[u] <= unit (its range is not empty)
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) / 2;
        if (uoff[mid] <= unit) lo = mid;
        else hi = mid;
    }
    const uint32_t c0 = first[lo] + (unit - uoff[lo]) * cols;
    desc[2 * (size_t)unit] = make_uint4(c0, first[lo + 1], bt[lo], bt[lo + 1]);
    desc[2 * (size_t)unit + 1] = make_uint4(nrec[lo], 0, 0, 0);
}

void launch_contain_plan(const uint32_t *first, const uint32_t *nrec, uint32_t nb, uint32_t cols, uint32_t *uoff,
                         unsigned long long *tests, hipStream_t s, const uint32_t *bt, uint32_t bound, uint4 *desc) {
    IG_REQUIRE(nb >= 1 && cols >= 1, IG_E_INVAL, "empty bucket plan");
    hipLaunchKernelGGL(k_contain_plan, dim3(1), dim3(1024), 0, s, first, nrec, nb, cols, uoff, tests);
    IG_HIP(hipGetLastError());
    if (desc && bound) {
        hipLaunchKernelGGL(k_contain_units, dim3((bound + 255) / 256), dim3(256), 0, s, uoff, nb, first, bt, nrec,
                           cols, bound, desc);
        IG_HIP(hipGetLastError());
    }
}

// One workgroup of 1024 threads.  foff = exclusive scan of cnt (L entries, plus the
// total); cursor = foff; units of (class c, bucket u), index c * L + u:
// ceil(tiles / rt) * ceil(cnt[u] / cols), 0 when either is 0; uoff = their
// exclusive scan (2L entries, plus the total); the queue starts at 0.
__global__ __launch_bounds__(1024) void k_prune_plan(const uint32_t *__restrict__ cnt, const uint32_t *__restrict__ bt0,
                                                     const uint32_t *__restrict__ bt1, uint32_t L, uint32_t rt,
                                                     uint32_t cols, uint32_t *__restrict__ foff,
                                                     uint32_t *__restrict__ cursor, uint32_t *__restrict__ uoff,
                                                     uint32_t *__restrict__ queue) {
    __shared__ uint32_t sh[1024];
    const uint32_t tid = threadIdx.x;
    // flow lists: thread tid scans entries [tid * per, tid * per + per)
    {
        const uint32_t per = (L + 1023) / 1024, b = tid * per;
        uint32_t sum = 0;
        for (uint32_t i = b; i < b + per && i < L; ++i) sum += cnt[i];
        uint32_t run = block_excl_scan(sum, sh);
        for (uint32_t i = b; i < b + per && i < L; ++i) {
            foff[i] = run;
            cursor[i] = run;
            run += cnt[i];
        }
        if (tid == 1023) foff[L] = run;   // the last thread's run ends at the total
    }
    // work units
    {
        const uint32_t n2 = 2 * L, per = (n2 + 1023) / 1024, b = tid * per;
        auto units = [&](uint32_t i) {
            const uint32_t c = i >= L, u = i - c * L;
            const uint32_t *bt = c ? bt1 : bt0;
            const uint32_t tiles = bt[u + 1] - bt[u];
            return ((tiles + rt - 1) / rt) * ((cnt[u] + cols - 1) / cols);
        };
        uint32_t sum = 0;
        for (uint32_t i = b; i < b + per && i < n2; ++i) sum += units(i);
        uint32_t run = block_excl_scan(sum, sh);
        for (uint32_t i = b; i < b + per && i < n2; ++i) {
            uoff[i] = run;
            run += units(i);
        }
        if (tid == 1023) {
            uoff[n2] = run;
            *queue = 0;
        }
    }
}

// list[cursor[u]++] = t for every token u of every valid flow t.  Each workgroup
// counts its flows per token in LDS, reserves one block per token with a single
// atomic, and fills it.
__global__ __launch_bounds__(256) void k_prune_scatter(const uint16_t *__restrict__ codes, uint32_t n, uint32_t d,
                                                       const uint32_t *__restrict__ off,
                                                       const uint16_t *__restrict__ nbins, uint32_t L,
                                                       uint32_t *__restrict__ cursor, uint32_t *__restrict__ list) {
    __shared__ uint32_t rank[kMaxBuckets], base[kMaxBuckets];
    for (uint32_t u = threadIdx.x; u < L; u += blockDim.x) rank[u] = 0;
    __syncthreads();
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const uint16_t *row = codes + (size_t)(t < n ? t : 0u) * d;
    const bool ok = t < n && flow_valid(row, d, nbins);
    if (ok)
        for (uint32_t f = 0; f < d; ++f) atomicAdd(&rank[off[f] + row[f]], 1u);
    __syncthreads();
    for (uint32_t u = threadIdx.x; u < L; u += blockDim.x) {
        base[u] = rank[u] ? atomicAdd(&cursor[u], rank[u]) : 0u;
        rank[u] = 0;
    }
    __syncthreads();
    if (ok)
        for (uint32_t f = 0; f < d; ++f) {
            const uint32_t u = off[f] + row[f];
            list[base[u] + atomicAdd(&rank[u], 1u)] = t;
        }
}

// the lists and units, then (at a multiple of 4 words) the flows' operands: 2 KO
// uint4 per flow
static size_t prune_list_words(uint32_t L, uint32_t n_flows, uint32_t d) {
    return (5ull * L + 3 + (size_t)n_flows * d + 3) & ~(size_t)3;
}

size_t prune_scratch_words(uint32_t L, uint32_t n_flows, uint32_t d, uint32_t KO) {
    return prune_list_words(L, n_flows, d) + 8ull * KO * n_flows;
}

void launch_prune_lists(const uint16_t *codes, uint32_t n, uint32_t d, const uint32_t *off, const uint16_t *nbins,
                        uint32_t L, const uint32_t *bt0, const uint32_t *bt1, uint32_t rt, uint32_t cols,
                        int64_t *out, PruneWork &w, hipStream_t s) {
    IG_REQUIRE(L >= 1 && L <= kMaxBuckets, IG_E_UNSUPPORTED, "pruned scoring needs 1 to 4096 tokens");
    IG_REQUIRE(rt >= 1 && cols >= 1, IG_E_INVAL, "empty work units");
    launch_fill_u32(w.cnt, 0u, L, s);
    const unsigned blocks = (unsigned)((n + 255) / 256);
    if (n) hipLaunchKernelGGL(k_prune_count, dim3(blocks), dim3(256), 0, s, codes, n, d, off, nbins, L, w.cnt, out);
    IG_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_prune_plan, dim3(1), dim3(1024), 0, s, w.cnt, bt0, bt1, L, rt, cols, w.foff, w.cursor, w.uoff,
                       w.queue);
    IG_HIP(hipGetLastError());
    if (n) hipLaunchKernelGGL(k_prune_scatter, dim3(blocks), dim3(256), 0, s, codes, n, d, off, nbins, L, w.cursor,
                              w.list);
    IG_HIP(hipGetLastError());
}

PruneWork prune_work(uint32_t *ws, uint32_t L, uint32_t n_flows, uint32_t d) {
    PruneWork w;
    w.ops = reinterpret_cast<uint4 *>(ws + prune_list_words(L, n_flows, d));
    w.cnt = ws;
    w.cursor = ws + L;
    w.foff = ws + 2 * (size_t)L;
    w.uoff = w.foff + L + 1;
    w.queue = w.uoff + 2 * (size_t)L + 1;
    w.list = w.queue + 1;
    return w;
}

}  // namespace ig
