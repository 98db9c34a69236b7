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
// key[e] = the bucket of candidate e: its token with the fewest records (cnt),
// the lowest such token on ties, or L for a candidate without a token; hist[u] +=
// the candidates of bucket u (u <= L).  Candidate e is the pair id ids[e] of the
// records X [n][KS] (their intersection), or row e of W [m][KS] when ids is null.
__global__ __launch_bounds__(256) void k_cand_bucket_keys(const uint64_t *__restrict__ X, uint32_t n, uint32_t KS,
                                                          const uint32_t *__restrict__ ids,
                                                          const uint64_t *__restrict__ W, size_t m, uint32_t L,
                                                          const uint32_t *__restrict__ cnt, uint32_t *__restrict__ key,
                                                          uint32_t *__restrict__ hist) {
    __shared__ uint32_t h[kMaxBuckets + 1];
    for (uint32_t u = threadIdx.x; u <= L; u += blockDim.x) h[u] = 0;
    __syncthreads();
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < m) {
        uint32_t i = 0, j = 0;
        if (ids) decode_pair(ids[e], n, i, j);
        uint32_t best = L, bc = ~0u;
        for (uint32_t k = 0; k < KS; ++k) {
            uint64_t w = ids ? (X[(size_t)i * KS + k] & X[(size_t)j * KS + k]) : W[e * KS + k];
            while (w) {
                const uint32_t tok = 64 * k + (uint32_t)__builtin_ctzll(w);
                w &= w - 1;
                if (tok >= L) break;
                const uint32_t c = cnt[tok];
                if (c < bc) {   // tokens come in ascending order: ties keep the lowest
                    bc = c;
                    best = tok;
                }
            }
        }
        key[e] = best;
        atomicAdd(&h[best], 1u);
    }
    __syncthreads();
    for (uint32_t u = threadIdx.x; u <= L; u += blockDim.x)
        if (h[u]) atomicAdd(&hist[u], h[u]);
}

// perm[cs[key[e]] + (place of e among its bucket's candidates)] = e.  Each
// workgroup counts its elements per bucket, reserves a range of each bucket
// (cursor, zero at launch), and places its elements there (the order inside a
// bucket is not fixed; the results do not depend on it).
constexpr uint32_t BP_T = 256, BP_I = 8;
__global__ __launch_bounds__(BP_T) void k_bucket_place(const uint32_t *__restrict__ key, size_t m, uint32_t L,
                                                       const uint32_t *__restrict__ cs, uint32_t *__restrict__ cursor,
                                                       uint32_t *__restrict__ perm) {
    __shared__ uint32_t h[kMaxBuckets + 1];
    for (uint32_t u = threadIdx.x; u <= L; u += BP_T) h[u] = 0;
    __syncthreads();
    const size_t base = (size_t)blockIdx.x * (BP_T * BP_I);
    uint32_t k[BP_I], r[BP_I];
#pragma unroll
    for (uint32_t it = 0; it < BP_I; ++it) {
        const size_t e = base + (size_t)it * BP_T + threadIdx.x;
        k[it] = e < m ? key[e] : ~0u;
        r[it] = k[it] != ~0u ? atomicAdd(&h[k[it]], 1u) : 0u;
    }
    __syncthreads();
    for (uint32_t u = threadIdx.x; u <= L; u += BP_T)
        if (h[u]) h[u] = cs[u] + atomicAdd(&cursor[u], h[u]);   // the workgroup's first slot
    __syncthreads();
#pragma unroll
    for (uint32_t it = 0; it < BP_I; ++it) {
        const size_t e = base + (size_t)it * BP_T + threadIdx.x;
        if (k[it] != ~0u) perm[h[k[it]] + r[it]] = (uint32_t)e;
    }
}

// The records of X [n][KS] under each token u < L they hold: list[ro[u] + slot]
// (slots taken from cursor, zero at launch); bucket L lists every record in order.
__global__ void k_bucket_records(const uint64_t *__restrict__ X, uint32_t n, uint32_t KS, uint32_t L,
                                 const uint32_t *__restrict__ ro, uint32_t *__restrict__ cursor,
                                 uint32_t *__restrict__ list) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    list[ro[L] + r] = r;
    for (uint32_t k = 0; k < KS; ++k) {
        uint64_t w = X[(size_t)r * KS + k];
        while (w) {
            const uint32_t tok = 64 * k + (uint32_t)__builtin_ctzll(w);
            w &= w - 1;
            if (tok >= L) break;
            list[ro[tok] + atomicAdd(&cursor[tok], 1u)] = r;
        }
    }
}

void launch_cand_bucket_keys(const uint64_t *X, uint32_t n, uint32_t KS, const uint32_t *ids, const uint64_t *W,
                             size_t m, uint32_t L, const uint32_t *cnt, uint32_t *key, uint32_t *hist, hipStream_t s) {
    IG_REQUIRE(L >= 1 && L <= kMaxBuckets, IG_E_UNSUPPORTED, "token buckets need 1 to 4096 tokens");
    IG_REQUIRE((ids && X) || (!ids && W), IG_E_INVAL, "candidates need pair ids and records, or rows");
    launch_fill_u32(hist, 0u, L + 1, s);
    if (!m) return;
    hipLaunchKernelGGL(k_cand_bucket_keys, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, X, n, KS, ids, W, m,
                       L, cnt, key, hist);
    IG_HIP(hipGetLastError());
}

void launch_bucket_place(const uint32_t *key, size_t m, uint32_t L, const uint32_t *cs, uint32_t *cursor,
                         uint32_t *perm, hipStream_t s) {
    IG_REQUIRE(L >= 1 && L <= kMaxBuckets, IG_E_UNSUPPORTED, "token buckets need 1 to 4096 tokens");
    launch_fill_u32(cursor, 0u, L + 1, s);
    if (!m) return;
    const size_t per = (size_t)BP_T * BP_I;
    hipLaunchKernelGGL(k_bucket_place, dim3((unsigned)((m + per - 1) / per)), dim3(BP_T), 0, s, key, m, L, cs, cursor,
                       perm);
    IG_HIP(hipGetLastError());
}

void launch_bucket_records(const uint64_t *X, uint32_t n, uint32_t KS, uint32_t L, const uint32_t *ro,
                           uint32_t *cursor, uint32_t *list, hipStream_t s) {
    IG_REQUIRE(L >= 1 && L <= kMaxBuckets, IG_E_UNSUPPORTED, "token buckets need 1 to 4096 tokens");
    launch_fill_u32(cursor, 0u, L + 1, s);
    if (!n) return;
    hipLaunchKernelGGL(k_bucket_records, dim3((n + 255) / 256), dim3(256), 0, s, X, n, KS, L, ro, cursor, list);
    IG_HIP(hipGetLastError());
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

size_t prune_scratch_words(uint32_t L, uint32_t n_flows, uint32_t d) {
    return 5ull * L + 3 + (size_t)n_flows * d;
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

PruneWork prune_work(uint32_t *ws, uint32_t L) {
    PruneWork w;
    w.cnt = ws;
    w.cursor = ws + L;
    w.foff = ws + 2 * (size_t)L;
    w.uoff = w.foff + L + 1;
    w.queue = w.uoff + 2 * (size_t)L + 1;
    w.list = w.queue + 1;
    return w;
}

}  // namespace ig
