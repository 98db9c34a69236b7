// Candidate enumeration (Eq. 1) and exact de-duplication on the device.
//
// A candidate is identified by its pair id q (see decode_pair): the record q, or
// the AND of records i < j.  Candidates are never materialised here: the rows
// of one class stay resident (L2-sized) and every kernel recomputes
// x_i AND x_j from the pair id.  De-duplication sorts (hash, id) pairs and then
// compares the full bitsets inside runs of equal hash, so a hash collision can
// never merge two different candidates.
#include "common.h"
#include "kernels.h"

namespace ig {

__device__ __forceinline__ uint64_t mix64(uint64_t h) {
    h ^= h >> 32;
    h *= 0xd6e8feb86659fd93ull;
    h ^= h >> 32;
    h *= 0xd6e8feb86659fd93ull;
    h ^= h >> 32;
    return h;
}

// keys[e] = (segment id in the top `segbits` bits) | (hash of b >> segbits),
// vals[e] = q, for q in [q0, q0 + count).  Empty intersections get the
// sentinel (~0, ~0) and are dropped by the de-duplication.
__global__ void k_pair_hash(const uint64_t *__restrict__ X, uint32_t n, uint32_t KS, uint32_t K, uint64_t q0,
                            uint64_t count, uint64_t seg_hi, int segbits, uint64_t *__restrict__ keys,
                            uint32_t *__restrict__ vals) {
    uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    uint64_t q = q0 + e;
    uint32_t i, j;
    decode_pair(q, n, i, j);
    const uint64_t *xi = X + (size_t)i * KS, *xj = X + (size_t)j * KS;
    uint64_t h = 0x9e3779b97f4a7c15ull ^ K;
    uint64_t any = 0;
    for (uint32_t k = 0; k < K; ++k) {
        uint64_t b = xi[k] & xj[k];
        any |= b;
        h = mix64(h ^ b) + 0x632be59bd9b4e019ull;
    }
    if (any) {
        keys[e] = seg_hi | (h >> segbits);
        vals[e] = (uint32_t)q;
    } else {
        keys[e] = ~0ull;
        vals[e] = ~0u;
    }
}

struct RowsOfSeg {
    const uint64_t *X;
    uint32_t n, KS, K;
};

__device__ __forceinline__ bool same_candidate(const RowsOfSeg &r, uint32_t qa, uint32_t qb) {
    uint32_t ia, ja, ib, jb;
    decode_pair(qa, r.n, ia, ja);
    decode_pair(qb, r.n, ib, jb);
    const uint64_t *a0 = r.X + (size_t)ia * r.KS, *a1 = r.X + (size_t)ja * r.KS;
    const uint64_t *b0 = r.X + (size_t)ib * r.KS, *b1 = r.X + (size_t)jb * r.KS;
    for (uint32_t k = 0; k < r.K; ++k)
        if ((a0[k] & a1[k]) != (b0[k] & b1[k])) return false;
    return true;
}

// flags[e] = 1 when element e is the first occurrence of its bitset among the
// sorted elements (earlier elements with the same key are compared in full).
// Also counts the distinct candidates of every segment.
__global__ void k_dedup_flags(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ vals, size_t m,
                              const RowsOfSeg *__restrict__ segs, int segbits, uint32_t *__restrict__ flags,
                              uint32_t *__restrict__ seg_counts) {
    size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t rep = 0, seg = 0;
    if (e < m) {
        uint32_t q = vals[e];
        if (q != ~0u) {
            uint64_t key = keys[e];
            seg = (uint32_t)(key >> (64 - segbits));
            RowsOfSeg r = segs[seg];
            rep = 1;
            for (size_t p = e; p-- > 0;) {
                if (keys[p] != key) break;
                const uint32_t qp = vals[p];
                if (qp == ~0u) continue;   // empty-intersection sentinel
                if (same_candidate(r, qp, q)) { rep = 0; break; }
            }
        }
        flags[e] = rep;
    }
    if (rep) atomicAdd(&seg_counts[seg], 1u);
}

__global__ void k_compact(const uint32_t *__restrict__ flags, const uint32_t *__restrict__ pos,
                          const uint32_t *__restrict__ vals, size_t m, uint32_t *__restrict__ out) {
    size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < m && flags[e]) out[pos[e]] = vals[e];
}

// key of word k of candidate q (for ordering): x_i[k] AND x_j[k]
__global__ void k_gather_word(const uint64_t *__restrict__ X, uint32_t n, uint32_t KS, uint32_t k,
                              const uint32_t *__restrict__ ids, size_t m, uint64_t *__restrict__ keys) {
    size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    uint32_t i, j;
    decode_pair(ids[e], n, i, j);
    keys[e] = X[(size_t)i * KS + k] & X[(size_t)j * KS + k];
}

// OR and AND of every word over the candidates ids[0..m): constant bits need no sort pass.
__global__ void k_word_range(const uint64_t *__restrict__ X, uint32_t n, uint32_t KS, uint32_t K,
                             const uint32_t *__restrict__ ids, size_t m, unsigned long long *__restrict__ orv,
                             unsigned long long *__restrict__ andv) {
    size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t i = 0, j = 0;
    bool valid = e < m;
    if (valid) decode_pair(ids[e], n, i, j);
    for (uint32_t k = 0; k < K; ++k) {
        uint64_t w = valid ? (X[(size_t)i * KS + k] & X[(size_t)j * KS + k]) : 0ull;
        uint64_t wa = valid ? w : ~0ull;
        // wave-level reduction first
        for (int o = 32; o > 0; o >>= 1) {
            w |= __shfl_xor(w, o, 64);
            wa &= __shfl_xor(wa, o, 64);
        }
        if ((threadIdx.x & 63) == 0) {
            atomicOr(&orv[k], (unsigned long long)w);
            atomicAnd(&andv[k], (unsigned long long)wa);
        }
    }
}

// rows of the ordered candidates, plus "differs from predecessor" flags (for
// merging duplicates that came from different pair-space chunks)
__global__ void k_materialize(const uint64_t *__restrict__ X, uint32_t n, uint32_t KS, const uint32_t *__restrict__ ids,
                              size_t m, uint64_t *__restrict__ W, uint32_t *__restrict__ newflag) {
    size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    uint32_t i, j, pi, pj;
    decode_pair(ids[e], n, i, j);
    bool differs = (e == 0);
    if (e > 0) decode_pair(ids[e - 1], n, pi, pj);
    for (uint32_t k = 0; k < KS; ++k) {
        uint64_t w = X[(size_t)i * KS + k] & X[(size_t)j * KS + k];
        W[e * KS + k] = w;
        if (e > 0 && !differs) differs = w != (X[(size_t)pi * KS + k] & X[(size_t)pj * KS + k]);
    }
    if (newflag) newflag[e] = differs ? 1u : 0u;
}

// out[pos[e]] = W[e] for flagged e (row copy)
__global__ void k_compact_rows(const uint64_t *__restrict__ W, const uint32_t *__restrict__ flags,
                               const uint32_t *__restrict__ pos, size_t m, uint32_t KS, uint64_t *__restrict__ out) {
    size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= m * KS) return;
    size_t e = g / KS, k = g % KS;
    if (flags[e]) out[(size_t)pos[e] * KS + k] = W[g];
}

// rows W[ids[e]] in the order of ids (ordering of given pattern sets)
__global__ void k_gather_rows(const uint64_t *__restrict__ W, const uint32_t *__restrict__ ids, size_t m,
                              uint32_t KS, uint64_t *__restrict__ out, const uint32_t *__restrict__ fin,
                              uint32_t *__restrict__ fout) {
    size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= m * KS) return;
    size_t e = g / KS, k = g % KS;
    out[g] = W[(size_t)ids[e] * KS + k];
    if (fin && k == 0) fout[e] = fin[ids[e]];
}

__global__ void k_row_word(const uint64_t *__restrict__ W, const uint32_t *__restrict__ ids, size_t m, uint32_t KS,
                           uint32_t k, uint64_t *__restrict__ keys) {
    size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < m) keys[e] = W[(size_t)ids[e] * KS + k];
}

__global__ void k_iota(uint32_t *__restrict__ v, size_t m) {
    size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < m) v[e] = (uint32_t)e;
}

__global__ void k_adjacent_equal(const uint64_t *__restrict__ W, size_t m, uint32_t KS, uint32_t *__restrict__ cnt) {
    size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e == 0 || e >= m) return;
    bool eq = true;
    for (uint32_t k = 0; k < KS; ++k) eq &= W[e * KS + k] == W[(e - 1) * KS + k];
    if (eq) atomicAdd(cnt, 1u);
}

__global__ void k_weights(const uint64_t *__restrict__ W, const uint32_t *__restrict__ f, size_t m, uint32_t KS,
                          int64_t *__restrict__ S) {
    size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    uint32_t len = 0;
    for (uint32_t k = 0; k < KS; ++k) len += (uint32_t)__popcll(W[e * KS + k]);
    S[e] = (int64_t)f[e] * (int64_t)len * (int64_t)len;
}

static dim3 blocks_for(size_t n, unsigned bs = 256) { return dim3((unsigned)((n + bs - 1) / bs)); }

void launch_pair_hash(const uint64_t *X, uint32_t n, uint32_t KS, uint32_t K, uint64_t q0, uint64_t count,
                      uint32_t seg, int segbits, uint64_t *keys, uint32_t *vals, hipStream_t s) {
    if (!count) return;
    uint64_t seg_hi = (uint64_t)seg << (64 - segbits);
    hipLaunchKernelGGL(k_pair_hash, blocks_for(count), dim3(256), 0, s, X, n, KS, K, q0, count, seg_hi, segbits, keys,
                       vals);
    IG_HIP(hipGetLastError());
}

void launch_dedup_flags(const uint64_t *keys, const uint32_t *vals, size_t m, const void *segs_dev, int segbits,
                        uint32_t *flags, uint32_t *seg_counts, hipStream_t s) {
    if (!m) return;
    hipLaunchKernelGGL(k_dedup_flags, blocks_for(m), dim3(256), 0, s, keys, vals, m, (const RowsOfSeg *)segs_dev,
                       segbits, flags, seg_counts);
    IG_HIP(hipGetLastError());
}

size_t rows_of_seg_size() { return sizeof(RowsOfSeg); }
void fill_rows_of_seg(void *dst, const uint64_t *X, uint32_t n, uint32_t KS, uint32_t K) {
    RowsOfSeg r{X, n, KS, K};
    *static_cast<RowsOfSeg *>(dst) = r;
}

void launch_compact(const uint32_t *flags, const uint32_t *pos, const uint32_t *vals, size_t m, uint32_t *out,
                    hipStream_t s) {
    if (!m) return;
    hipLaunchKernelGGL(k_compact, blocks_for(m), dim3(256), 0, s, flags, pos, vals, m, out);
    IG_HIP(hipGetLastError());
}

void launch_gather_word(const uint64_t *X, uint32_t n, uint32_t KS, uint32_t k, const uint32_t *ids, size_t m,
                        uint64_t *keys, hipStream_t s) {
    if (!m) return;
    hipLaunchKernelGGL(k_gather_word, blocks_for(m), dim3(256), 0, s, X, n, KS, k, ids, m, keys);
    IG_HIP(hipGetLastError());
}

void launch_word_range(const uint64_t *X, uint32_t n, uint32_t KS, uint32_t K, const uint32_t *ids, size_t m,
                       unsigned long long *orv, unsigned long long *andv, hipStream_t s) {
    if (!m) return;
    hipLaunchKernelGGL(k_word_range, blocks_for(m), dim3(256), 0, s, X, n, KS, K, ids, m, orv, andv);
    IG_HIP(hipGetLastError());
}

void launch_materialize(const uint64_t *X, uint32_t n, uint32_t KS, const uint32_t *ids, size_t m, uint64_t *W,
                        uint32_t *newflag, hipStream_t s) {
    if (!m) return;
    hipLaunchKernelGGL(k_materialize, blocks_for(m), dim3(256), 0, s, X, n, KS, ids, m, W, newflag);
    IG_HIP(hipGetLastError());
}

void launch_compact_rows(const uint64_t *W, const uint32_t *flags, const uint32_t *pos, size_t m, uint32_t KS,
                         uint64_t *out, hipStream_t s) {
    if (!m) return;
    hipLaunchKernelGGL(k_compact_rows, blocks_for(m * KS), dim3(256), 0, s, W, flags, pos, m, KS, out);
    IG_HIP(hipGetLastError());
}

void launch_gather_rows(const uint64_t *W, const uint32_t *ids, size_t m, uint32_t KS, uint64_t *out,
                        const uint32_t *fin, uint32_t *fout, hipStream_t s) {
    if (!m) return;
    hipLaunchKernelGGL(k_gather_rows, blocks_for(m * KS), dim3(256), 0, s, W, ids, m, KS, out, fin, fout);
    IG_HIP(hipGetLastError());
}

void launch_row_word(const uint64_t *W, const uint32_t *ids, size_t m, uint32_t KS, uint32_t k, uint64_t *keys,
                     hipStream_t s) {
    if (!m) return;
    hipLaunchKernelGGL(k_row_word, blocks_for(m), dim3(256), 0, s, W, ids, m, KS, k, keys);
    IG_HIP(hipGetLastError());
}

void launch_adjacent_equal(const uint64_t *W, size_t m, uint32_t KS, uint32_t *d_count, hipStream_t s) {
    if (m < 2) return;
    hipLaunchKernelGGL(k_adjacent_equal, blocks_for(m), dim3(256), 0, s, W, m, KS, d_count);
    IG_HIP(hipGetLastError());
}

void launch_weights(const uint64_t *W, const uint32_t *f, size_t m, uint32_t KS, int64_t *S, hipStream_t s) {
    if (!m) return;
    hipLaunchKernelGGL(k_weights, blocks_for(m), dim3(256), 0, s, W, f, m, KS, S);
    IG_HIP(hipGetLastError());
}

void launch_iota(uint32_t *v, size_t m, hipStream_t s) {
    if (!m) return;
    hipLaunchKernelGGL(k_iota, blocks_for(m), dim3(256), 0, s, v, m);
    IG_HIP(hipGetLastError());
}

}  // namespace ig
