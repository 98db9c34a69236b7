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

// keys[e] = (segment id in the top `segbits` bits) | (hash of b >> segbits), with
// the bits under `keep` cleared, vals[e] = q, for q in [q0, q0 + count).  Empty
// intersections get the sentinel (~0, ~0) and are dropped by the de-duplication.
__global__ void k_pair_hash(const uint64_t *__restrict__ X, uint32_t n, uint32_t KS, uint32_t K, uint64_t q0,
                            uint64_t count, uint64_t seg_hi, int segbits, uint64_t keep, uint64_t *__restrict__ keys,
                            uint32_t *__restrict__ vals) {
    uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    uint64_t q = q0 + e;
    uint32_t i, j;
    decode_pair(q, n, i, j);
    const uint64_t *xi = X + (size_t)i * KS, *xj = X + (size_t)j * KS;
    uint64_t h = 0x9e3779b97f4a7c15ull ^ K;
    uint64_t any = 0;
    for (uint32_t k0 = 0; k0 < K; k0 += 8) {
        // eight words' loads in flight at once, then the hash chain in word order
        uint64_t b[8];
#pragma unroll
        for (uint32_t u = 0; u < 8; ++u) b[u] = k0 + u < K ? xi[k0 + u] & xj[k0 + u] : 0ull;
#pragma unroll
        for (uint32_t u = 0; u < 8; ++u)
            if (k0 + u < K) {
                any |= b[u];
                h = mix64(h ^ b[u]) + 0x632be59bd9b4e019ull;
            }
    }
    if (any) {
        keys[e] = (seg_hi | (h >> segbits)) & keep;
        vals[e] = (uint32_t)q;
    } else {
        // the largest key the sort sees (masked like the others, so a run of equal
        // keys that sentinels join is still one run; the run scan skips them)
        keys[e] = keep;
        vals[e] = ~0u;
    }
}

struct RowsOfSeg {
    const uint64_t *X;
    uint32_t n, KS, K;
};

// b[u] = xi[k0 + u] AND xj[k0 + u] for the words k0 + u < K of two rows (0 past K;
// k0 a multiple of 8).  vec (rows of an even number of words, so 16-byte aligned):
// two words per load, half as many scattered loads (a word past K that is loaded
// with its pair is still inside the row).
__device__ __forceinline__ void rows_and8(const uint64_t *xi, const uint64_t *xj, uint32_t k0, uint32_t K, bool vec,
                                          uint64_t (&b)[8]) {
    if (vec) {
        const uint4 *vi = reinterpret_cast<const uint4 *>(xi + k0), *vj = reinterpret_cast<const uint4 *>(xj + k0);
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u) {
            uint4 a = make_uint4(0, 0, 0, 0), c = a;
            if (k0 + 2 * u < K) {
                a = vi[u];
                c = vj[u];
            }
            b[2 * u] = ((uint64_t)a.y << 32 | a.x) & ((uint64_t)c.y << 32 | c.x);
            b[2 * u + 1] = k0 + 2 * u + 1 < K ? ((uint64_t)a.w << 32 | a.z) & ((uint64_t)c.w << 32 | c.z) : 0ull;
        }
    } else {
#pragma unroll
        for (uint32_t u = 0; u < 8; ++u) b[u] = k0 + u < K ? xi[k0 + u] & xj[k0 + u] : 0ull;
    }
}

__device__ __forceinline__ bool same_candidate(const RowsOfSeg &r, uint32_t qa, uint32_t qb) {
    uint32_t ia, ja, ib, jb;
    decode_pair(qa, r.n, ia, ja);
    decode_pair(qb, r.n, ib, jb);
    const uint64_t *a0 = r.X + (size_t)ia * r.KS, *a1 = r.X + (size_t)ja * r.KS;
    const uint64_t *b0 = r.X + (size_t)ib * r.KS, *b1 = r.X + (size_t)jb * r.KS;
    const bool vec = (r.KS & 1u) == 0;
    for (uint32_t k0 = 0; k0 < r.K; k0 += 8) {
        uint64_t x[8], y[8];   // eight words of the four rows loaded together
        rows_and8(a0, a1, k0, r.K, vec, x);
        rows_and8(b0, b1, k0, r.K, vec, y);
        uint64_t diff = 0;
#pragma unroll
        for (uint32_t u = 0; u < 8; ++u) diff |= x[u] ^ y[u];
        if (diff) return false;
    }
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
}

// ------------------------------------------- partitioned de-duplication ----
// The same de-duplication with two radix passes instead of five, for one pass over
// the pair space of both classes (segments 0 and 1): item g of segment c is pair
// id q0[c] + (g - gbase[c]).  Each item gets a key: its class in the top bit and 63
// bits of a 64-bit hash of its intersection (the class mixed in after the words).
// A stable sort on the top 16 bits splits the items into 2 x 32,768 partitions,
// class 0's first, in item order inside each; one workgroup per partition finds
// equal keys with an LDS hash table whose entries keep the lowest local index per
// key (the first occurrence in item order, as after the full sort), and every
// other copy is then compared with that first one in full (k_dedup_verify): a
// difference (two candidates sharing a key) or a partition with too many distinct
// keys sets *err, and the caller falls back to the full sort.  The candidates come
// out class by class in the partitions' order.
struct DedupArgs {
    RowsOfSeg seg[2];
    uint64_t q0[2], gbase[2];
};

__device__ __forceinline__ void dedup_item_of(const DedupArgs &a, uint64_t g, int &c, uint32_t &q) {
    c = g >= a.gbase[1] ? 1 : 0;
    q = (uint32_t)(a.q0[c] + (g - a.gbase[c]));
}

// keys[g] = item g's class << 63 | 63 bits of the hash of its intersection, vals[g]
// = g.  Empty intersections get vals[g] = ~0 and a key spread by g (so that no
// partition collects them).
__global__ __launch_bounds__(256) void k_pair_hash64(DedupArgs a, uint64_t items, uint64_t *__restrict__ keys,
                                                     uint32_t *__restrict__ vals) {
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= items) return;
    int c;
    uint32_t q;
    dedup_item_of(a, g, c, q);
    const RowsOfSeg &r = a.seg[c];
    uint32_t i, j;
    decode_pair(q, r.n, i, j);
    const uint64_t *xi = r.X + (size_t)i * r.KS, *xj = r.X + (size_t)j * r.KS;
    uint64_t hh = 0x9e3779b97f4a7c15ull ^ r.K;
    uint64_t any = 0;
    const bool vec = (r.KS & 1u) == 0;
    for (uint32_t k0 = 0; k0 < r.K; k0 += 8) {
        uint64_t b[8];
        rows_and8(xi, xj, k0, r.K, vec, b);
#pragma unroll
        for (uint32_t u = 0; u < 8; ++u)
            if (k0 + u < r.K) {
                any |= b[u];
                hh = mix64(hh ^ b[u]) + 0x632be59bd9b4e019ull;
            }
    }
    // the class enters after the words: mixed into the starting state, a difference
    // there could be cancelled by one in the first word (the same two tokens of a
    // feature in either class would then hash alike)
    const uint64_t h = any ? mix64(hh ^ ((uint64_t)(c + 1) * 0x9ddfea08eb382d69ull)) : mix64(g + 0x51afd7ed558ccdull);
    keys[g] = (uint64_t)c << 63 | h >> 1;
    vals[g] = any ? (uint32_t)g : ~0u;
}

#ifndef IG_PART_BITS
#define IG_PART_BITS 16
#endif
constexpr uint32_t kPartBits = IG_PART_BITS;   // partitions: the top bits of the hash (14 to 16)
constexpr uint32_t kPartSlots = 2048;       // LDS hash table of a partition (distinct hashes)

// starts[p] = the first sorted position of partition p (starts[2^16] = m).
__global__ void k_part_starts(const uint64_t *__restrict__ keys, size_t m, uint32_t *__restrict__ starts) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e > m) return;
    const uint32_t np = 1u << kPartBits;
    const uint32_t p = e < m ? (uint32_t)(keys[e] >> (64 - kPartBits)) : np;
    const uint32_t prev = e > 0 ? (uint32_t)(keys[e - 1] >> (64 - kPartBits)) : 0u;
    // the partitions after the previous element's, up to this one, start here
    for (uint32_t q = e > 0 ? prev + 1 : 0u; q <= p; ++q) starts[q] = (uint32_t)e;
}

// flags[e] = 1 for the first copy (in item order) of each key among the sorted
// items of a partition, own[e] = the sorted position of that first copy.
__global__ __launch_bounds__(256) void k_part_dedup(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ vals,
                                                    const uint32_t *__restrict__ starts, uint32_t *__restrict__ flags,
                                                    uint32_t *__restrict__ own, uint32_t *__restrict__ err) {
    __shared__ unsigned long long tab[kPartSlots];
    const uint32_t s0 = starts[blockIdx.x], s1 = starts[blockIdx.x + 1];
    if (s1 - s0 >= (1u << 26)) {   // uniform: local indices beyond an entry's 26 bits
        if (threadIdx.x == 0) atomicOr(err, 1u);
        return;
    }
    for (uint32_t t = threadIdx.x; t < kPartSlots; t += 256) tab[t] = 0ull;
    __syncthreads();
    // entry: key bits above the slot index (never zero) << 26 | local index (copies
    // of one candidate share an entry, so a partition may hold many more items than
    // slots); a table that fills up sets *err
    const uint32_t mask = kPartSlots - 1;
    for (uint32_t li = threadIdx.x; li < s1 - s0; li += 256) {
        if (vals[s0 + li] == ~0u) continue;
        const uint64_t h = keys[s0 + li];
        const unsigned long long tag = ((h >> 11) & ((1ull << 37) - 1)) | (1ull << 37);
        const unsigned long long v = tag << 26 | li;
        uint32_t slot = (uint32_t)h & mask, probes = 0;
        for (;; slot = (slot + 1) & mask) {
            const unsigned long long seen = tab[slot];
            if ((seen >> 26) == tag && seen <= v) break;   // an earlier copy holds the entry
            const unsigned long long cur = seen ? seen : atomicCAS(&tab[slot], 0ull, v);
            if (cur == 0ull) break;
            if ((cur >> 26) == tag) {
                if (v < cur) atomicMin(&tab[slot], v);
                break;
            }
            if (++probes == kPartSlots) {
                atomicOr(err, 1u);
                break;
            }
        }
    }
    __syncthreads();
    for (uint32_t li = threadIdx.x; li < s1 - s0; li += 256) {
        uint32_t f = 0, o = s0 + li;
        if (vals[s0 + li] != ~0u) {
            const uint64_t h = keys[s0 + li];
            const unsigned long long tag = ((h >> 11) & ((1ull << 37) - 1)) | (1ull << 37);
            uint32_t probes = 0;
            for (uint32_t slot = (uint32_t)h & mask;; slot = (slot + 1) & mask) {
                const unsigned long long cur = tab[slot];
                if (cur == 0ull || ++probes > kPartSlots) {   // not inserted: the table filled up
                    atomicOr(err, 1u);
                    break;
                }
                if ((cur >> 26) != tag) continue;
                const uint32_t lo = (uint32_t)(cur & ((1ull << 26) - 1));
                o = s0 + lo;
                f = lo == li ? 1u : 0u;
                if (keys[o] != h) atomicOr(err, 1u);   // two keys share a tag
                break;
            }
        }
        flags[s0 + li] = f;
        own[s0 + li] = o;
    }
}

// Every copy is compared in full with the first one of its key: a difference sets
// *err.
__global__ __launch_bounds__(256) void k_dedup_verify(DedupArgs a, uint64_t items, const uint32_t *__restrict__ vals,
                                                      const uint32_t *__restrict__ own, uint32_t *__restrict__ err) {
    const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= items) return;
    const uint32_t g = vals[e], o = own[e];
    if (g == ~0u || o == (uint32_t)e) return;
    int c, oc;
    uint32_t q, oq;
    dedup_item_of(a, g, c, q);
    dedup_item_of(a, vals[o], oc, oq);
    if (oc != c || !same_candidate(a.seg[c], oq, q)) atomicOr(err, 1u);
}

// out[pos[e]] = the pair id of sorted item e, for the flagged ones.
__global__ __launch_bounds__(256) void k_dedup_compact(DedupArgs a, uint64_t items, const uint32_t *__restrict__ flags,
                                                       const uint32_t *__restrict__ pos,
                                                       const uint32_t *__restrict__ vals, uint32_t *__restrict__ out) {
    const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= items || !flags[e]) return;
    int c;
    uint32_t q;
    dedup_item_of(a, vals[e], c, q);
    out[pos[e]] = q;
}

// seg_counts[0] = flags set among the sorted items of class 0 (those before
// *boundary), [1] = the rest (pos: the exclusive scan of the flags, total: their sum).
__global__ void k_dedup_seg_counts(const uint32_t *__restrict__ pos, const uint32_t *__restrict__ total,
                                   const uint32_t *__restrict__ boundary, uint64_t items,
                                   uint32_t *__restrict__ seg_counts) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const uint64_t items0 = *boundary;
        const uint32_t d0 = items0 < items ? pos[items0] : *total;
        seg_counts[0] = d0;
        seg_counts[1] = *total - d0;
    }
}

// Distinct candidates per segment from the scan of the flags: the keys are
// sorted with the segment id in their top bits, so segment s occupies one
// contiguous range, found by binary search (no atomics).
__global__ void k_seg_counts(const uint64_t *__restrict__ keys, size_t m, const uint32_t *__restrict__ pos,
                             const uint32_t *__restrict__ total, int segbits, uint32_t nseg,
                             uint32_t *__restrict__ seg_counts, uint32_t *__restrict__ seg_offsets) {
    uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nseg) return;
    auto lower = [&](uint64_t v) -> size_t {   // first index with key >= v
        size_t lo = 0, hi = m;
        while (lo < hi) {
            size_t mid = (lo + hi) >> 1;
            if (keys[mid] < v) lo = mid + 1;
            else hi = mid;
        }
        return lo;
    };
    const uint64_t a = (uint64_t)s << (64 - segbits);
    const size_t ia = lower(a);
    const size_t ib = (s + 1 < (1u << segbits)) ? lower((uint64_t)(s + 1) << (64 - segbits)) : m;
    const uint32_t pa = ia < m ? pos[ia] : *total;
    const uint32_t pb = ib < m ? pos[ib] : *total;
    seg_counts[s] = pb - pa;
    if (seg_offsets) seg_offsets[s] = pa;
}

__global__ void k_compact(const uint32_t *__restrict__ flags, const uint32_t *__restrict__ pos,
                          const uint32_t *__restrict__ vals, size_t m, uint32_t *__restrict__ out,
                          uint32_t *__restrict__ idx, const uint32_t *__restrict__ perm) {
    size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < m && flags[e]) {
        const uint32_t v = perm ? perm[e] : (uint32_t)e;
        out[pos[e]] = vals[v];
        if (idx) idx[pos[e]] = v;
    }
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

// OR and AND of every word over the candidates ids[0..m): constant bits need no
// sort pass.  A bounded grid strides over the ids; each workgroup reduces in
// registers and LDS and adds one atomic per word.
__global__ __launch_bounds__(256) void k_word_range(const uint64_t *__restrict__ X, uint32_t n, uint32_t KS, uint32_t K,
                                                   const uint32_t *__restrict__ ids, size_t m,
                                                   unsigned long long *__restrict__ orv,
                                                   unsigned long long *__restrict__ andv) {
    __shared__ unsigned long long sor[4][64], sand[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (uint32_t k0 = 0; k0 < K; k0 += 64) {
        const uint32_t kk = K - k0 < 64 ? K - k0 : 64;
        // per-thread partials for words k0 + (0..kk), one word at a time to bound registers
        for (uint32_t k = 0; k < kk; ++k) {
            uint64_t o = 0, a = ~0ull;
            for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (size_t)gridDim.x * blockDim.x) {
                uint32_t i, j;
                decode_pair(ids[e], n, i, j);
                uint64_t w = X[(size_t)i * KS + k0 + k] & X[(size_t)j * KS + k0 + k];
                o |= w;
                a &= w;
            }
            for (int sh = 32; sh > 0; sh >>= 1) {
                o |= __shfl_xor(o, sh, 64);
                a &= __shfl_xor(a, sh, 64);
            }
            if (lane == 0) { sor[wave][k] = o; sand[wave][k] = a; }
        }
        __syncthreads();
        if (threadIdx.x < kk) {
            const int k = threadIdx.x;
            unsigned long long o = sor[0][k] | sor[1][k] | sor[2][k] | sor[3][k];
            unsigned long long a = sand[0][k] & sand[1][k] & sand[2][k] & sand[3][k];
            atomicOr(&orv[k0 + k], o);
            atomicAnd(&andv[k0 + k], a);
        }
        __syncthreads();
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

// The same rows without the repeat flags, one thread per word: the KS threads of a
// row read and write its words side by side, so loads and stores coalesce.  A
// workgroup takes 256 / KS rows.
__global__ __launch_bounds__(256) void k_materialize_words(const uint64_t *__restrict__ X, uint32_t n, uint32_t KS,
                                                          const uint32_t *__restrict__ ids, size_t m,
                                                          uint64_t *__restrict__ W) {
    const uint32_t per = 256u / KS, lr = threadIdx.x / KS, k = threadIdx.x - lr * KS;
    const size_t e = (size_t)blockIdx.x * per + lr;
    if (lr >= per || e >= m) return;
    uint32_t i, j;
    decode_pair(ids[e], n, i, j);
    W[e * KS + k] = X[(size_t)i * KS + k] & X[(size_t)j * KS + k];
}

// The same for rows of an even number of words, two words (16 bytes) per thread;
// len[e] (when given) = the number of tokens of row e, |b| of Eq. 2.
__global__ __launch_bounds__(256) void k_materialize_words16(const uint4 *__restrict__ X, uint32_t n, uint32_t K2,
                                                            const uint32_t *__restrict__ ids, size_t m,
                                                            uint4 *__restrict__ W, uint32_t *__restrict__ len) {
    __shared__ uint32_t cnt[256];
    const uint32_t per = 256u / K2, lr = threadIdx.x / K2, k = threadIdx.x - lr * K2;
    const size_t e = (size_t)blockIdx.x * per + lr;
    const bool act = lr < per && e < m;
    if (len) {
        cnt[threadIdx.x] = 0;
        __syncthreads();
    }
    if (act) {
        uint32_t i, j;
        decode_pair(ids[e], n, i, j);
        const uint4 a = X[(size_t)i * K2 + k], b = X[(size_t)j * K2 + k];
        const uint4 v = make_uint4(a.x & b.x, a.y & b.y, a.z & b.z, a.w & b.w);
        W[e * K2 + k] = v;
        if (len) atomicAdd(&cnt[lr], (uint32_t)(__popc(v.x) + __popc(v.y) + __popc(v.z) + __popc(v.w)));
    }
    if (len) {
        __syncthreads();
        if (act && k == 0) len[e] = cnt[lr];
    }
}

// S[e] = f[e] |b_e|^2 from the rows' token counts (Eq. 2)
__global__ void k_weights_len(const uint32_t *__restrict__ f, const uint32_t *__restrict__ len, size_t m,
                              int64_t *__restrict__ S) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < m) S[e] = (int64_t)f[e] * (int64_t)len[e] * (int64_t)len[e];
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
// out [m][KD] = the first KD <= KS words of rows ids[e] of W [.][KS]
__global__ void k_gather_rows(const uint64_t *__restrict__ W, const uint32_t *__restrict__ ids, size_t m,
                              uint32_t KS, uint32_t KD, uint64_t *__restrict__ out, const uint32_t *__restrict__ fin,
                              uint32_t *__restrict__ fout, const uint32_t *__restrict__ ids2) {
    size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= m * KD) return;
    size_t e = g / KD, k = g % KD;
    const uint32_t r = ids2 ? ids2[ids[e]] : ids[e];
    out[g] = W[(size_t)r * KS + k];
    if (fin && k == 0) fout[e] = fin[r];
}

// Whole rows of an even number of words, one thread per 16-byte piece (P pieces
// per row): consecutive lanes read a row's pieces together and write contiguously.
template <int P>
__global__ void k_gather_rows16(const uint4 *__restrict__ W, const uint32_t *__restrict__ ids, size_t m,
                                uint4 *__restrict__ out, const uint32_t *__restrict__ fin, uint32_t *__restrict__ fout,
                                const uint32_t *__restrict__ ids2) {
    const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= m * P) return;
    const size_t e = g / P;
    const uint32_t k = (uint32_t)(g % P);
    const uint32_t r = ids2 ? ids2[ids[e]] : ids[e];
    out[g] = W[(size_t)r * P + k];
    if (fin && k == 0) fout[e] = fin[r];
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

// S = f |b|^2 for 256 rows per workgroup: the rows' words are read contiguously
// across the workgroup (a row is KS words, so one lane per row would stride),
// their popcounts kept in LDS, then each lane sums its own row.
constexpr uint32_t kWeightRows = 256;
__global__ __launch_bounds__(256) void k_weights(const uint64_t *__restrict__ W, const uint32_t *__restrict__ f,
                                                 size_t m, uint32_t KS, int64_t *__restrict__ S) {
    __shared__ uint8_t pc[kWeightRows * 64];   // KS <= 64
    const size_t row0 = (size_t)blockIdx.x * kWeightRows;
    const uint32_t rows = (uint32_t)min((size_t)kWeightRows, m - row0);
    const uint32_t words = rows * KS;
    const uint64_t *base = W + row0 * KS;
    for (uint32_t t = threadIdx.x; t < words; t += blockDim.x) pc[t] = (uint8_t)__popcll(base[t]);
    __syncthreads();
    if (threadIdx.x < rows) {
        uint32_t len = 0;
        for (uint32_t k = 0; k < KS; ++k) len += pc[threadIdx.x * KS + k];
        const size_t e = row0 + threadIdx.x;
        S[e] = (int64_t)f[e] * (int64_t)len * (int64_t)len;
    }
}

static dim3 blocks_for(size_t n, unsigned bs = 256) { return dim3((unsigned)((n + bs - 1) / bs)); }

void launch_pair_hash(const uint64_t *X, uint32_t n, uint32_t KS, uint32_t K, uint64_t q0, uint64_t count,
                      uint32_t seg, int segbits, uint64_t *keys, uint32_t *vals, hipStream_t s, int key_bytes) {
    if (!count) return;
    uint64_t seg_hi = (uint64_t)seg << (64 - segbits);
    const uint64_t keep = key_bytes >= 8 ? ~0ull : ~((1ull << (64 - 8 * key_bytes)) - 1);
    hipLaunchKernelGGL(k_pair_hash, blocks_for(count), dim3(256), 0, s, X, n, KS, K, q0, count, seg_hi, segbits, keep,
                       keys, vals);
    IG_HIP(hipGetLastError());
}

void launch_dedup_flags(const uint64_t *keys, const uint32_t *vals, size_t m, const void *segs_dev, int segbits,
                        uint32_t *flags, uint32_t *seg_counts, hipStream_t s) {
    if (!m) return;
    hipLaunchKernelGGL(k_dedup_flags, blocks_for(m), dim3(256), 0, s, keys, vals, m, (const RowsOfSeg *)segs_dev,
                       segbits, flags, seg_counts);
    IG_HIP(hipGetLastError());
}

void launch_seg_counts(const uint64_t *keys, size_t m, const uint32_t *pos, const uint32_t *total, int segbits,
                       uint32_t nseg, uint32_t *seg_counts, hipStream_t s, uint32_t *seg_offsets) {
    if (!nseg) return;
    if (!m) {
        launch_fill_u32(seg_counts, 0u, nseg, s);
        if (seg_offsets) launch_fill_u32(seg_offsets, 0u, nseg, s);
        return;
    }
    hipLaunchKernelGGL(k_seg_counts, dim3((nseg + 63) / 64), dim3(64), 0, s, keys, m, pos, total, segbits, nseg,
                       seg_counts, seg_offsets);
    IG_HIP(hipGetLastError());
}

bool dedup_partitioned_fits(uint64_t items) { return items > 0 && items < (1ull << 32) - 1; }

void launch_dedup_partitioned(const uint64_t *X0, uint32_t n0, uint64_t q00, uint64_t cnt0, const uint64_t *X1,
                              uint32_t n1, uint64_t q01, uint64_t cnt1, uint32_t KS, uint32_t K, uint32_t *cand,
                              uint32_t *total, uint32_t *seg_counts, uint32_t *err, hipStream_t s) {
    const uint64_t items = cnt0 + cnt1;
    IG_REQUIRE(dedup_partitioned_fits(items), IG_E_INVAL, "partitioned de-duplication of that many items");
    DedupArgs a{};
    a.seg[0] = RowsOfSeg{X0, n0, KS, K};
    a.seg[1] = RowsOfSeg{X1, n1, KS, K};
    a.q0[0] = q00;
    a.q0[1] = q01;
    a.gbase[0] = 0;
    a.gbase[1] = cnt0;
    Scratch<uint64_t> k0(items, s), k1(items, s);
    Scratch<uint32_t> v0(items, s), v1(items, s), starts((1u << kPartBits) + 1, s);
    launch_fill_u32(err, 0u, 1, s);
    const unsigned blocks = (unsigned)((items + 255) / 256);
    hipLaunchKernelGGL(k_pair_hash64, dim3(blocks), dim3(256), 0, s, a, items, k0.get(), v0.get());
    IG_HIP(hipGetLastError());
    const int where = radix_sort_pairs(k0.get(), v0.get(), k1.get(), v1.get(), items, 0xc0u, s);   // the top 16 bits
    const uint64_t *ks = where ? k1.get() : k0.get();
    const uint32_t *vs = where ? v1.get() : v0.get();
    hipLaunchKernelGGL(k_part_starts, dim3((unsigned)((items + 1 + 255) / 256)), dim3(256), 0, s, ks, (size_t)items,
                       starts.get());
    IG_HIP(hipGetLastError());
    // the other key array and value array are free now: flags and first copies
    uint32_t *flags = where ? v0.get() : v1.get();
    uint32_t *own = reinterpret_cast<uint32_t *>(where ? k0.get() : k1.get());
    uint32_t *pos = own + items;
    hipLaunchKernelGGL(k_part_dedup, dim3(1u << kPartBits), dim3(256), 0, s, ks, vs, starts.get(), flags, own, err);
    IG_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_dedup_verify, dim3(blocks), dim3(256), 0, s, a, items, vs, own, err);
    IG_HIP(hipGetLastError());
    scan_exclusive_u32(flags, pos, items, total, s);
    hipLaunchKernelGGL(k_dedup_compact, dim3(blocks), dim3(256), 0, s, a, items, flags, pos, vs, cand);
    IG_HIP(hipGetLastError());
    // class 1's partitions begin at 2^15
    hipLaunchKernelGGL(k_dedup_seg_counts, dim3(1), dim3(64), 0, s, pos, total, starts.get() + (1u << (kPartBits - 1)),
                       items, seg_counts);
    IG_HIP(hipGetLastError());
}

size_t rows_of_seg_size() { return sizeof(RowsOfSeg); }
void fill_rows_of_seg(void *dst, const uint64_t *X, uint32_t n, uint32_t KS, uint32_t K) {
    RowsOfSeg r{X, n, KS, K};
    *static_cast<RowsOfSeg *>(dst) = r;
}

void launch_compact(const uint32_t *flags, const uint32_t *pos, const uint32_t *vals, size_t m, uint32_t *out,
                    hipStream_t s, uint32_t *idx, const uint32_t *perm) {
    if (!m) return;
    hipLaunchKernelGGL(k_compact, blocks_for(m), dim3(256), 0, s, flags, pos, vals, m, out, idx, perm);
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
    unsigned g = (unsigned)((m + 255) / 256);
    if (g > 1024) g = 1024;
    hipLaunchKernelGGL(k_word_range, dim3(g), dim3(256), 0, s, X, n, KS, K, ids, m, orv, andv);
    IG_HIP(hipGetLastError());
}

bool launch_materialize(const uint64_t *X, uint32_t n, uint32_t KS, const uint32_t *ids, size_t m, uint64_t *W,
                        uint32_t *newflag, hipStream_t s, uint32_t *len) {
    if (!m) return len != nullptr;
    if (!newflag && KS % 2 == 0 && KS <= 512) {
        // rows are 16-byte aligned: two words per thread
        const uint32_t K2 = KS / 2;
        const size_t per = 256 / K2;
        hipLaunchKernelGGL(k_materialize_words16, dim3((unsigned)((m + per - 1) / per)), dim3(256), 0, s,
                           reinterpret_cast<const uint4 *>(X), n, K2, ids, m, reinterpret_cast<uint4 *>(W), len);
        IG_HIP(hipGetLastError());
        return len != nullptr;
    } else if (!newflag && KS <= 256) {
        const size_t per = 256 / KS;
        hipLaunchKernelGGL(k_materialize_words, dim3((unsigned)((m + per - 1) / per)), dim3(256), 0, s, X, n, KS, ids,
                           m, W);
    } else {
        hipLaunchKernelGGL(k_materialize, blocks_for(m), dim3(256), 0, s, X, n, KS, ids, m, W, newflag);
    }
    IG_HIP(hipGetLastError());
    return false;
}

void launch_compact_rows(const uint64_t *W, const uint32_t *flags, const uint32_t *pos, size_t m, uint32_t KS,
                         uint64_t *out, hipStream_t s) {
    if (!m) return;
    hipLaunchKernelGGL(k_compact_rows, blocks_for(m * KS), dim3(256), 0, s, W, flags, pos, m, KS, out);
    IG_HIP(hipGetLastError());
}

void launch_gather_rows(const uint64_t *W, const uint32_t *ids, size_t m, uint32_t KS, uint32_t KD, uint64_t *out,
                        const uint32_t *fin, uint32_t *fout, hipStream_t s, const uint32_t *ids2) {
    if (!m) return;
    IG_REQUIRE(KD >= 1 && KD <= KS, IG_E_INVAL, "gathered rows wider than the stored rows");
    if (KD == KS && KS % 2 == 0 && KS <= 32) {
        const uint4 *W4 = reinterpret_cast<const uint4 *>(W);
        uint4 *o4 = reinterpret_cast<uint4 *>(out);
        switch (KS / 2) {
#define IG_GR(P)                                                                                                   \
    case P:                                                                                                        \
        hipLaunchKernelGGL(k_gather_rows16<P>, blocks_for(m * P), dim3(256), 0, s, W4, ids, m, o4, fin, fout, ids2); \
        IG_HIP(hipGetLastError());                                                                                 \
        return;
            IG_GR(1) IG_GR(2) IG_GR(3) IG_GR(4) IG_GR(5) IG_GR(6) IG_GR(7) IG_GR(8)
            IG_GR(9) IG_GR(10) IG_GR(11) IG_GR(12) IG_GR(13) IG_GR(14) IG_GR(15) IG_GR(16)
#undef IG_GR
            default: break;
        }
    }
    hipLaunchKernelGGL(k_gather_rows, blocks_for(m * KD), dim3(256), 0, s, W, ids, m, KS, KD, out, fin, fout, ids2);
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

void launch_weights_len(const uint32_t *f, const uint32_t *len, size_t m, int64_t *S, hipStream_t s) {
    if (!m) return;
    hipLaunchKernelGGL(k_weights_len, blocks_for(m), dim3(256), 0, s, f, len, m, S);
    IG_HIP(hipGetLastError());
}

void launch_weights(const uint64_t *W, const uint32_t *f, size_t m, uint32_t KS, int64_t *S, hipStream_t s) {
    if (!m) return;
    IG_REQUIRE(KS >= 1 && KS <= 64, IG_E_UNSUPPORTED, "pattern rows wider than 64 words");
    hipLaunchKernelGGL(k_weights, blocks_for(m, kWeightRows), dim3(256), 0, s, W, f, m, KS, S);
    IG_HIP(hipGetLastError());
}

void launch_iota(uint32_t *v, size_t m, hipStream_t s) {
    if (!m) return;
    hipLaunchKernelGGL(k_iota, blocks_for(m), dim3(256), 0, s, v, m);
    IG_HIP(hipGetLastError());
}

// ------------------------------------------------------ compressed sort keys ----
// Pieces come sorted by key word, then significance, so each lane walks them in
// order: a row word is loaded when the piece list reaches it, a key word is
// written when the list leaves it.  The piece list is uniform over the wave.
__global__ __launch_bounds__(256) void k_compress_keys(const uint64_t *__restrict__ X, uint32_t n, uint32_t KS,
                                                      const uint32_t *__restrict__ ids, size_t m,
                                                      const KeyPiece *__restrict__ pieces, uint32_t npieces,
                                                      uint64_t *__restrict__ keys) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    const uint64_t *ra, *rb;
    if (ids) {
        uint32_t i, j;
        decode_pair(ids[e], n, i, j);
        ra = X + (size_t)i * KS;
        rb = X + (size_t)j * KS;
    } else {
        ra = rb = X + e * KS;   // X holds the rows themselves
    }
    uint32_t cur_word = 0xffffffffu, cur_kw = 0;
    uint64_t word = 0, acc = 0;
    for (uint32_t p = 0; p < npieces; ++p) {
        const KeyPiece g = pieces[p];
        if (g.word != cur_word) {
            cur_word = g.word;
            word = ra[cur_word] & rb[cur_word];
        }
        if (g.kw != cur_kw) {
            keys[(size_t)cur_kw * m + e] = acc;
            acc = 0;
            cur_kw = g.kw;
        }
        const uint64_t x = (word >> g.lo) & (g.width >= 64 ? ~0ull : ((1ull << g.width) - 1));
        const uint64_t code = x ? (uint64_t)__ffsll((unsigned long long)x) : 0ull;
        acc |= code << g.shift;
    }
    keys[(size_t)cur_kw * m + e] = acc;
}

__global__ __launch_bounds__(256) void k_key_range(const uint64_t *__restrict__ keys, size_t m,
                                                  unsigned long long *__restrict__ orv,
                                                  unsigned long long *__restrict__ andv) {
    __shared__ unsigned long long so[4], sa[4];
    const uint32_t k = blockIdx.y;
    const uint64_t *kk = keys + (size_t)k * m;
    uint64_t o = 0, a = ~0ull;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (size_t)gridDim.x * blockDim.x) {
        const uint64_t v = kk[e];
        o |= v;
        a &= v;
    }
    for (int sh = 32; sh > 0; sh >>= 1) {
        o |= __shfl_xor(o, sh, 64);
        a &= __shfl_xor(a, sh, 64);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) { so[wave] = o; sa[wave] = a; }
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicOr(&orv[k], so[0] | so[1] | so[2] | so[3]);
        atomicAnd(&andv[k], sa[0] & sa[1] & sa[2] & sa[3]);
    }
}

template <class T>
__global__ void k_permute(const T *__restrict__ src, const uint32_t *__restrict__ perm, size_t m, T *__restrict__ out) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < m) out[e] = src[perm[e]];
}

void launch_compress_keys(const uint64_t *X, uint32_t n, uint32_t KS, const uint32_t *ids, size_t m,
                          const KeyPiece *pieces, uint32_t npieces, uint64_t *keys, hipStream_t s) {
    if (!m) return;
    hipLaunchKernelGGL(k_compress_keys, blocks_for(m), dim3(256), 0, s, X, n, KS, ids, m, pieces, npieces, keys);
    IG_HIP(hipGetLastError());
}

void launch_key_range(const uint64_t *keys, uint32_t nk, size_t m, unsigned long long *orv,
                      unsigned long long *andv, hipStream_t s) {
    if (!m || !nk) return;
    unsigned g = (unsigned)((m + 255) / 256);
    if (g > 256) g = 256;
    hipLaunchKernelGGL(k_key_range, dim3(g, nk), dim3(256), 0, s, keys, m, orv, andv);
    IG_HIP(hipGetLastError());
}

void launch_permute_u64(const uint64_t *src, const uint32_t *perm, size_t m, uint64_t *out, hipStream_t s) {
    if (!m) return;
    hipLaunchKernelGGL(k_permute<uint64_t>, blocks_for(m), dim3(256), 0, s, src, perm, m, out);
    IG_HIP(hipGetLastError());
}

void launch_permute_u32(const uint32_t *src, const uint32_t *perm, size_t m, uint32_t *out, hipStream_t s) {
    if (!m) return;
    hipLaunchKernelGGL(k_permute<uint32_t>, blocks_for(m), dim3(256), 0, s, src, perm, m, out);
    IG_HIP(hipGetLastError());
}

}  // namespace ig
