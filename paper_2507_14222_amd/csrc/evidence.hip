// Evidence of a decision: the coherent patterns inside a flow (Sections 2 and 5
// present them as the readable account of a detection).  For a flow t and a class
// c they are exactly the terms Eq. 4 adds into A(t) (c = 1) or N(t) (c = 0).  The
// k reported are the heaviest: weight S descending, then the words ascending in
// the canonical order (w_0 most significant, unsigned), so the list is unique.
//
// One workgroup per (flow, class).  The flow's words sit in LDS; the patterns
// that can lie inside it are those of the token buckets of its d tokens (a
// pattern inside the flow holds its bucket token, Eq. 6), or all of the class
// when the model has no buckets.  Each thread tests one pattern per round;
// patterns inside that beat the current k-th best are appended to an LDS list,
// which is merged into the best k by a bitonic sort after the round.
#include "common.h"
#include "kernels.h"

namespace ig {

constexpr uint32_t EV_T = 256;          // threads: one pattern each per round
constexpr uint32_t EV_SLOTS = 512;      // best k (<= 256) + one round of candidates
constexpr uint32_t EV_KMAX = EV_SLOTS - EV_T;
constexpr uint32_t EV_NONE = ~0u;

struct EvidenceArgs {
    const uint64_t *W[2];      // pattern rows [np][KS]
    const uint32_t *f[2];
    const int64_t *S[2];
    uint64_t np[2];
    const uint32_t *bperm[2];  // rows grouped by bucket (null: no buckets)
    const uint32_t *brow[2];   // [L + 1] bucket starts in bperm
    uint32_t KS, K, d, k;
    const uint16_t *codes;     // flows [n][d]
    const uint32_t *off;       // token offsets of the features
    const uint16_t *nbins;
    uint32_t *count;           // [n][2]
    uint64_t *words;           // [n][2][k][K]
    uint32_t *fo;              // [n][2][k]
    int64_t *So;               // [n][2][k]
};

// whether pattern p ranks before pattern q (EV_NONE ranks last)
__device__ __forceinline__ bool ranks_before(const EvidenceArgs &a, int c, uint32_t p, int64_t sp, uint32_t q,
                                             int64_t sq) {
    if (q == EV_NONE) return p != EV_NONE;
    if (p == EV_NONE) return false;
    if (sp != sq) return sp > sq;
    const uint64_t *wp = a.W[c] + (size_t)p * a.KS, *wq = a.W[c] + (size_t)q * a.KS;
    for (uint32_t k = 0; k < a.K; ++k)
        if (wp[k] != wq[k]) return wp[k] < wq[k];
    return false;
}

__global__ __launch_bounds__(EV_T) void k_evidence(EvidenceArgs a) {
    const uint32_t t = blockIdx.x, tid = threadIdx.x;
    const int c = (int)blockIdx.y;
    __shared__ uint64_t tw[64];
    __shared__ uint32_t row[EV_SLOTS];
    __shared__ int64_t wt[EV_SLOTS];
    __shared__ uint32_t ncand, nbest, invalid, total;
    for (uint32_t k = tid; k < a.KS; k += EV_T) tw[k] = 0;
    if (tid == 0) {
        ncand = 0;
        nbest = 0;
        invalid = 0;
        total = 0;
    }
    __syncthreads();
    const uint16_t *code = a.codes + (size_t)t * a.d;
    for (uint32_t f = tid; f < a.d; f += EV_T) {
        const uint32_t v = code[f];
        if (v >= a.nbins[f]) {
            atomicOr(&invalid, 1u);
        } else {
            const uint32_t tok = a.off[f] + v;
            atomicOr(reinterpret_cast<unsigned long long *>(&tw[tok >> 6]), 1ull << (tok & 63));
        }
    }
    __syncthreads();
    const size_t o = (size_t)t * 2 + c;
    if (invalid) {   // uniform: a code out of range, no evidence
        if (tid == 0) a.count[o] = EV_NONE;
        for (uint32_t j = tid; j < a.k; j += EV_T) {
            a.fo[o * a.k + j] = 0;
            a.So[o * a.k + j] = 0;
            for (uint32_t w = 0; w < a.K; ++w) a.words[(o * a.k + j) * a.K + w] = 0;
        }
        return;
    }
    const uint64_t *W = a.W[c];
    const int64_t *S = a.S[c];
    const uint32_t *perm = a.bperm[c];
    const uint32_t nranges = perm ? a.d : 1u;
    uint32_t mine = 0;
    for (uint32_t r = 0; r < nranges; ++r) {
        uint32_t lo = 0, hi = (uint32_t)a.np[c];
        if (perm) {
            const uint32_t tok = a.off[r] + code[r];
            lo = a.brow[c][tok];
            hi = a.brow[c][tok + 1];
        }
        for (uint32_t base = lo; base < hi; base += EV_T) {
            const uint32_t pos = base + tid;
            if (pos < hi) {
                const uint32_t p = perm ? perm[pos] : pos;
                bool in = true;
                for (uint32_t k = 0; k < a.KS && in; ++k) in = (W[(size_t)p * a.KS + k] & ~tw[k]) == 0;
                if (in) {
                    ++mine;
                    const int64_t sp = S[p];
                    const uint32_t nb = nbest;   // unchanged during the round
                    const bool keep = nb < a.k || ranks_before(a, c, p, sp, row[a.k - 1], wt[a.k - 1]);
                    if (keep) {
                        const uint32_t i = atomicAdd(&ncand, 1u);
                        row[nb + i] = p;
                        wt[nb + i] = sp;
                    }
                }
            }
            __syncthreads();
            const uint32_t m = nbest + ncand;   // uniform
            if (m > nbest) {
                for (uint32_t j = m + tid; j < EV_SLOTS; j += EV_T) row[j] = EV_NONE;
                __syncthreads();
                // bitonic sort of the EV_SLOTS entries, best first
                for (uint32_t size = 2; size <= EV_SLOTS; size <<= 1) {
                    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
                        const uint32_t i = tid;   // EV_SLOTS / 2 pairs, one per thread
                        const uint32_t x = (i / stride) * 2 * stride + (i % stride), y = x + stride;
                        const bool up = (x & size) == 0;   // this run sorts best first
                        const bool yx = ranks_before(a, c, row[y], wt[y], row[x], wt[x]);
                        const bool xy = ranks_before(a, c, row[x], wt[x], row[y], wt[y]);
                        if (up ? yx : xy) {
                            const uint32_t tr = row[x];
                            const int64_t ts = wt[x];
                            row[x] = row[y];
                            wt[x] = wt[y];
                            row[y] = tr;
                            wt[y] = ts;
                        }
                        __syncthreads();
                    }
                }
                if (tid == 0) nbest = m < a.k ? m : a.k;
            }
            if (tid == 0) ncand = 0;
            __syncthreads();
        }
    }
    atomicAdd(&total, mine);
    __syncthreads();
    if (tid == 0) a.count[o] = total;
    for (uint32_t j = tid; j < a.k; j += EV_T) {
        const bool have = j < nbest;
        const uint32_t p = have ? row[j] : 0u;
        a.fo[o * a.k + j] = have ? a.f[c][p] : 0u;
        a.So[o * a.k + j] = have ? wt[j] : 0;
        for (uint32_t w = 0; w < a.K; ++w) a.words[(o * a.k + j) * a.K + w] = have ? W[(size_t)p * a.KS + w] : 0ull;
    }
}

uint32_t evidence_max_k() { return EV_KMAX; }

void launch_evidence(const EvidenceModel &m, const uint16_t *codes, uint32_t n, uint32_t k, uint32_t *count,
                     uint64_t *words, uint32_t *f, int64_t *S, hipStream_t s) {
    IG_REQUIRE(k >= 1 && k <= EV_KMAX, IG_E_INVAL, "k must be in 1..256");
    IG_REQUIRE(m.KS <= 64, IG_E_UNSUPPORTED, "rows wider than 64 words");
    if (!n) return;
    EvidenceArgs a{};
    for (int c = 0; c < 2; ++c) {
        a.W[c] = m.W[c];
        a.f[c] = m.f[c];
        a.S[c] = m.S[c];
        a.np[c] = m.np[c];
        a.bperm[c] = m.bperm[c];
        a.brow[c] = m.brow[c];
    }
    IG_REQUIRE((m.bperm[0] != nullptr) == (m.bperm[1] != nullptr), IG_E_DEVICE, "bucket lists of one class only");
    a.KS = m.KS;
    a.K = m.K;
    a.d = m.d;
    a.k = k;
    a.codes = codes;
    a.off = m.off;
    a.nbins = m.nbins;
    a.count = count;
    a.words = words;
    a.fo = f;
    a.So = S;
    hipLaunchKernelGGL(k_evidence, dim3(n, 2), dim3(EV_T), 0, s, a);
    IG_HIP(hipGetLastError());
}

}  // namespace ig
