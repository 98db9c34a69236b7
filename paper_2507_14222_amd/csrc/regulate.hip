// The classifier of Section 3.1 on the device: Regulations 1-3 applied to the
// evidence (A, N) of each flow (Eq. 4), and the detection metrics of Table 2.
//
//   Regulation 1  attack when A >= N
//   Regulation 2  attack when A = N = 0 (already attack by Regulation 1; it is
//                 reported as the deciding rule)
//   Regulation 3  attack when N < mu_N - r sigma_N, with mu_N and sigma_N the mean
//                 and the population standard deviation of N over the normal
//                 training records and r a given constant
//
// Everything is integer: the moments are exact multi-word sums, the Regulation 3
// cut is an integer threshold found on the host with exact big-integer
// arithmetic, and the metrics are counts (the AUC as an exact fraction).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"
#include "kernels.h"

namespace ig {

// ------------------------------------------------------------- moments ----
// One workgroup of 1024 threads: the count, the sum (128 bits) and the sum of
// squares (192 bits) of N over the records labelled 0 whose scores are valid;
// *err |= 1 for a label other than 0 or 1.  out[0] = count, out[1..2] = sum,
// out[3..5] = sum of squares (little-endian words).
__device__ __forceinline__ void add_words(uint64_t *acc, const uint64_t *v, int nw) {
    uint64_t carry = 0;
    for (int i = 0; i < nw; ++i) {
        const uint64_t a = acc[i], s1 = a + v[i], c1 = s1 < a;
        const uint64_t s2 = s1 + carry, c2 = s2 < s1;
        acc[i] = s2;
        carry = c1 | c2;
    }
}

__global__ __launch_bounds__(1024) void k_normal_moments(const int64_t *__restrict__ scores,
                                                         const uint8_t *__restrict__ labels, uint32_t n,
                                                         unsigned long long *__restrict__ out,
                                                         uint32_t *__restrict__ err) {
    __shared__ uint64_t sh[1024][6];
    uint64_t acc[6] = {0, 0, 0, 0, 0, 0};
    uint32_t bad = 0;
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
        const uint32_t lab = labels[i];
        bad |= lab > 1u;
        const int64_t A = scores[2 * (size_t)i], N = scores[2 * (size_t)i + 1];
        if (lab != 0u || (A == -1 && N == -1) || N < 0) continue;
        const uint64_t v = (uint64_t)N;
        const uint64_t one[1] = {1};
        const uint64_t s[2] = {v, 0};
        const uint64_t q[3] = {v * v, __umul64hi(v, v), 0};
        add_words(acc, one, 1);
        add_words(acc + 1, s, 2);
        add_words(acc + 3, q, 3);
    }
    if (bad) atomicOr(err, 1u);
    for (int w = 0; w < 6; ++w) sh[threadIdx.x][w] = acc[w];
    __syncthreads();
    for (uint32_t o = 512; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            uint64_t *a = sh[threadIdx.x];
            const uint64_t *b = sh[threadIdx.x + o];
            add_words(a, b, 1);
            add_words(a + 1, b + 1, 2);
            add_words(a + 3, b + 3, 3);
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) out[threadIdx.x] = sh[0][threadIdx.x];
}

void normal_moments(const int64_t *scores, const uint8_t *labels, uint32_t n, ig_moments *h, hipStream_t s) {
    Scratch<unsigned long long> d(6, s);
    Scratch<uint32_t> err(1, s);
    launch_fill_u32(err.get(), 0u, 1, s);
    hipLaunchKernelGGL(k_normal_moments, dim3(1), dim3(1024), 0, s, scores, labels, n, d.get(), err.get());
    IG_HIP(hipGetLastError());
    unsigned long long r[6];
    uint32_t e = 0;
    IG_HIP(hipMemcpyAsync(r, d.get(), sizeof(r), hipMemcpyDeviceToHost, s));
    IG_HIP(hipMemcpyAsync(&e, err.get(), 4, hipMemcpyDeviceToHost, s));
    IG_HIP(hipStreamSynchronize(s));
    IG_REQUIRE(!e, IG_E_INVAL, "a label is not 0 or 1");
    h->count = r[0];
    h->sum[0] = r[1];
    h->sum[1] = r[2];
    h->sumsq[0] = r[3];
    h->sumsq[1] = r[4];
    h->sumsq[2] = r[5];
}

// ----------------------------------------------- the Regulation 3 cut ----
// Non-negative big integers (32-bit limbs, least significant first), only what
// the threshold needs: products, shifts, comparison.
namespace {
struct Big {
    std::vector<uint32_t> l;
    static Big of(const uint64_t *w, int nw) {
        Big b;
        for (int i = 0; i < nw; ++i) {
            b.l.push_back((uint32_t)w[i]);
            b.l.push_back((uint32_t)(w[i] >> 32));
        }
        b.trim();
        return b;
    }
    static Big u64(uint64_t v) { return of(&v, 1); }
    void trim() {
        while (!l.empty() && l.back() == 0) l.pop_back();
    }
};

Big mul(const Big &a, const Big &b) {
    Big r;
    if (a.l.empty() || b.l.empty()) return r;
    r.l.assign(a.l.size() + b.l.size(), 0);
    for (size_t i = 0; i < a.l.size(); ++i) {
        uint64_t carry = 0;
        for (size_t j = 0; j < b.l.size(); ++j) {
            const uint64_t t = (uint64_t)a.l[i] * b.l[j] + r.l[i + j] + carry;
            r.l[i + j] = (uint32_t)t;
            carry = t >> 32;
        }
        size_t k = i + b.l.size();
        while (carry) {
            const uint64_t t = (uint64_t)r.l[k] + carry;
            r.l[k++] = (uint32_t)t;
            carry = t >> 32;
        }
    }
    r.trim();
    return r;
}

Big shl(const Big &a, uint32_t bits) {
    if (a.l.empty()) return a;
    Big r;
    const uint32_t limbs = bits / 32, sh = bits % 32;
    r.l.assign(a.l.size() + limbs + 1, 0);
    for (size_t i = 0; i < a.l.size(); ++i) {
        const uint64_t v = (uint64_t)a.l[i] << sh;
        r.l[i + limbs] |= (uint32_t)v;
        r.l[i + limbs + 1] |= (uint32_t)(v >> 32);
    }
    r.trim();
    return r;
}

int cmp(const Big &a, const Big &b) {
    if (a.l.size() != b.l.size()) return a.l.size() < b.l.size() ? -1 : 1;
    for (size_t i = a.l.size(); i-- > 0;)
        if (a.l[i] != b.l[i]) return a.l[i] < b.l[i] ? -1 : 1;
    return 0;
}

// a - b for a >= b
Big sub(const Big &a, const Big &b) {
    Big r = a;
    int64_t borrow = 0;
    for (size_t i = 0; i < r.l.size(); ++i) {
        int64_t t = (int64_t)r.l[i] - (i < b.l.size() ? (int64_t)b.l[i] : 0) - borrow;
        borrow = t < 0;
        if (t < 0) t += (int64_t)1 << 32;
        r.l[i] = (uint32_t)t;
    }
    r.trim();
    return r;
}
}  // namespace

// Regulation 3 fires for N exactly when G = S1 - n N > 0 and
// G^2 > r^2 (n S2 - S1^2), with S1, S2 the sum and the sum of squares of the
// normal records' N and n their count (mu = S1 / n, sigma^2 = (n S2 - S1^2) / n^2).
// With r = M 2^E (M an integer, the exact value of the double) both sides are
// integers after scaling by a power of two.  The condition weakens as N grows, so
// it holds exactly for N < T; T is found by bisection over [0, ceil(S1 / n)].
int64_t r3_threshold(const ig_moments &mo, double r) {
    IG_REQUIRE(std::isfinite(r) && r >= 0.0, IG_E_INVAL, "r must be a finite non-negative number");
    IG_REQUIRE(mo.count > 0, IG_E_INVAL, "no normal training records: mu_N and sigma_N are undefined");
    const Big n = Big::u64(mo.count), S1 = Big::of(mo.sum, 2), S2 = Big::of(mo.sumsq, 3);
    const Big nS2 = mul(n, S2), S1sq = mul(S1, S1);
    IG_REQUIRE(cmp(nS2, S1sq) >= 0, IG_E_INVAL, "inconsistent moments (negative variance)");
    const Big D = sub(nS2, S1sq);
    // r = M * 2^E exactly
    int ex = 0;
    const double fr = std::frexp(r, &ex);            // r = fr * 2^ex, fr in [0.5, 1)
    const uint64_t M = (uint64_t)std::ldexp(fr, 53);  // exact: 53 significant bits
    const int E = ex - 53;
    const Big M2D = mul(mul(Big::u64(M), Big::u64(M)), D);
    // fires(N): G > 0 and G^2 * 2^(-2E) > M^2 D (E < 0), or G^2 > M^2 D 2^(2E) (E >= 0)
    const Big rhs = E >= 0 ? shl(M2D, (uint32_t)(2 * E)) : M2D;
    auto fires = [&](uint64_t N) {
        const Big nN = mul(n, Big::u64(N));
        if (cmp(S1, nN) <= 0) return false;
        const Big G = sub(S1, nN);
        Big G2 = mul(G, G);
        if (E < 0) G2 = shl(G2, (uint32_t)(-2 * E));
        return cmp(G2, rhs) > 0;
    };
    // hi = ceil(S1 / n) fits 64 bits (every N < 2^63); fires(hi) is false
    uint64_t lo = 0, hi;
    {
        // S1 / n by bisection on 64-bit values (S1 < 2^95, n >= 1)
        uint64_t a = 0, b = ~0ull >> 1;
        while (a < b) {   // smallest q with q * n >= S1
            const uint64_t mid = a + (b - a) / 2;
            if (cmp(mul(n, Big::u64(mid)), S1) >= 0) b = mid;
            else a = mid + 1;
        }
        hi = a;
    }
    if (!fires(lo)) return 0;
    // fires(lo), !fires(hi): the threshold is the first N that does not fire
    while (hi - lo > 1) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if (fires(mid)) lo = mid;
        else hi = mid;
    }
    return (int64_t)hi;
}

// -------------------------------------------------------------- labels ----
// label[t]: 1 attack, 0 normal, 255 for a flow without valid scores (-1, -1);
// rule[t]: the regulation that decided (1, 2 or 3; 0 for an invalid flow).
__global__ void k_classify(const int64_t *__restrict__ scores, uint32_t n, int64_t r3_cut, uint32_t use_r2,
                           uint32_t use_r3, uint8_t *__restrict__ label, uint8_t *__restrict__ rule) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int64_t A = scores[2 * (size_t)t], N = scores[2 * (size_t)t + 1];
    uint8_t lab, why;
    if (A == -1 && N == -1) {
        lab = 255;
        why = 0;
    } else {
        lab = A >= N ? 1 : 0;
        why = 1;
        if (use_r2 && A == 0 && N == 0) why = 2;
        if (use_r3 && lab == 0 && N < r3_cut) {
            lab = 1;
            why = 3;
        }
    }
    label[t] = lab;
    if (rule) rule[t] = why;
}

void classify(const int64_t *scores, uint32_t n, int64_t r3_cut, uint32_t flags, uint8_t *label, uint8_t *rule,
              hipStream_t s) {
    if (!n) return;
    hipLaunchKernelGGL(k_classify, dim3((n + 255) / 256), dim3(256), 0, s, scores, n, r3_cut,
                       (flags & IG_CLASSIFY_NO_R2) ? 0u : 1u, (flags & IG_CLASSIFY_R3) ? 1u : 0u, label, rule);
    IG_HIP(hipGetLastError());
}

// ------------------------------------------------------------- metrics ----
// Confusion counts (attack = positive) over the flows with a valid label, and the
// margins A - N split by truth, as keys whose unsigned order is the signed order.
// cnt: 0 tp, 1 fp, 2 tn, 3 fn, 4 invalid, 5 positives, 6 negatives (u64); err |= 1
// for a truth other than 0 or 1.
__global__ void k_confusion(const int64_t *__restrict__ scores, const uint8_t *__restrict__ pred,
                            const uint8_t *__restrict__ truth, uint32_t n, unsigned long long *__restrict__ cnt,
                            uint64_t *__restrict__ pos_keys, uint64_t *__restrict__ neg_keys, uint32_t *__restrict__ err) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const uint32_t tr = truth[t], p = pred[t];
    if (tr > 1u) {
        atomicOr(err, 1u);
        return;
    }
    if (p > 1u) {
        atomicAdd(&cnt[4], 1ull);
        return;
    }
    atomicAdd(&cnt[tr ? (p ? 0 : 3) : (p ? 1 : 2)], 1ull);
    const int64_t margin = scores[2 * (size_t)t] - scores[2 * (size_t)t + 1];
    const uint64_t key = (uint64_t)margin ^ (1ull << 63);
    if (tr) pos_keys[atomicAdd(&cnt[5], 1ull)] = key;
    else neg_keys[atomicAdd(&cnt[6], 1ull)] = key;
}

// auc += 2 * (negatives with a smaller margin) + (negatives with the same margin),
// for every positive, against the ascending negative keys
__global__ void k_auc_pairs(const uint64_t *__restrict__ pos_keys, uint64_t npos, const uint64_t *__restrict__ neg,
                            uint64_t nneg, unsigned long long *__restrict__ auc) {
    __shared__ unsigned long long part[256];
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long v = 0;
    if (i < npos) {
        const uint64_t k = pos_keys[i];
        uint64_t a = 0, b = nneg;   // first >= k
        while (a < b) {
            const uint64_t m = (a + b) / 2;
            if (neg[m] < k) a = m + 1;
            else b = m;
        }
        const uint64_t below = a;
        b = nneg;                    // first > k
        while (a < b) {
            const uint64_t m = (a + b) / 2;
            if (neg[m] <= k) a = m + 1;
            else b = m;
        }
        v = 2 * below + (a - below);
    }
    part[threadIdx.x] = v;
    __syncthreads();
    for (uint32_t o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0 && part[0]) atomicAdd(auc, part[0]);
}

void detection_metrics(const int64_t *scores, const uint8_t *pred, const uint8_t *truth, uint32_t n, ig_metrics *h,
                       hipStream_t s) {
    std::memset(h, 0, sizeof(*h));
    if (!n) return;
    Scratch<unsigned long long> cnt(8, s);
    Scratch<uint64_t> pos(n, s), neg(n, s), neg2(n, s);
    Scratch<uint32_t> err(1, s), v0(n, s), v1(n, s);
    launch_fill_u64(reinterpret_cast<uint64_t *>(cnt.get()), 0ull, 8, s);
    launch_fill_u32(err.get(), 0u, 1, s);
    const unsigned blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_confusion, dim3(blocks), dim3(256), 0, s, scores, pred, truth, n, cnt.get(), pos.get(),
                       neg.get(), err.get());
    IG_HIP(hipGetLastError());
    unsigned long long c[8];
    uint32_t e = 0;
    IG_HIP(hipMemcpyAsync(c, cnt.get(), sizeof(c), hipMemcpyDeviceToHost, s));
    IG_HIP(hipMemcpyAsync(&e, err.get(), 4, hipMemcpyDeviceToHost, s));
    IG_HIP(hipStreamSynchronize(s));
    IG_REQUIRE(!e, IG_E_INVAL, "a truth label is not 0 or 1");
    const uint64_t npos = c[5], nneg = c[6];
    const uint64_t *sorted = neg.get();
    if (nneg > 1) {
        launch_iota(v0.get(), nneg, s);
        const int where = radix_sort_pairs(neg.get(), v0.get(), neg2.get(), v1.get(), nneg, 0xffu, s);
        sorted = where ? neg2.get() : neg.get();
    }
    launch_fill_u64(reinterpret_cast<uint64_t *>(cnt.get()) + 7, 0ull, 1, s);
    if (npos && nneg) {
        hipLaunchKernelGGL(k_auc_pairs, dim3((unsigned)((npos + 255) / 256)), dim3(256), 0, s, pos.get(), npos,
                           sorted, nneg, cnt.get() + 7);
        IG_HIP(hipGetLastError());
    }
    unsigned long long auc = 0;
    IG_HIP(hipMemcpyAsync(&auc, cnt.get() + 7, 8, hipMemcpyDeviceToHost, s));
    IG_HIP(hipStreamSynchronize(s));
    h->tp = c[0];
    h->fp = c[1];
    h->tn = c[2];
    h->fn = c[3];
    h->invalid = c[4];
    h->auc_num = auc;
    h->auc_den = 2 * npos * nneg;
}

}  // namespace ig
