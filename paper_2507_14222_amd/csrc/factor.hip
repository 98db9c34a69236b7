// Operand rows for the matrix-core subset tests: the one-hot words themselves, or
// their factored form (bit and presence tokens per feature; see FactorView).
#include <algorithm>
#include <cstddef>

#include "common.h"
#include "kernels.h"

namespace ig {

// Bin of feature ft in a one-hot row (word(w) returns word w), or -1 when the row
// holds none of its tokens.  Rows of a fit from codes hold at most one.
template <class Word>
__device__ __forceinline__ int feature_code(const Word &word, const FacFeature ft) {
    const uint32_t a = ft.off, b = ft.off + ft.nb;
    for (uint32_t w = a / 64; w * 64 < b; ++w) {
        const uint32_t lo = a > w * 64 ? a - w * 64 : 0;
        const uint32_t hi = b < w * 64 + 64 ? b - w * 64 : 64;
        uint64_t x = word(w) >> lo;
        if (hi - lo < 64) x &= (1ull << (hi - lo)) - 1;
        if (x) return (int)(w * 64 + lo + (uint32_t)__builtin_ctzll(x) - a);
    }
    return -1;
}

// The feature walk is uniform over the wave (every lane follows the same table);
// each lane's row words are re-read from L1/L2 when a feature needs them, and the
// tokens of its bin come from the mask table (L1/L2 resident).
__global__ __launch_bounds__(256) void k_operand_rows(const uint64_t *__restrict__ X, uint32_t n,
                                                     const uint32_t *__restrict__ ids,
                                                     const uint64_t *__restrict__ W, uint32_t KS, size_t m,
                                                     FactorView fv, uint32_t KO, uint64_t flip,
                                                     uint64_t *__restrict__ out) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    const uint64_t *ra, *rb;
    if (ids) {
        uint32_t i, j;
        decode_pair(ids[e], n, i, j);
        ra = X + (size_t)i * KS;
        rb = X + (size_t)j * KS;
    } else {
        ra = rb = W + e * KS;
    }
    auto word = [&](uint32_t w) { return ra[w] & rb[w]; };
    if (!fv.KF) {
        for (uint32_t k = 0; k < KO; ++k) out[e * KO + k] = word(k) ^ flip;
        return;
    }
    for (uint32_t ow = 0; ow < KO; ++ow) {
        uint64_t acc = 0, pres = 0;
        for (uint32_t f = fv.fbeg[ow]; f < fv.fend[ow]; ++f) {
            const FacFeature ft = fv.feat[f];
            if (ow - ft.w0 >= ft.nw) continue;   // a one-bin feature has no tokens
            const int code = feature_code(word, ft);
            if (code >= 0) {
                acc |= fv.mask[ft.mask + (uint32_t)code * ft.nw + (ow - ft.w0)];
                pres |= fv.fbit[2 * f + (ow - ft.w0)];
            }
        }
        if (fv.ternary) {
            out[e * 2 * KO + ow] = pres;
            out[e * 2 * KO + KO + ow] = acc;
        } else {
            out[e * KO + ow] = acc ^ flip;
        }
    }
}

// One-hot operand rows (no factoring table): one lane per output word, so the
// loads of a row's words and the stores are contiguous across the wave.
__global__ __launch_bounds__(256) void k_operand_rows_onehot(const uint64_t *__restrict__ X, uint32_t n,
                                                            const uint32_t *__restrict__ ids,
                                                            const uint64_t *__restrict__ W, uint32_t KS, size_t m,
                                                            uint64_t flip, uint64_t *__restrict__ out) {
    const size_t total = m * KS;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
        uint64_t v;
        if (ids) {
            const size_t e = t / KS;
            const uint32_t k = (uint32_t)(t - e * KS);
            uint32_t i, j;
            decode_pair(ids[e], n, i, j);
            v = X[(size_t)i * KS + k] & X[(size_t)j * KS + k];
        } else {
            v = W[t];
        }
        out[t] = v ^ flip;
    }
}

// Factoring for rows of at most 40 one-hot words, masks in LDS: each lane loads
// its row once into registers and walks the pieces of each word.  The piece table
// is read one 16-byte piece at a time at wave-uniform addresses (scalar loads), every step is
// branch-free (a piece with no bit set ORs zeros), and the output word is a
// wave-uniform register index.  Workgroups stride over the rows, so each stages
// the masks once.
// At most 2 masks per one-hot token: 16 x 64 tokens fill the narrow widths' table.
constexpr uint32_t kLdsMasks = 2048;   // u64 masks staged in LDS (16 KB)
// wider storage (20 to 40 words) stages its whole mask table: 2 masks per token at most
__host__ __device__ constexpr uint32_t lds_masks(int KS) { return KS <= 16 ? kLdsMasks : 2u * 64u * (uint32_t)KS; }
static_assert(sizeof(FacPiece) == 16 && offsetof(FacPiece, base) == 4 && offsetof(FacPiece, mask) == 8,
              "the kernel reads a piece as four dwords");

// LPIECES: the piece table is staged in LDS too (a launch of few rows would
// otherwise wait on one scalar-cache miss per piece on every CU it touches) and
// read back to scalar registers with readfirstlane.
constexpr uint32_t kLdsPieces = 512;

// TERN: a ternary view (FactorView::ternary): rows of 2 KO words, P (the tokens
// of each feature whose bin the row holds, fbit of the piece's feature) then V.
template <int KS, bool LPIECES, bool TERN>
__global__ __launch_bounds__(256) void k_operand_rows_reg(const uint64_t *__restrict__ X, uint32_t n,
                                                         const uint32_t *__restrict__ ids,
                                                         const uint64_t *__restrict__ W, size_t m, FactorView fv,
                                                         uint32_t KO, uint64_t flip, uint64_t *__restrict__ out) {
    __shared__ uint64_t smask[lds_masks(KS) + 1];   // + 1: the second word read next to the last entry
    __shared__ uint4 spiece[LPIECES ? kLdsPieces : 1];
    for (uint32_t t = threadIdx.x; t <= fv.nmask; t += blockDim.x) smask[t] = t < fv.nmask ? fv.mask[t] : 0ull;
    const uint4 *pw = reinterpret_cast<const uint4 *>(fv.piece);
    if (LPIECES)
        for (uint32_t t = threadIdx.x; t < fv.npiece; t += blockDim.x) spiece[t] = pw[t];
    __syncthreads();
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (size_t)gridDim.x * blockDim.x) {
        uint64_t w[KS];
        if (ids) {
            uint32_t i, j;
            decode_pair(ids[e], n, i, j);
#pragma unroll
            for (int k = 0; k < KS; ++k) w[k] = X[(size_t)i * KS + k] & X[(size_t)j * KS + k];
        } else {
#pragma unroll
            for (int k = 0; k < KS; ++k) w[k] = W[e * KS + k];
        }
        uint64_t acc[16] = {};
        uint64_t pres[TERN ? 16 : 1] = {};
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const uint32_t p1 = fv.pbeg[k + 1];
            for (uint32_t p = fv.pbeg[k]; p < p1; ++p) {
                uint4 pc;
                if (LPIECES) {
                    const uint4 v = spiece[p];   // same address in every lane
                    pc = make_uint4(__builtin_amdgcn_readfirstlane(v.x), __builtin_amdgcn_readfirstlane(v.y),
                                    __builtin_amdgcn_readfirstlane(v.z),
                                    TERN ? __builtin_amdgcn_readfirstlane(v.w) : 0u);
                } else {
                    pc = pw[p];
                }
                const uint32_t shape = pc.x, base = pc.y & 0xffffu, mk = pc.z;
                const uint32_t lo = shape & 255u, width = (shape >> 8) & 255u, w0 = (shape >> 16) & 15u;
                const uint32_t nw = shape >> 24;
                const uint64_t keep = width < 64 ? (1ull << width) - 1 : ~0ull;
                const uint64_t x = (w[k] >> lo) & keep;
                // bin base + (lowest set bit), or bin base when the row holds none
                // of the piece's tokens (its masks are then dropped)
                const uint32_t idx = mk + (base + (x ? (uint32_t)__builtin_ctzll(x) : 0u)) * nw;
                const uint64_t m0 = x ? smask[idx] : 0ull;
                const uint64_t m1 = x && nw > 1 ? smask[idx + 1] : 0ull;
                acc[w0] |= m0;
                acc[(w0 + 1) & 15] |= m1;
                if (TERN) {
                    // the feature's tokens when the row holds one of its bins
                    const uint64_t f0 = fv.fbit[2 * pc.w], f1 = nw > 1 ? fv.fbit[2 * pc.w + 1] : 0ull;
                    pres[w0] |= x ? f0 : 0ull;
                    pres[(w0 + 1) & 15] |= x ? f1 : 0ull;
                }
            }
        }
        if (TERN) {
#pragma unroll
            for (int o = 0; o < 16; ++o)
                if ((uint32_t)o < KO) {
                    out[e * 2 * KO + o] = pres[o];
                    out[e * 2 * KO + KO + o] = acc[o];
                }
        } else {
#pragma unroll
            for (int o = 0; o < 16; ++o)
                if ((uint32_t)o < KO) out[e * KO + o] = acc[o] ^ flip;
        }
    }
}

// Rows of record pairs in factored form (see launch_pair_rows_factored).  Two
// records hold the same bin of a feature exactly when their tokens of that
// feature agree, so the pair's row keeps FR[i] AND FR[j] on the features where
// (FR[i] XOR FR[j]) has no bit in the feature's token range and clears the rest.
// A feature whose tokens span two words is tested on both (first pass, one bit
// per such feature).  Each thread takes R rows at once, so one wave-uniform table
// entry (a scalar load) serves R rows.
// TERN: ternary rows (P then V, 2 KO words): the pair keeps P_i AND P_j on the
// features where V_i and V_j agree, and V_i on those.
template <int KO, int R, bool TERN>
__global__ __launch_bounds__(256) void k_pair_rows_factored(const uint64_t *__restrict__ FR, uint32_t n,
                                                           const uint32_t *__restrict__ ids, size_t m,
                                                           const uint4 *__restrict__ wfe,
                                                           const uint32_t *__restrict__ wbeg,
                                                           uint64_t *__restrict__ out) {
    constexpr int RW = TERN ? 2 * KO : KO;   // words per row
    const size_t T = (size_t)gridDim.x * blockDim.x;
    for (size_t e0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e0 < m; e0 += T * R) {
        uint64_t x[R][KO], keep[R][KO], val[R][TERN ? KO : 1];
        uint32_t D[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const size_t e = e0 + r * T;
            uint32_t i = 0, j = 0;
            if (e < m) decode_pair(ids[e], n, i, j);
            if (TERN) {
                // both rows as 16-byte loads (2 KO words each; rows are 16-byte aligned):
                // half as many scattered loads as word by word
                uint64_t wi[RW], wj[RW];
                const uint4 *ri = reinterpret_cast<const uint4 *>(FR + (size_t)i * RW);
                const uint4 *rj = reinterpret_cast<const uint4 *>(FR + (size_t)j * RW);
#pragma unroll
                for (int q = 0; q < KO; ++q) {
                    const uint4 a = ri[q], b = rj[q];
                    wi[2 * q] = (uint64_t)a.y << 32 | a.x;
                    wi[2 * q + 1] = (uint64_t)a.w << 32 | a.z;
                    wj[2 * q] = (uint64_t)b.y << 32 | b.x;
                    wj[2 * q + 1] = (uint64_t)b.w << 32 | b.z;
                }
#pragma unroll
                for (int o = 0; o < KO; ++o) {
                    x[r][o] = wi[KO + o] ^ wj[KO + o];
                    keep[r][o] = wi[o] & wj[o];
                    val[r][TERN ? o : 0] = wi[KO + o];
                }
            } else {
#pragma unroll
                for (int o = 0; o < KO; ++o) {
                    const uint64_t a = FR[(size_t)i * KO + o], b = FR[(size_t)j * KO + o];
                    x[r][o] = a ^ b;
                    keep[r][o] = a & b;
                }
            }
            D[r] = 0;
        }
#pragma unroll
        for (int o = 0; o < KO; ++o)
            for (uint32_t q = wbeg[o]; q < wbeg[o + 1]; ++q) {
                const uint4 t = wfe[q];
                if (!t.y) continue;
                const uint64_t rg = (uint64_t)t.w << 32 | t.z;
#pragma unroll
                for (int r = 0; r < R; ++r) D[r] |= (x[r][o] & rg) ? 1u << t.x : 0u;
            }
#pragma unroll
        for (int o = 0; o < KO; ++o)
            for (uint32_t q = wbeg[o]; q < wbeg[o + 1]; ++q) {
                const uint4 t = wfe[q];
                const uint64_t rg = (uint64_t)t.w << 32 | t.z;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const bool differ = t.y ? ((D[r] >> t.x) & 1u) != 0 : (x[r][o] & rg) != 0;
                    keep[r][o] &= differ ? ~rg : ~0ull;
                }
            }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const size_t e = e0 + r * T;
            if (e < m)
#pragma unroll
                for (int o = 0; o < KO; ++o) {
                    out[e * RW + o] = keep[r][o];
                    if (TERN) out[e * RW + KO + o] = val[r][TERN ? o : 0] & keep[r][o];
                }
        }
    }
}

void launch_pair_rows_factored(const uint64_t *FR, uint32_t n, const uint32_t *ids, size_t m, const FactorView &fv,
                               uint64_t *out, hipStream_t s) {
    if (!m) return;
    IG_REQUIRE(fv.KF >= 1 && fv.KF <= 16 && fv.wfe && fv.wbeg && n > 0, IG_E_DEVICE,
               "factored pair rows without a token-range table");
    const size_t cap = (size_t)device_cus() * 8;
#define IG_PR(V, RR)                                                                                               \
    case V: {                                                                                                      \
        const dim3 grid((unsigned)std::min<size_t>((m + 256 * RR - 1) / (256 * RR), cap));                       \
        if (fv.ternary)                                                                                            \
            hipLaunchKernelGGL((k_pair_rows_factored<V, RR, true>), grid, dim3(256), 0, s, FR, n, ids, m, fv.wfe,  \
                               fv.wbeg, out);                                                                      \
        else                                                                                                       \
            hipLaunchKernelGGL((k_pair_rows_factored<V, RR, false>), grid, dim3(256), 0, s, FR, n, ids, m, fv.wfe, \
                               fv.wbeg, out);                                                                      \
        break;                                                                                                     \
    }
    switch (fv.KF) {
        IG_PR(1, 4) IG_PR(2, 4) IG_PR(3, 4) IG_PR(4, 4) IG_PR(5, 4) IG_PR(6, 2) IG_PR(7, 2) IG_PR(8, 2)
        IG_PR(9, 1) IG_PR(10, 1) IG_PR(11, 1) IG_PR(12, 1) IG_PR(13, 1) IG_PR(14, 1) IG_PR(15, 1) IG_PR(16, 1)
        default: throw Error(IG_E_UNSUPPORTED, "factored pair rows of more than 16 words");
    }
#undef IG_PR
    IG_HIP(hipGetLastError());
}

void launch_operand_rows(const uint64_t *X, uint32_t n, const uint32_t *ids, const uint64_t *W, uint32_t KS, size_t m,
                         const FactorView &fv, bool complement, uint64_t *out, hipStream_t s) {
    if (!m) return;
    const uint32_t KO = fv.KF ? fv.KF : KS;
    // the register kernel walks the pieces of every one of the KS words
    IG_REQUIRE(!fv.KF || fv.nwords == KS, IG_E_DEVICE, "factoring table built for another storage width");
    IG_REQUIRE(!fv.ternary || !complement, IG_E_DEVICE, "ternary rows are never complemented");
    const dim3 grid((unsigned)((m + 255) / 256));
    const uint64_t flip = complement ? ~0ull : 0ull;
    const bool reg_width = KS <= 16 || KS == 20 || KS == 24 || KS == 28 || KS == 32 || KS == 40;
    if (fv.KF && reg_width && KO <= 16 && fv.nmask <= lds_masks((int)KS)) {
        // strided over the rows: a few workgroups per CU, each staging the masks once
        const dim3 sgrid((unsigned)std::min<size_t>((m + 255) / 256, (size_t)device_cus() * 8));
#define IG_OR_K(V)                                                                                             \
    case V:                                                                                                    \
        if (fv.ternary) {                                                                                      \
            if (fv.npiece <= kLdsPieces)                                                                       \
                hipLaunchKernelGGL((k_operand_rows_reg<V, true, true>), sgrid, dim3(256), 0, s, X, n, ids, W, m, \
                                   fv, KO, flip, out);                                                         \
            else                                                                                               \
                hipLaunchKernelGGL((k_operand_rows_reg<V, false, true>), sgrid, dim3(256), 0, s, X, n, ids, W, m, \
                                   fv, KO, flip, out);                                                         \
        } else if (fv.npiece <= kLdsPieces)                                                                    \
            hipLaunchKernelGGL((k_operand_rows_reg<V, true, false>), sgrid, dim3(256), 0, s, X, n, ids, W, m, fv, \
                               KO, flip, out);                                                                 \
        else                                                                                                   \
            hipLaunchKernelGGL((k_operand_rows_reg<V, false, false>), sgrid, dim3(256), 0, s, X, n, ids, W, m, fv, \
                               KO, flip, out);                                                                 \
        break;
        switch (KS) {   // the compiled storage widths up to 40 words
            IG_OR_K(1) IG_OR_K(2) IG_OR_K(3) IG_OR_K(4) IG_OR_K(5) IG_OR_K(6) IG_OR_K(7) IG_OR_K(8)
            IG_OR_K(10) IG_OR_K(12) IG_OR_K(14) IG_OR_K(16) IG_OR_K(20) IG_OR_K(24) IG_OR_K(28) IG_OR_K(32)
            IG_OR_K(40)
            default: throw Error(IG_E_UNSUPPORTED, "storage width without a factoring kernel");
        }
#undef IG_OR_K
    } else if (!fv.KF) {
        const dim3 ogrid((unsigned)std::min<size_t>((m * KS + 255) / 256, (size_t)device_cus() * 16));
        hipLaunchKernelGGL(k_operand_rows_onehot, ogrid, dim3(256), 0, s, X, n, ids, W, KS, m, flip, out);
    } else {
        hipLaunchKernelGGL(k_operand_rows, grid, dim3(256), 0, s, X, n, ids, W, KS, m, fv, KO, flip, out);
    }
    IG_HIP(hipGetLastError());
}

}  // namespace ig
