// The subset-test kernels of libig (gfx950, wave64).
//
// Every kernel evaluates Eq. 6 of the paper: b is inside r exactly when
// (b AND NOT r) is zero on every word.  The rows that all lanes of a wave test
// against are wave-uniform and come in through scalar loads into SGPRs; each lane
// holds its own bitsets in VGPRs, pre-complemented where that saves an op, so a
// 64-bit word costs two v_and_or_b32 (one per 32-bit half) and a test ends with
// one v_cmp whose lane mask is examined by the scalar unit.
//
//   k_coherence  Eq. 3: lanes = candidates (x_i AND x_j rebuilt from the pair
//                id), uniform = complemented rows of the other class, scanned in
//                input order; a wave stops when all its candidates are covered.
//   k_support    Eq. 2: lanes = ordered patterns, uniform = complemented rows of
//                the same class; counts the rows containing each pattern.
//   k_score      Eq. 4: lanes = flows (packed from their codes in registers and
//                complemented), uniform = patterns with their weights.
#include <atomic>

#include "common.h"
#include "kernels.h"

namespace ig {

typedef const __attribute__((address_space(4))) uint32_t *cptr32;   // scalar-loadable view
typedef const __attribute__((address_space(4))) int64_t *cptr64;
typedef const __attribute__((address_space(1))) uint32_t *gptr32;    // global (not flat) loads

__device__ __forceinline__ gptr32 global_rows(const uint64_t *p) { return (gptr32)(const void *)p; }
__device__ __forceinline__ uint32_t from_lane0(uint32_t v) { return __builtin_amdgcn_readlane(v, 0); }

// OR over words of (r AND b) with r uniform in SGPRs and b per lane, as one
// v_and_or_b32 per 32-bit word.  Written as inline-asm blocks of 8/4/2 words:
// left to itself the compiler rebalances the chain into a tree with ~40% more
// instructions, and one asm statement per word costs an s_nop each.
#define IG_AO_S(i) "s"(s[i])
#define IG_AO_V(i) "v"(v[i])
__device__ __forceinline__ uint32_t ao8(uint32_t acc, const uint32_t *s, const uint32_t *v, bool first) {
    if (first)
        asm("v_and_b32 %0, %1, %9\n\tv_and_or_b32 %0, %2, %10, %0\n\tv_and_or_b32 %0, %3, %11, %0\n\t"
            "v_and_or_b32 %0, %4, %12, %0\n\tv_and_or_b32 %0, %5, %13, %0\n\tv_and_or_b32 %0, %6, %14, %0\n\t"
            "v_and_or_b32 %0, %7, %15, %0\n\tv_and_or_b32 %0, %8, %16, %0"
            : "=&v"(acc)
            : IG_AO_S(0), IG_AO_S(1), IG_AO_S(2), IG_AO_S(3), IG_AO_S(4), IG_AO_S(5), IG_AO_S(6), IG_AO_S(7),
              IG_AO_V(0), IG_AO_V(1), IG_AO_V(2), IG_AO_V(3), IG_AO_V(4), IG_AO_V(5), IG_AO_V(6), IG_AO_V(7));
    else
        asm("v_and_or_b32 %0, %1, %9, %0\n\tv_and_or_b32 %0, %2, %10, %0\n\tv_and_or_b32 %0, %3, %11, %0\n\t"
            "v_and_or_b32 %0, %4, %12, %0\n\tv_and_or_b32 %0, %5, %13, %0\n\tv_and_or_b32 %0, %6, %14, %0\n\t"
            "v_and_or_b32 %0, %7, %15, %0\n\tv_and_or_b32 %0, %8, %16, %0"
            : "+v"(acc)
            : IG_AO_S(0), IG_AO_S(1), IG_AO_S(2), IG_AO_S(3), IG_AO_S(4), IG_AO_S(5), IG_AO_S(6), IG_AO_S(7),
              IG_AO_V(0), IG_AO_V(1), IG_AO_V(2), IG_AO_V(3), IG_AO_V(4), IG_AO_V(5), IG_AO_V(6), IG_AO_V(7));
    return acc;
}
__device__ __forceinline__ uint32_t ao4(uint32_t acc, const uint32_t *s, const uint32_t *v, bool first) {
    if (first)
        asm("v_and_b32 %0, %1, %5\n\tv_and_or_b32 %0, %2, %6, %0\n\tv_and_or_b32 %0, %3, %7, %0\n\t"
            "v_and_or_b32 %0, %4, %8, %0"
            : "=&v"(acc)
            : IG_AO_S(0), IG_AO_S(1), IG_AO_S(2), IG_AO_S(3), IG_AO_V(0), IG_AO_V(1), IG_AO_V(2), IG_AO_V(3));
    else
        asm("v_and_or_b32 %0, %1, %5, %0\n\tv_and_or_b32 %0, %2, %6, %0\n\tv_and_or_b32 %0, %3, %7, %0\n\t"
            "v_and_or_b32 %0, %4, %8, %0"
            : "+v"(acc)
            : IG_AO_S(0), IG_AO_S(1), IG_AO_S(2), IG_AO_S(3), IG_AO_V(0), IG_AO_V(1), IG_AO_V(2), IG_AO_V(3));
    return acc;
}
__device__ __forceinline__ uint32_t ao2(uint32_t acc, const uint32_t *s, const uint32_t *v, bool first) {
    if (first)
        asm("v_and_b32 %0, %1, %3\n\tv_and_or_b32 %0, %2, %4, %0" : "=&v"(acc)
            : IG_AO_S(0), IG_AO_S(1), IG_AO_V(0), IG_AO_V(1));
    else
        asm("v_and_or_b32 %0, %1, %3, %0\n\tv_and_or_b32 %0, %2, %4, %0" : "+v"(acc)
            : IG_AO_S(0), IG_AO_S(1), IG_AO_V(0), IG_AO_V(1));
    return acc;
}
#undef IG_AO_S
#undef IG_AO_V

template <int W>   // W (even) 32-bit words: OR_k (r_k AND b_k), r uniform
__device__ __forceinline__ uint32_t masked_or(cptr32 r, const uint32_t (&b)[W]) {
    uint32_t s[W];
#pragma unroll
    for (int k = 0; k < W; ++k) s[k] = r[k];
    uint32_t acc = 0;
    int k = 0;
#pragma unroll
    for (; k + 8 <= W; k += 8) acc = ao8(acc, s + k, b + k, k == 0);
    if (k + 4 <= W) { acc = ao4(acc, s + k, b + k, k == 0); k += 4; }
    if (k + 2 <= W) { acc = ao2(acc, s + k, b + k, k == 0); k += 2; }
    return acc;
}

__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ void load_pair_row(const uint64_t *__restrict__ X, uint32_t KS, uint64_t q, uint32_t n,
                                              bool active, uint32_t *out, int W) {
    uint32_t i = 0, j = 0;
    if (active) decode_pair(q, n, i, j);
    const uint32_t *a = reinterpret_cast<const uint32_t *>(X + (size_t)i * KS);
    const uint32_t *b = reinterpret_cast<const uint32_t *>(X + (size_t)j * KS);
    for (int k = 0; k < W; ++k) out[k] = active ? (a[k] & b[k]) : 0u;
}

// ------------------------------------------------------------ coherence ----
// One phase of the coherence filter: the candidates of each segment's input list
// are tested against other-class records [r_begin, r_end) in input order.  A
// candidate covered at record r is dropped and adds t(b) = r + 1 to the segment's
// test count; an uncovered one is appended to the output list -- the next
// phase's input, or the coherent set when the phase reaches the last record.
// Phases keep lanes busy: a wave stops when its candidates are covered or the
// phase ends, so a covered candidate idles at most until the end of its phase.
template <int KS, int CPL>
__global__ __launch_bounds__(256) void k_coherence(const CohSeg *__restrict__ segs, uint32_t nseg, uint32_t r_begin,
                                                  uint32_t r_end, uint32_t *__restrict__ queue) {
    constexpr int W = 2 * KS;
    constexpr uint32_t PER_TASK = 64u * CPL;
    const int lane = threadIdx.x & 63;
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    // tasks of every segment, from the input counts left on the device by the previous step
    uint32_t ntasks = 0;
    for (uint32_t sg = 0; sg < nseg; ++sg) ntasks += (uniform(*segs[sg].ncand) + PER_TASK - 1) / PER_TASK;
    ntasks = uniform(ntasks);
    unsigned long long *tests_at = nullptr;   // sum of t(b) kept per wave, flushed per segment
    uint64_t tests_acc = 0;
    for (;;) {
        uint32_t t = 0;
        if (lane == 0) t = atomicAdd(queue, 1u);
        t = from_lane0(t);
        if (t >= ntasks) break;
        uint32_t sg = 0, first = 0, ncand = 0;
        for (;; ++sg) {
            ncand = uniform(*segs[sg].ncand);
            const uint32_t nt = (ncand + PER_TASK - 1) / PER_TASK;
            if (t < first + nt) break;
            first += nt;
        }
        sg = uniform(sg);
        const CohSeg g = segs[sg];
        const uint32_t *cand = g.cand + (g.cand_off ? uniform(*g.cand_off) : 0u);
        const uint32_t base = (t - first) * PER_TASK;
        const uint32_t n_o = g.n_o;
        const uint32_t rb = r_begin < n_o ? r_begin : n_o;
        const uint32_t re = r_end < n_o ? r_end : n_o;
        const bool last = r_end >= n_o;

        uint32_t b[CPL][W];
        uint32_t pid[CPL];
        uint64_t cov[CPL];
        uint32_t tpos[CPL];
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            const uint32_t idx = base + c * 64 + lane;
            const bool act = idx < ncand;
            pid[c] = act ? ((const __attribute__((address_space(1))) uint32_t *)(const void *)cand)[idx] : 0u;
            uint32_t i = 0, j = 0;
            if (act) decode_pair(pid[c], g.n, i, j);
            gptr32 ra = global_rows(g.X + (size_t)i * KS);
            gptr32 rb2 = global_rows(g.X + (size_t)j * KS);
#pragma unroll
            for (int k = 0; k < W; ++k) b[c][k] = ra[k] & rb2[k];
            cov[c] = ~__ballot(act);   // lanes without a candidate count as done
            tpos[c] = 0;
        }
        cptr32 R = (cptr32)(const void *)g.NXo;
        for (uint32_t r = rb; r < re; ++r) {
            cptr32 rr = R + (size_t)r * W;
            uint64_t done = ~0ull;
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const uint32_t acc = masked_or<W>(rr, b[c]);
                const uint64_t nw = __ballot(acc == 0u) & ~cov[c];
                if (nw) {
                    if ((nw >> lane) & 1ull) tpos[c] = r + 1;
                    cov[c] |= nw;
                }
                done &= cov[c];
            }
            if (done == ~0ull) break;
        }
        uint64_t tsum = 0;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            const uint32_t idx = base + c * 64 + lane;
            const bool act = idx < ncand;
            const bool keep = act && !((cov[c] >> lane) & 1ull);
            const uint64_t km = __ballot(keep);
            if (km) {
                uint32_t at = 0;
                if (lane == 0) at = atomicAdd(g.nout, (uint32_t)__popcll(km));
                at = from_lane0(at);
                if (keep) g.out[at + (uint32_t)__popcll(km & lt)] = pid[c];
            }
            if (act && tpos[c]) tsum += tpos[c];
            if (keep && last) tsum += n_o;
        }
        for (int o = 32; o > 0; o >>= 1) tsum += __shfl_xor(tsum, o, 64);
        if (g.tests != tests_at) {
            if (lane == 0 && tests_acc) atomicAdd(tests_at, (unsigned long long)tests_acc);
            tests_at = g.tests;
            tests_acc = 0;
        }
        tests_acc += tsum;
    }
    if (lane == 0 && tests_acc) atomicAdd(tests_at, (unsigned long long)tests_acc);
}

// ------------------------------------------------ coherence as a contraction ----
// The coherence test as a dense matrix product on the matrix cores: V[r][b] =
// sum over tokens of r'[token] * b[token], with b the candidate's 0/1 tokens and
// r' the record's side, is 0 exactly when record r contains candidate b (Eq. 6)
// and positive otherwise.  On one-hot tokens r' = NOT r and V counts b's tokens
// missing from r; on factored tokens r' is the signed side (FactorView::tok) and
// V counts the bits in which the bin indices differ.  Every operand is exact in
// fp4 (e2m1: 1.0 = 0x2, -1.0 = 0xA) and every V is a small integer, exact in the
// fp32 accumulators.  One v_mfma_scale_f32_32x32x64_f8f6f4 covers 64 tokens (one
// 64-bit word): lanes l and l+32 of a row / column supply its two 32-bit halves.
// Records are the A operand (rows), candidates the B operand (columns).
typedef int v4i_t __attribute__((ext_vector_type(4)));
typedef int v8i_t __attribute__((ext_vector_type(8)));
typedef int v16i_t __attribute__((ext_vector_type(16)));
typedef float v16f_t __attribute__((ext_vector_type(16)));

// 8 bits -> 8 nibbles, bit i -> nibble i = (bit ? 1.0 : 0) in e2m1
__device__ __forceinline__ uint32_t spread8(uint32_t b) {
    uint32_t x = b & 0xffu;
    x = (x | (x << 12)) & 0x000f000fu;
    x = (x | (x << 6)) & 0x03030303u;
    x = (x | (x << 3)) & 0x11111111u;
    return x << 1;
}

// Streaming A-operand tiles through LDS.  The tiles [t0, t1) of a fragment array
// (TW uint4 per 32-row tile) pass through a ring of NB LDS buffers of G tiles
// each.  Loads go from memory straight to LDS (global_load_lds_dwordx4: lane l of
// a wave writes bytes [16 l, 16 l + 16) of the wave's 1 KB slice) and are issued
// NB - 1 groups ahead, so that several groups of multiplications cover their
// latency; one barrier per group.  Every wave issues the same number of loads per
// group (slices past the group go to a 1 KB scratch slot), which lets vmcnt tell
// exactly when a group has landed.  Loads past t1 are clamped to the last element
// of the range (the copies are never read).
typedef uint32_t v4u_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void load_to_lds16(const v4u_t *src, v4u_t *wave_slice) {
    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)src,
                                     (__attribute__((address_space(3))) void *)wave_slice, 16, 0, 0);
}

template <int N>
__device__ __forceinline__ void wait_loads() {
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// LDS (uint4) of a ring: NB buffers of G tiles of TW uint4 (each buffer rounded up
// to whole 64-uint4 wave slices), plus the scratch slot
template <int TW, int G, int NB>
constexpr int ring_stride() { return (G * TW + 63) / 64 * 64; }
template <int TW, int G, int NB>
constexpr int ring_lds() { return NB * ring_stride<TW, G, NB>() + 64; }

template <int TW, int G, int NB, int NT, class Pre, class Body>
__device__ __forceinline__ void stream_tiles_after(const uint4 *__restrict__ frag_in, uint32_t t0, uint32_t t1,
                                                   uint4 *lds_in, Pre pre, Body body) {
    constexpr int N = G * TW;                          // uint4 per group
    constexpr int NS = ring_stride<TW, G, NB>();       // LDS uint4 per buffer (a whole number of slices)
    constexpr int PER = (N + NT - 1) / NT;             // loads per thread per group
    static_assert(NB >= 2 && NB <= 4 && (NB - 2) * PER <= 63, "ring depth");
    const v4u_t *frag = reinterpret_cast<const v4u_t *>(frag_in);
    v4u_t *lds = reinterpret_cast<v4u_t *>(lds_in);
    v4u_t *dummy = lds + NB * NS;
    const uint32_t lane = threadIdx.x & 63, wave_base = threadIdx.x & ~63u;
    const uint32_t ng = (t1 - t0 + G - 1) / G;
    auto issue = [&](uint32_t gi) __attribute__((always_inline)) {
        const uint32_t t = t0 + gi * G;
        const uint32_t avail = (t1 - t) * TW;
        const uint32_t last = (avail < (uint32_t)N ? avail : (uint32_t)N) - 1;
        const v4u_t *src = frag + (size_t)t * TW;
        v4u_t *buf = lds + (gi % NB) * NS;   // a slice that starts below N ends inside the buffer
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const uint32_t q0 = wave_base + i * NT;   // first slot of this wave's slice
            const uint32_t q = q0 + lane;
            load_to_lds16(src + (q < last ? q : last), q0 < (uint32_t)N ? buf + q0 : dummy);
        }
    };
#pragma unroll
    for (int p = 0; p < NB - 1; ++p)
        if ((uint32_t)p < ng) issue(p);
    // work that overlaps the first groups' loads (its own loads are counted by vmcnt
    // after the ring's, so the waits below only wait longer)
    pre();
    for (uint32_t g = 0; g < ng; ++g) {
        // groups issued after g: min(NB - 2, ng - 1 - g); wait until only those are in flight
        const uint32_t ahead = ng - 1 - g < (uint32_t)(NB - 2) ? ng - 1 - g : (uint32_t)(NB - 2);
        if (NB >= 4 && ahead >= 2) wait_loads<(NB >= 4 ? 2 : 0) * PER>();
        else if (NB >= 3 && ahead >= 1) wait_loads<PER>();
        else wait_loads<0>();
        // all of group g is in LDS, and every wave is done with group g - 1's buffer
        __syncthreads();
        if (g + NB - 1 < ng) issue(g + NB - 1);
        const uint32_t t = t0 + g * G;
        const uint32_t nt = t1 - t < (uint32_t)G ? t1 - t : (uint32_t)G;
        const uint4 *cur = lds_in + (g % NB) * NS;
        for (uint32_t j = 0; j < nt; ++j) body(cur + j * TW);
    }
}

template <int TW, int G, int NB, int NT, class Body>
__device__ __forceinline__ void stream_tiles(const uint4 *__restrict__ frag_in, uint32_t t0, uint32_t t1,
                                             uint4 *lds_in, Body body) {
    stream_tiles_after<TW, G, NB, NT>(frag_in, t0, t1, lds_in, [] {}, body);
}

// Other-class records, complemented (one-hot tokens), in the A-operand layout of
// each 32-record tile: frag[(tile * KS + word) * 64 + lane] = the 32 nibbles of
// half (lane/32) of word `word` of record tile*32 + lane%32.  Rows past n are all
// ones (the empty record), which never contain a candidate.
__global__ void k_mfma_records(const uint64_t *__restrict__ NX, uint32_t n, uint32_t KS, uint32_t ntiles,
                               uint4 *__restrict__ frag) {
    const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (size_t)ntiles * KS * 64) return;
    const uint32_t lane = (uint32_t)(g % 64), word = (uint32_t)((g / 64) % KS), tile = (uint32_t)(g / (64 * KS));
    const uint32_t r = tile * 32 + lane % 32;
    const uint32_t d = r < n ? (uint32_t)(NX[(size_t)r * KS + word] >> (32 * (lane / 32))) : 0xffffffffu;
    frag[g] = make_uint4(spread8(d), spread8(d >> 8), spread8(d >> 16), spread8(d >> 24));
}

// The signed side of the factored tokens (FactorView::tok): the e2m1 nibble of
// token `desc` for a row whose bin index of the token's feature has the given bit
// (bit tokens) and popcount pc (presence tokens: two parts e2m1 holds exactly).
__device__ __forceinline__ uint32_t signed_nibble(uint32_t desc, uint32_t bit, uint32_t pc) {
    const uint32_t kind = desc & 3u;
    if (kind == 1u) return bit ? 0xAu : 0x2u;   // -1.0 / +1.0
    if (kind == 0u) return 0u;
    const uint32_t first = pc >= 6u ? 6u : min(pc, 4u);
    const uint32_t v = kind == 2u ? first : pc - first;
    return (0x7065420u >> (4u * v)) & 0xFu;   // e2m1 of 0, 1, 2, 3, 4, -, 6
}

// Records in the A-operand layout of k_mfma_records, on the signed side of the
// factored tokens, from their factored rows FR [n][KO] (every feature present).
// Rows past n are +1.0 on every token: a candidate sets a presence token for each
// feature it holds, so it never lies inside them.
__global__ void k_mfma_records_signed(const uint64_t *__restrict__ FR, uint32_t n, uint32_t KO, uint32_t ntiles,
                                      FactorView fv, uint4 *__restrict__ frag) {
    const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (size_t)ntiles * KO * 64) return;
    const uint32_t lane = (uint32_t)(g % 64), word = (uint32_t)((g / 64) % KO), tile = (uint32_t)(g / (64 * KO));
    const uint32_t r = tile * 32 + lane % 32, h = lane / 32;
    if (r >= n) {
        frag[g] = make_uint4(0x22222222u, 0x22222222u, 0x22222222u, 0x22222222u);
        return;
    }
    const uint64_t *R = FR + (size_t)r * KO;
    const uint32_t mine = (uint32_t)(R[word] >> (32 * h));
    uint64_t lo = 0, hi = 0;
    for (uint32_t j = 0; j < 32; ++j) {
        const uint32_t desc = fv.tok[word * 64 + 32 * h + j];
        uint32_t pc = 0;
        if ((desc & 3u) >= 2u) {
            const uint32_t f = desc >> 16;
            const FacFeature ft = fv.feat[f];
            pc = (uint32_t)__popcll(R[ft.w0] & fv.fbit[2 * f]);
            if (ft.nw > 1) pc += (uint32_t)__popcll(R[ft.w0 + 1] & fv.fbit[2 * f + 1]);
        }
        const uint32_t nib = signed_nibble(desc, (mine >> j) & 1u, pc);
        if (j < 16) lo |= (uint64_t)nib << (4 * j);
        else hi |= (uint64_t)nib << (4 * (j - 16));
    }
    frag[g] = make_uint4((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32));
}

// Ternary rows (P then V, KO words each) as A-operand tiles: lane l of slice w
// holds half l / 32 of word w of row tile * 32 + l % 32 as nibbles, P AND NOT V
// +1.0 (0x2), P AND V -1.0 (0xA), else 0.  The top nslots tokens of the last word
// (no bit token lies there) are the bias slots: +1.0 on the top one, +6.0 below it,
// against which each candidate row carries the nibbles that add 1 - |P|.  Rows past
// n are 0 everywhere, so every product with them is 0, never the 1 of a record that
// contains the candidate.
// Slice (word, half h) of a record tile row: record r of FR, or none (all zero).
__device__ __forceinline__ uint4 ternary_record_slice(const uint64_t *__restrict__ FR, uint32_t KO, uint32_t nslots,
                                                      bool has, uint32_t r, uint32_t word, uint32_t h) {
    uint32_t P = 0, V = 0;
    if (has) {
        P = (uint32_t)(FR[(size_t)r * 2 * KO + word] >> (32 * h));
        V = (uint32_t)(FR[(size_t)r * 2 * KO + KO + word] >> (32 * h));
    }
    uint32_t q[4] = {spread8(P) | spread8(V) * 4u, spread8(P >> 8) | spread8(V >> 8) * 4u,
                     spread8(P >> 16) | spread8(V >> 16) * 4u, spread8(P >> 24) | spread8(V >> 24) * 4u};
    if (has && word == KO - 1 && h == 1) {
        // the bias slots, from the top token down: +1.0, then +6.0
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const uint32_t slot = 31u - (uint32_t)(8 * j + i);
                if (slot < nslots) q[j] |= (slot ? 0x7u : 0x2u) << (4 * i);
            }
    }
    return make_uint4(q[0], q[1], q[2], q[3]);
}

__global__ void k_mfma_records_ternary(const uint64_t *__restrict__ FR, uint32_t n, uint32_t KO, uint32_t ntiles,
                                       uint32_t nslots, uint4 *__restrict__ frag) {
    const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (size_t)ntiles * KO * 64) return;
    const uint32_t lane = (uint32_t)(g % 64), word = (uint32_t)((g / 64) % KO), tile = (uint32_t)(g / (64 * KO));
    const uint32_t r = tile * 32 + lane % 32;
    frag[g] = ternary_record_slice(FR, KO, nslots, r < n, r, word, lane / 32);
}

// The same tiles of the records listed per bucket: bucket u < nb holds the brec[u]
// records list[ro[u] ..] in tiles [bt[u], bt[u + 1]), its last tile padded with
// empty rows.
__global__ void k_mfma_records_ternary_lists(const uint64_t *__restrict__ FR, uint32_t KO, uint32_t ntiles,
                                             uint32_t nslots, const uint32_t *__restrict__ list,
                                             const uint32_t *__restrict__ ro, const uint32_t *__restrict__ bt,
                                             const uint32_t *__restrict__ brec, uint32_t nb,
                                             uint4 *__restrict__ frag) {
    const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (size_t)ntiles * KO * 64) return;
    const uint32_t lane = (uint32_t)(g % 64), word = (uint32_t)((g / 64) % KO), tile = (uint32_t)(g / (64 * KO));
    uint32_t lo = 0, hi = nb;   // the bucket of the tile: bt[u] <= tile < bt[u + 1]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) / 2;
        if (bt[mid] <= tile) lo = mid;
        else hi = mid;
    }
    const uint32_t slot = (tile - bt[lo]) * 32 + lane % 32;
    const bool has = slot < brec[lo];
    frag[g] = ternary_record_slice(FR, KO, nslots, has, has ? list[ro[lo] + slot] : 0u, word, lane / 32);
}

// One workgroup: 8 waves x 2 column sets x 32 candidates = 512 candidates; each
// wave keeps its candidates' B operands in registers for the whole scan.
constexpr int MF_NT = 512;                  // threads per matrix-core workgroup
constexpr int MF_FB = 2;                    // 32-column sets per wave (scoring)
// 32-column sets per wave of the subset-test contraction: three up to 5 operand
// words, two up to 8, one beyond (the B operands of a set take 4 VGPRs per word;
// more sets share each A tile read from LDS among more multiplications)
#ifndef IG_MF_SETS_NARROW
#define IG_MF_SETS_NARROW 3
#endif
template <int KS>
constexpr int mf_sets() { return KS <= 5 ? IG_MF_SETS_NARROW : KS <= 8 ? 2 : 1; }
// the most sets whose B operands and accumulators fit 128 VGPRs (4 waves per SIMD)
__host__ __device__ constexpr int mf_max_sets(int KS) { return KS <= 5 ? 3 : KS <= 8 ? 2 : 1; }
template <int FB>
constexpr int mf_cols() { return MF_NT / 64 * FB * 32; }
// two workgroups per CU (4 waves per SIMD: at most 128 VGPRs each, 2 x 64 KB of LDS),
// so that one workgroup's waves multiply while the other's wait at a barrier
constexpr int MF_WAVES_PER_SIMD = 4;
#ifndef IG_MF_GTOK
#define IG_MF_GTOK 32
#endif
#ifndef IG_MF_NB
#define IG_MF_NB 2
#endif
constexpr int MF_NB = IG_MF_NB;   // LDS ring depth
template <int KS>
constexpr int mf_group() { return IG_MF_GTOK / KS > 0 ? IG_MF_GTOK / KS : 1; }   // tiles per LDS buffer
// The pruned contraction's workgroups: a work unit streams only its bucket's few
// tiles, so a smaller ring and workgroup let more units overlap their set-up (4
// waves and 4 tiles per buffer at 3 words: four workgroups per CU; measured at 15k
// against 8 waves and 10 tiles: coherence 0.92 against 1.00 ms, support 0.68
// against 0.72 ms)
#ifndef IG_MFP_NT
#define IG_MFP_NT 256
#endif
#ifndef IG_MFP_GTOK
#define IG_MFP_GTOK 12
#endif
#ifndef IG_MFP_NB
#define IG_MFP_NB IG_MF_NB
#endif
constexpr int MP_NT = IG_MFP_NT;
constexpr int MP_NB = IG_MFP_NB;
template <int KS>
constexpr int mp_group() { return IG_MFP_GTOK / KS > 0 ? IG_MFP_GTOK / KS : 1; }
template <int FB>
constexpr int mp_cols() { return MP_NT / 64 * FB * 32; }

// Bits [lo, hi) of a 128-bit string, as its 32-bit word j.
__device__ __forceinline__ uint32_t bit_range_word(int lo, int hi, int j) {
    const int a = max(lo - 32 * j, 0), b = min(hi - 32 * j, 32);
    return b <= a ? 0u : (b - a == 32 ? ~0u : ((1u << (b - a)) - 1u)) << a;
}

// Word j (tokens 8 j .. 8 j + 7) of the candidate's nibbles in the bias slots of a
// ternary view (the upper half of its last word; slot s is token 31 - s of that
// half, see tern_bias_slots): they add 1 - np to its product with every record
// tile row, whose slots hold +1.0 (slot 0) and +6.0 (the others).  np = 0: +1.0 on
// slot 0.  Else, with v = np - 1 = 36 q + 3 k + i: -i on slot 0, -6.0 (36) on slots
// 1 .. q, and 3 k as two slots of -k1 / 2 and -k2 / 2 (times 6), k1 the largest of
// 0, 1, 2, 3, 4, 6, 8 not above k and k2 = k - k1 <= 3.
__device__ __forceinline__ uint32_t tern_bias_word(uint32_t np, int j) {
    if (np == 0) return j == 3 ? 0x2u << 28 : 0u;
    const uint32_t v = np - 1, q = v / 36, r = v % 36, i = r % 3, k = r / 3;
    const uint32_t k1 = k >= 8 ? 8u : k >= 6 ? 6u : k >= 4 ? 4u : k, k2 = k - k1;
    // e2m1 codes of k / 2 for k = 0 .. 8 (0, 0.5, 1, 1.5, 2, -, 3, -, 4), negated
    const uint32_t c1 = k1 ? (k1 <= 4 ? k1 : k1 == 6 ? 5u : 6u) | 8u : 0u, c2 = k2 ? k2 | 8u : 0u;
    const uint32_t c0 = i == 0 ? 0u : i == 1 ? 0xAu : 0xCu;
    const int top = 4 * 31;   // bit of slot 0
    uint32_t w = bit_range_word(top - 4 * (int)q, top, j);   // slots 1 .. q: 0xF (-6.0)
    const int p0 = top, p1 = top - 4 * ((int)q + 1), p2 = top - 4 * ((int)q + 2);
    if ((p0 >> 5) == j) w |= c0 << (p0 & 31);
    if ((p1 >> 5) == j) w |= c1 << (p1 & 31);
    if ((p2 >> 5) == j) w |= c2 << (p2 & 31);
    return w;
}

// B operand of one 32-column set: operand row `r` of B (inactive columns: none).
template <int KS, bool TERN>
__device__ __forceinline__ void contain_operand(const uint64_t *__restrict__ B, uint32_t r, bool act, int half,
                                                v8i_t (&b)[KS]) {
    constexpr int RW = TERN ? 2 * KS : KS;   // words per operand row
    const uint32_t *row = reinterpret_cast<const uint32_t *>(B + (size_t)(act ? r : 0u) * RW);
    uint32_t tokens = 0;
#pragma unroll
    for (int w = 0; w < KS; ++w) {
        if (TERN) {
            // inactive columns: no tokens, so their result is ignored anyway
            const uint32_t P = act ? row[2 * w + half] : 0u, V = act ? row[2 * (KS + w) + half] : 0u;
            tokens += __popc(P);
            b[w] = v8i_t{(int)(spread8(P) | spread8(V) * 4u), (int)(spread8(P >> 8) | spread8(V >> 8) * 4u),
                         (int)(spread8(P >> 16) | spread8(V >> 16) * 4u), (int)(spread8(P >> 24) | spread8(V >> 24) * 4u),
                         0, 0, 0, 0};
        } else {
            const uint32_t v = row[2 * w + half];   // unconditional: the loads overlap
            // inactive columns: all tokens, so their result is ignored anyway
            const uint32_t d = act ? v : 0xffffffffu;
            b[w] = v8i_t{(int)spread8(d), (int)spread8(d >> 8), (int)spread8(d >> 16), (int)spread8(d >> 24), 0, 0, 0, 0};
        }
    }
    if (TERN) {
        // both halves of the wave hold the same column: |P| over both; the bias
        // slots lie in the upper half of the last word
        const uint32_t np = tokens + (uint32_t)__shfl_xor((int)tokens, 32, 64);
#pragma unroll
        for (int j = 0; j < 4; ++j) b[KS - 1][j] |= half ? (int)tern_bias_word(np, j) : 0;
    }
}

// One record tile against the wave's column sets.  An accumulator ends at the
// number of candidate tokens the record lacks (ternary: at 1 - 2 (bits in which the
// bin indices differ), or 0 on padding).  best (see k_contain_mfma) takes the tile.
template <int KS, bool COUNT, int FB, bool TERN>
__device__ __forceinline__ void contain_tile(const uint4 *tf, int lane, const v8i_t (&b)[FB][KS], uint32_t (&best)[FB],
                                             uint32_t one) {
    v16f_t acc[FB];
#pragma unroll
    for (int f = 0; f < FB; ++f) acc[f] = v16f_t{0};
#pragma unroll
    for (int w = 0; w < KS; ++w) {
        const uint4 a4 = tf[w * 64 + lane];
        const v8i_t a = {(int)a4.x, (int)a4.y, (int)a4.z, (int)a4.w, 0, 0, 0, 0};
#pragma unroll
        for (int f = 0; f < FB; ++f)
            acc[f] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b[f][w], acc[f], 4, 4, 0, 127, 0, 127);
    }
#pragma unroll
    for (int f = 0; f < FB; ++f) {
        if (COUNT && TERN) {
            // the records that lack the candidate: the negative values (sign bit
            // set); 1.0 and the 0 of a padding row have it clear.  A byte permute
            // copies the signs of two accumulators into two bytes (selectors 9 and
            // 11 repeat bit 31 of its second and first source), and the population
            // count adds 8 per sign.
#pragma unroll
            for (int r = 0; r < 16; r += 2)
                best[f] += __builtin_popcount(__builtin_amdgcn_perm(__float_as_uint(acc[f][r]),
                                                                    __float_as_uint(acc[f][r + 1]), 0x0c0c0b09u));
        } else if (COUNT) {
            // +0.0 (all bits zero) exactly when the record contains the candidate;
            // min(bits, one) with `one` not a literal: the compiler would turn
            // min(bits, 1) into a compare again
            uint32_t lacking = 0;
#pragma unroll
            for (int r = 0; r < 16; ++r) lacking += min(__float_as_uint(acc[f][r]), one);
            best[f] += 16u - lacking;
        } else if (TERN) {
            // as integers the bits keep the order of 1.0 over 0 and the negatives
            int hi = (int)best[f];
#pragma unroll
            for (int r = 0; r < 16; ++r) hi = max(hi, (int)__float_as_uint(acc[f][r]));
            best[f] = (uint32_t)hi;
        } else {
            uint32_t lo = best[f];
#pragma unroll
            for (int r = 0; r < 16; ++r) lo = min(lo, __float_as_uint(acc[f][r]));
            best[f] = lo;
        }
    }
}

// Columns: operand rows B [m][KS], expanded bit -> nibble into the B operand in
// registers (lane % 32 = column, lane / 32 = 32-token half of each word); the A
// side streams the record tiles.  COUNT = false (coherence, Eq. 3): out[e] = 1
// when no record contains row e; COUNT = true (support, Eq. 2): out[e] = the
// number of records that contain it.  FB 32-column sets per wave.
// TERN: rows B [m][2 KS] are ternary (P then V; FactorView::ternary) and the tiles
// hold the records' ternary nibbles and bias slots: with the column's bias nibbles
// an accumulator ends at 1 - 2 (bits in which the bin indices differ), so at 1.0
// exactly when the record contains the candidate, at most -1.0 otherwise and 0 on
// the padding rows of the last tile.
// The accumulators hold exact small integers, and their bit patterns are compared
// as integers (no float compares, whose lane masks cost hazard waits).
template <int KS, bool COUNT, int FB, bool TERN>
__global__ __launch_bounds__(MF_NT, MF_WAVES_PER_SIMD) void k_contain_mfma(const uint64_t *__restrict__ B, uint32_t m,
                                                                         const uint4 *__restrict__ frag,
                                                                         uint32_t ntiles, uint32_t pad,
                                                                         uint32_t *__restrict__ out) {
    constexpr int G = mf_group<KS>();
    constexpr int RW = TERN ? 2 * KS : KS;             // words per operand row
    __shared__ uint4 lds[ring_lds<KS * 64, G, MF_NB>()];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, half = lane >> 5, col = lane & 31;
    v8i_t b[FB][KS];
    uint32_t e[FB];
    // coherence: the least accumulator (one-hot and factored: 0 when a record
    // contains the column) or the greatest (ternary: 1.0 when one does) so far;
    // support: the records that contain the column (ternary: 8 x those that lack it)
    uint32_t best[FB];
#pragma unroll
    for (int f = 0; f < FB; ++f) {
        e[f] = blockIdx.x * mf_cols<FB>() + wave * (FB * 32) + f * 32 + col;
        contain_operand<KS, TERN>(B, e[f], e[f] < m, half, b[f]);
        best[f] = COUNT || TERN ? 0u : ~0u;
    }
    const uint32_t one = m != 0u;   // 1 (the kernel runs only with columns)
    if (ntiles)
        stream_tiles<KS * 64, G, MF_NB, MF_NT>(frag, 0, ntiles, lds, [&](const uint4 *tf) __attribute__((always_inline)) {
            contain_tile<KS, COUNT, FB, TERN>(tf, lane, b, best, one);
        });
#pragma unroll
    for (int f = 0; f < FB; ++f) {
        // the two halves of the wave hold different record rows of the same column
        const uint32_t o = (uint32_t)__shfl_xor((int)best[f], 32, 64);
        uint32_t h;
        if (COUNT && TERN) {
            h = 32u * ntiles - pad - (best[f] + o) / 8u;   // real records less those that lack it
        } else if (COUNT) {
            h = best[f] + o;
            // One-hot and factored: a row with no tokens (a pattern of one-bin
            // features only) gives 0 against every A row, the padding rows of the
            // last tile too: they are not records, so they come off its count.
            // (Coherence needs no such care: a real record of the tile contains
            // that row as well.  Ternary padding rows give 0, not 1.0.)
            if (pad && half == 0 && e[f] < m) {
                uint64_t any = 0;
                for (int w = 0; w < KS; ++w) any |= B[(size_t)e[f] * RW + w];
                if (!any) h -= pad;
            }
        } else if (TERN) {
            h = max((int)best[f], (int)o) > 0 ? 1u : 0u;   // covered by a record
        } else {
            h = min(best[f], o) == 0u ? 1u : 0u;
        }
        if (half == 0 && e[f] < m) out[e[f]] = COUNT ? h : (h ? 0u : 1u);
    }
}

// The entry (bucket) that owns work unit `unit`: the last i < n2 with uoff[i] <= unit
// (uoff ascends from uoff[0] = 0, and that entry's range is not empty).  The 64
// lanes of one wave (all active, unit uniform) probe every stride-th entry, then
// the entries of the block found: two rounds of loads instead of a binary search.
__device__ __forceinline__ uint32_t unit_owner(const uint32_t *__restrict__ uoff, uint32_t n2, uint32_t unit) {
    const uint32_t lane = threadIdx.x & 63, stride = (n2 + 63) / 64;
    const uint32_t p = lane * stride;
    const uint32_t k = (uint32_t)__popcll(__ballot(p < n2 && uoff[p] <= unit)) - 1u;
    uint32_t cnt = 0;
    for (uint32_t c = 0; c < stride; c += 64) {
        const uint32_t q = k * stride + c + lane;
        cnt += (uint32_t)__popcll(__ballot(c + lane < stride && q < n2 && uoff[q] <= unit));
    }
    return k * stride + cnt - 1u;
}

// The same contraction pruned by token buckets (ternary rows only).  A record can
// contain a candidate only when it holds every token of it, in particular the
// candidate's bucket token u (one of its tokens, chosen by the caller); the
// records holding u form the tiles [bt[u], bt[u + 1]) (brec[u] real rows, see
// launch_bucket_tiles), and the candidates of bucket u are positions
// [cs[u], cs[u + 1]) of the order perm (position -> row of B and of out).
// Workgroup `unit` takes the candidates of bucket u with uoff[u] <= unit <
// uoff[u + 1], block unit - uoff[u] of mp_cols<FB>() of them, against the tiles of
// bucket u only: the results are those of k_contain_mfma against all records.  The
// ranges of every unit are precomputed (desc, launch_contain_plan), so a workgroup
// starts with one load; workgroups past the last unit (the grid is a bound set
// before the units are counted on the device) find an empty range and end.
template <int KS, bool COUNT, int FB>
__global__ __launch_bounds__(MP_NT, MF_WAVES_PER_SIMD) void k_contain_mfma_pruned(const uint64_t *__restrict__ B,
                                                                                const uint4 *__restrict__ frag,
                                                                                ContainBuckets k,
                                                                                uint32_t *__restrict__ out) {
    constexpr int G = mp_group<KS>();
    __shared__ uint4 lds[ring_lds<KS * 64, G, MP_NB>()];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, half = lane >> 5, col = lane & 31;
    const uint4 d = k.desc[2 * (size_t)blockIdx.x];
    const uint32_t c0 = d.x, c1 = d.y, t0 = d.z, t1 = d.w;
    if (c0 >= c1) return;   // past the last unit (the grid is a bound on the units)
    v8i_t b[FB][KS];
    uint32_t r[FB], best[FB];
    uint32_t pos[FB];
    bool act[FB];
#pragma unroll
    for (int f = 0; f < FB; ++f) {
        const uint32_t e = c0 + wave * (FB * 32) + f * 32 + col;
        act[f] = e < c1;
        pos[f] = e;
        r[f] = act[f] ? (k.perm ? k.perm[e] : e) : 0u;
        best[f] = 0u;
    }
    // a wave without candidates only helps to stream the tiles (same loads and barriers)
    if (__builtin_amdgcn_readfirstlane(c0 + wave * (FB * 32) < c1 ? 1 : 0)) {
        // the candidates' operands are built while the first tiles load
        stream_tiles_after<KS * 64, G, MP_NB, MP_NT>(
            frag, t0, t1, lds,
            [&]() __attribute__((always_inline)) {
#pragma unroll
                for (int f = 0; f < FB; ++f) contain_operand<KS, true>(B, r[f], act[f], half, b[f]);
            },
            [&](const uint4 *tf) __attribute__((always_inline)) {
                contain_tile<KS, COUNT, FB, true>(tf, lane, b, best, 1u);
            });
    } else {
        stream_tiles<KS * 64, G, MP_NB, MP_NT>(frag, t0, t1, lds, [&](const uint4 *) __attribute__((always_inline)) {});
    }
    const uint32_t nrec = k.desc[2 * (size_t)blockIdx.x + 1].x;
#pragma unroll
    for (int f = 0; f < FB; ++f) {
        const uint32_t o = (uint32_t)__shfl_xor((int)best[f], 32, 64);
        const uint32_t h = COUNT ? nrec - (best[f] + o) / 8u : (max((int)best[f], (int)o) > 0 ? 0u : 1u);
        if (half == 0 && act[f]) out[k.by_position ? pos[f] : r[f]] = h;
    }
}

// One contraction launch of width V with F column sets per wave (ternary rows at 5
// words take two sets: three spill).
template <int V, int F>
static void launch_cm(bool count, bool ternary, const uint64_t *B, size_t m, const uint4 *frag, uint32_t ntiles,
                      uint32_t pad, uint32_t *out, hipStream_t s) {
    constexpr int FT = (V == 5 && F == 3) ? 2 : F;
    const dim3 grid((unsigned)((m + mf_cols<F>() - 1) / mf_cols<F>()));
    const dim3 gridt((unsigned)((m + mf_cols<FT>() - 1) / mf_cols<FT>()));
    if (count && ternary)
        hipLaunchKernelGGL((k_contain_mfma<V, true, FT, true>), gridt, dim3(MF_NT), 0, s, B, (uint32_t)m, frag, ntiles,
                           pad, out);
    else if (count)
        hipLaunchKernelGGL((k_contain_mfma<V, true, F, false>), grid, dim3(MF_NT), 0, s, B, (uint32_t)m, frag, ntiles,
                           pad, out);
    else if (ternary)
        hipLaunchKernelGGL((k_contain_mfma<V, false, FT, true>), gridt, dim3(MF_NT), 0, s, B, (uint32_t)m, frag,
                           ntiles, pad, out);
    else
        hipLaunchKernelGGL((k_contain_mfma<V, false, F, false>), grid, dim3(MF_NT), 0, s, B, (uint32_t)m, frag, ntiles,
                           pad, out);
}

void launch_contain_mfma(int KO, bool count, const uint64_t *B, size_t m, const uint4 *frag, uint32_t n_rec,
                         uint32_t *out, hipStream_t s, int sets, bool ternary) {
    if (!m) return;
    IG_REQUIRE(m < (1ull << 32), IG_E_UNSUPPORTED, "more than 2^32 rows in one matrix-core launch");
    // the ternary support counts 8 per record lacking a candidate in 32 bits
    IG_REQUIRE(n_rec < (1u << 28), IG_E_UNSUPPORTED, "more than 2^28 records in one matrix-core launch");
    IG_REQUIRE(KO >= 1 && KO <= 16, IG_E_UNSUPPORTED, "the matrix-core subset tests handle up to 16 operand words");
    IG_REQUIRE(sets >= 0 && sets <= 3, IG_E_INVAL, "column sets per wave must be 0 (default) to 3");
    const int fb = sets ? std::min(sets, mf_max_sets(KO)) : 0;
    const uint32_t ntiles = (n_rec + 31) / 32, pad = 32 * ntiles - n_rec;
#define IG_CM(V)                                                                                                 \
    case V:                                                                                                      \
        if (fb == 1 || (fb == 0 && mf_sets<V>() == 1))                                                           \
            launch_cm<V, 1>(count, ternary, B, m, frag, ntiles, pad, out, s);                                    \
        else if (fb == 2 || (fb == 0 && mf_sets<V>() == 2))                                                      \
            launch_cm<V, (mf_max_sets(V) >= 2 ? 2 : 1)>(count, ternary, B, m, frag, ntiles, pad, out, s);        \
        else                                                                                                     \
            launch_cm<V, (mf_max_sets(V) >= 3 ? 3 : 1)>(count, ternary, B, m, frag, ntiles, pad, out, s);        \
        break;
    switch (KO) {
        IG_CM(1) IG_CM(2) IG_CM(3) IG_CM(4) IG_CM(5) IG_CM(6) IG_CM(7) IG_CM(8)
        IG_CM(9) IG_CM(10) IG_CM(11) IG_CM(12) IG_CM(13) IG_CM(14) IG_CM(15) IG_CM(16)
        default: break;
    }
#undef IG_CM
    IG_HIP(hipGetLastError());
}

// Column sets per wave of the pruned contraction at KO words (ternary rows).
static int pruned_sets(int KO, int sets) {
    int fb = sets ? std::min(sets, mf_max_sets(KO)) : (KO <= 5 ? IG_MF_SETS_NARROW : KO <= 8 ? 2 : 1);
    fb = std::min(fb, mf_max_sets(KO));
    if (KO == 5 && fb == 3) fb = 2;   // three spill with ternary rows at 5 words
    return fb;
}

uint32_t contain_pruned_cols(int KO, int sets) { return (uint32_t)(MP_NT / 64 * 32 * pruned_sets(KO, sets)); }

template <int V, int F>
static void launch_cmp(bool count, const uint64_t *B, const uint4 *frag, const ContainBuckets &k, uint32_t units,
                       uint32_t *out, hipStream_t s) {
    if (count)
        hipLaunchKernelGGL((k_contain_mfma_pruned<V, true, F>), dim3(units), dim3(MP_NT), 0, s, B, frag, k, out);
    else
        hipLaunchKernelGGL((k_contain_mfma_pruned<V, false, F>), dim3(units), dim3(MP_NT), 0, s, B, frag, k, out);
}

void launch_contain_mfma_pruned(int KO, bool count, const uint64_t *B, const uint4 *frag, const ContainBuckets &k,
                                uint32_t units, uint32_t *out, hipStream_t s, int sets) {
    if (!units) return;
    IG_REQUIRE(KO >= 1 && KO <= 16, IG_E_UNSUPPORTED, "the matrix-core subset tests handle up to 16 operand words");
    IG_REQUIRE(sets >= 0 && sets <= 3, IG_E_INVAL, "column sets per wave must be 0 (default) to 3");
    IG_REQUIRE(k.desc != nullptr, IG_E_INVAL, "no work-unit ranges");
    const int fb = pruned_sets(KO, sets);
#define IG_CMP(V)                                                                             \
    case V:                                                                                   \
        if (fb == 1) launch_cmp<V, 1>(count, B, frag, k, units, out, s);                      \
        else if (fb == 2) launch_cmp<V, (mf_max_sets(V) >= 2 ? 2 : 1)>(count, B, frag, k, units, out, s); \
        else launch_cmp<V, (mf_max_sets(V) >= 3 && V != 5 ? 3 : 1)>(count, B, frag, k, units, out, s); \
        break;
    switch (KO) {
        IG_CMP(1) IG_CMP(2) IG_CMP(3) IG_CMP(4) IG_CMP(5) IG_CMP(6) IG_CMP(7) IG_CMP(8)
        IG_CMP(9) IG_CMP(10) IG_CMP(11) IG_CMP(12) IG_CMP(13) IG_CMP(14) IG_CMP(15) IG_CMP(16)
        default: break;
    }
#undef IG_CMP
    IG_HIP(hipGetLastError());
}

// Scoring (Eq. 4) as the same contraction: V[b][t] = sum over tokens of
// b[token] * t'[token] is 0 exactly when pattern b lies inside flow t, with t' the
// complement of the flow's one-hot words or the signed side of its factored
// tokens.  Patterns are the A operand (rows), pre-expanded per model with their
// weights in accumulator order; flows are the B operand (columns), built from
// their codes in registers.  Accumulator register r of lane half h holds row
// (r / 4) * 8 + 4 h + r % 4 of the 32-row tile.
__device__ __forceinline__ uint32_t acc_row(uint32_t half, uint32_t r) { return (r >> 2) * 8 + half * 4 + (r & 3); }

// Scoring operands of a pattern set: KS * 64 + 8 uint4 per 32-row tile
// (score_tile_words).
//  words w < KS, frag[tile * (KS * 64 + 8) + w * 64 + lane]: the nibbles of half
//    (lane/32) of word w of row tile*32 + lane%32, as -1.0 (e2m1 0xA) per token
//    (empty past m), so that an accumulator started at 1.0 ends at 1 - V: 1
//    exactly when the pattern lies inside, at most 0 otherwise.  Ternary rows
//    (tern; W is [m][2 KS], P then V) take the candidate side of the fit's
//    ternary contraction instead, bias slots included, against flows on the
//    record side: an accumulator started at 0 ends at 1 exactly when the pattern
//    lies inside, at most -1 otherwise, and at 0 on the rows past m;
//  then 8 uint4, frag[tile * (KS * 64 + 8) + KS * 64 + 4 h + c]: the lanes of the
//    A operand of the weighting product (v_mfma_i32_32x32x32_i8) that are not
//    zero, lane 32 h + c for c < 4: byte j holds 7-bit chunk c of the weight of the
//    row in accumulator j of half h (0 past m); every other lane of that operand
//    is zero.
// One wave per 32-row tile (four per workgroup): lane l takes row l % 32 and half
// l / 32 of every word, and each word is one contiguous 1 KB store.  The weight
// slice gathers the 16 rows of a lane's accumulators with lane shuffles.
// With buckets, the tiles of bucket u are [bt[u], bt[u + 1]) and hold positions
// [brow[u], brow[u + 1]) of the order perm (position e is row perm[e]), 32 per
// tile, the last tile of a bucket padded with empty rows: every tile holds the
// patterns of one bucket only.  Without, tile t holds rows [32 t, 32 t + 32).
template <int KS>
__global__ __launch_bounds__(256) void k_mfma_patterns(const uint64_t *__restrict__ W, const int64_t *__restrict__ S,
                                                      uint32_t m, uint32_t ntiles, bool spare, bool tern,
                                                      const uint32_t *__restrict__ perm,
                                                      const uint32_t *__restrict__ bt,
                                                      const uint2 *__restrict__ tr, uint4 *__restrict__ frag) {
    const uint32_t tile = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tile >= ntiles) return;   // uniform over the wave
    const uint32_t lane = threadIdx.x & 63, half = lane >> 5, r = lane & 31;
    uint32_t pos = tile * 32 + r;
    bool in = pos < m;
    if (bt) {
        // the tile's first position and the end of its bucket's positions
        const uint2 t = tr[tile];
        pos = t.x + r;
        in = pos < t.y;
    }
    const uint32_t row = in ? (perm ? perm[pos] : pos) : 0u;
    uint4 *dst = frag + (size_t)tile * score_tile_words(KS);
    const uint32_t RW = tern ? 2 * KS : KS;   // words per row
    const uint32_t *rw = reinterpret_cast<const uint32_t *>(W + (size_t)row * RW) + half;
    // ternary rows (P then V, 2 KS words, 16-byte aligned) as 16-byte loads; this
    // lane's 32-bit half of each word picked from them
    uint32_t ph[KS], vh[KS];
    uint32_t np = 0;   // ternary: |P| of the row (both halves of the wave hold it)
    if (tern) {
        const uint4 *r4 = reinterpret_cast<const uint4 *>(W + (size_t)row * RW);
        uint32_t x[4 * KS];
#pragma unroll
        for (int q = 0; q < KS; ++q) {
            const uint4 v = in ? r4[q] : make_uint4(0, 0, 0, 0);
            x[4 * q] = v.x;
            x[4 * q + 1] = v.y;
            x[4 * q + 2] = v.z;
            x[4 * q + 3] = v.w;
        }
#pragma unroll
        for (int w = 0; w < KS; ++w) {
            ph[w] = half ? x[2 * w + 1] : x[2 * w];
            vh[w] = half ? x[2 * (KS + w) + 1] : x[2 * (KS + w)];
            np += __popc(ph[w]);
        }
        np += (uint32_t)__shfl_xor((int)np, 32, 64);
    }
#pragma unroll
    for (int w = 0; w < KS; ++w) {
        const uint32_t d = tern ? ph[w] : (in ? rw[2 * w] : 0u);
        uint4 v;
        if (tern) {
            // the candidate side of the ternary contraction (k_contain_mfma): +1.0
            // on P AND NOT V, -1.0 on P AND V, and the row's bias nibbles (1 - |P|;
            // rows past m have none) in the upper half of the last word
            const uint32_t V = vh[w];
            v = make_uint4(spread8(d) | spread8(V) * 4u, spread8(d >> 8) | spread8(V >> 8) * 4u,
                           spread8(d >> 16) | spread8(V >> 16) * 4u, spread8(d >> 24) | spread8(V >> 24) * 4u);
            if (in && half && w == KS - 1) {
                v.x |= tern_bias_word(np, 0);
                v.y |= tern_bias_word(np, 1);
                v.z |= tern_bias_word(np, 2);
                v.w |= tern_bias_word(np, 3);
            }
        } else {
            v = make_uint4(spread8(d) * 5u, spread8(d >> 8) * 5u, spread8(d >> 16) * 5u, spread8(d >> 24) * 5u);
            // +1.0 (0x2) at the spare token: bit 63 of the last word = top nibble of the upper half
            if (spare && w == KS - 1 && half) v.w = (v.w & 0x0fffffffu) | 0x20000000u;
        }
        dst[w * 64 + lane] = v;
    }
    const int64_t sv = in ? S[row] : 0;
    const uint32_t s_lo = (uint32_t)sv, s_hi = (uint32_t)((uint64_t)sv >> 32);
    uint32_t q[4] = {0, 0, 0, 0};
#pragma unroll
    for (uint32_t j = 0; j < 16; ++j) {
        const int src = (int)acc_row(half, j);   // lane src (half 0) holds that row's weight
        const uint64_t v = (uint64_t)(uint32_t)__shfl((int)s_lo, src, 64) |
                           (uint64_t)(uint32_t)__shfl((int)s_hi, src, 64) << 32;
        const uint32_t chunk = r < 4 ? (uint32_t)(v >> (7 * r)) & 127u : 0u;
        q[j / 4] |= chunk << (8 * (j % 4));
    }
    if (r < 4) dst[KS * 64 + half * 4 + r] = make_uint4(q[0], q[1], q[2], q[3]);
}

// tb[t] = the bucket u of tile t: bt[u] <= t < bt[u + 1] (the last such u).
__global__ void k_tile_bucket(const uint32_t *__restrict__ bt, const uint32_t *__restrict__ brow, uint32_t L,
                              uint32_t ntiles, uint2 *__restrict__ tr) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    // the bucket u of the tile: bt[u] <= t < bt[u + 1] (bt[0] = 0, bt[L] = ntiles)
    uint32_t lo = 0, hi = L;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) / 2;
        if (bt[mid] <= t) lo = mid;
        else hi = mid;
    }
    tr[t] = make_uint2(brow[lo] + (t - bt[lo]) * 32, brow[lo + 1]);
}

// Scoring workgroups: SC_NT threads, at most SC_WPS waves per SIMD (the weighting
// product's int32 accumulators need more registers than the fit's kernels).
#ifndef IG_SCORE_NT
#define IG_SCORE_NT 256
#endif
#ifndef IG_SCORE_WPS
#define IG_SCORE_WPS 3
#endif
// ring: groups of IG_SCORE_GTOK / (KS + 1) tiles (4 at four or five operand
// words), two buffers; three workgroups of 256 threads then fit a CU's LDS
#ifndef IG_SCORE_GTOK
#define IG_SCORE_GTOK 24
#endif
#ifndef IG_SCORE_NB
#define IG_SCORE_NB 2
#endif
constexpr int SC_NB = IG_SCORE_NB;
constexpr int SC_NT = IG_SCORE_NT;
constexpr int SC_WPS = IG_SCORE_WPS;
constexpr int SC_COLS = SC_NT / 64 * MF_FB * 32;
template <int KS>
constexpr int sc_group() { return IG_SCORE_GTOK / (KS + 1) > 0 ? IG_SCORE_GTOK / (KS + 1) : 1; }
// pruned scoring's ring (its work units stream a few tiles each)
#ifndef IG_PRUNE_GTOK
#define IG_PRUNE_GTOK IG_SCORE_GTOK
#endif
#ifndef IG_PRUNE_NB
#define IG_PRUNE_NB IG_SCORE_NB
#endif
constexpr int SP_NB = IG_PRUNE_NB;
template <int KS>
constexpr int sp_group() { return IG_PRUNE_GTOK / (KS + 1) > 0 ? IG_PRUNE_GTOK / (KS + 1) : 1; }

struct ScoreMfmaArgs {
    const uint4 *frag[2];
    uint32_t ntiles[2];
    uint32_t ranges;            // ranges over the tiles of class 0 then class 1 (a multiple of 8)
    uint32_t fblocks;           // workgroups over the flows
    const uint16_t *codes;      // [n][d] or null
    const uint64_t *words;      // [n][K] or null
    const uint32_t *meta;
    const uint16_t *nbins;
    int64_t *out;
    uint32_t n_flows, d, K;
    FactorView fv;              // fv.KF > 0: flows (codes) are factored like the patterns
    uint64_t tbias[2];          // ternary: the bias slots' constants, upper half of the last word
};

// B operand of flow t for one 32-column set of a wave (lane half `half` supplies
// the 32-token halves): the complement of its one-hot words, or the signed side
// of its factored tokens.  Returns whether the flow is active with every code in
// range; otherwise its operand is the empty set, inside which no pattern lies.
// Forms of the scoring contraction: one-hot or factored tokens with the count's
// starting +1 in the accumulator (SF_PLAIN) or on the spare token (SF_SPARE), or
// ternary bit tokens with bias slots (SF_TERN).
enum { SF_PLAIN = 0, SF_SPARE = 1, SF_TERN = 2 };

template <int KS, int SF>
__device__ __forceinline__ bool flow_operand(const ScoreMfmaArgs &a, uint32_t t, bool act, int half,
                                             v8i_t (&b)[KS]) {
    uint64_t wd[KS];
    bool ok = act;
    if (a.fv.KF) {
        // factored tokens: the flow is the signed side (FactorView::tok).  Its
        // bit tokens come from its factored row (bin bit 0: +1.0, 1: -1.0), its
        // presence tokens from the popcounts of its bin indices; an inactive or
        // invalid flow is +1.0 on every token (the empty set: no pattern lies inside).
        // Ternary: bit tokens only, the bias slots' constants of a record tile row,
        // and an inactive or invalid flow 0 everywhere (every product 0)
        const uint16_t *row = a.codes + (size_t)(act ? t : 0u) * a.d;
        if (act)
            for (uint32_t ft = 0; ft < a.d; ++ft) ok &= row[ft] < a.nbins[ft];
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            uint64_t v = 0;   // the flow's factored word k (pattern side: bits and presence)
            uint64_t lo = SF == SF_TERN ? 0ull : 0x2222222222222222ull, hi = lo;
            if (ok) {
                for (uint32_t f = a.fv.fbeg[k]; f < a.fv.fend[k]; ++f) {
                    const FacFeature ft = a.fv.feat[f];
                    if ((uint32_t)k - ft.w0 >= ft.nw) continue;
                    v |= a.fv.mask[ft.mask + (uint32_t)row[f] * ft.nw + (k - ft.w0)];
                }
                const uint64_t bw = a.fv.bitw[k];
                const uint32_t ones = (uint32_t)((v & bw) >> (32 * half)), zeros = (uint32_t)((~v & bw) >> (32 * half));
                lo = (uint64_t)(spread8(zeros) | spread8(ones) * 5u) |
                     (uint64_t)(spread8(zeros >> 8) | spread8(ones >> 8) * 5u) << 32;
                hi = (uint64_t)(spread8(zeros >> 16) | spread8(ones >> 16) * 5u) |
                     (uint64_t)(spread8(zeros >> 24) | spread8(ones >> 24) * 5u) << 32;
                for (uint32_t f = a.fv.fbeg[k]; SF != SF_TERN && f < a.fv.fend[k]; ++f) {
                    const uint32_t pt = a.fv.ptok[f];
                    if (pt == ~0u) continue;
                    const uint32_t pc = __popc(row[f]);
                    for (uint32_t part = 0; part < (pt >> 24); ++part) {
                        const uint32_t tk = (pt & 0xffffffu) + part;
                        if (tk / 64 != (uint32_t)k || (tk % 64) / 32 != (uint32_t)half) continue;
                        const uint32_t j = tk % 32;
                        const uint64_t nib = signed_nibble(2u + part, 0u, pc);
                        if (j < 16) lo |= nib << (4 * j);
                        else hi |= nib << (4 * (j - 16));
                    }
                }
            }
            // the spare token is +1.0 in every flow (it carries the count's starting +1)
            if (SF == SF_SPARE && k == KS - 1 && half) hi = (hi & 0x0fffffffffffffffull) | 0x2000000000000000ull;
            if (SF == SF_TERN && ok && k == KS - 1 && half) {
                lo |= a.tbias[0];
                hi |= a.tbias[1];
            }
            b[k] = v8i_t{(int)(uint32_t)lo, (int)(uint32_t)(lo >> 32), (int)(uint32_t)hi,
                         (int)(uint32_t)(hi >> 32), 0, 0, 0, 0};
        }
        return ok;
    }
    if (act && a.codes) {
        const uint16_t *row = a.codes + (size_t)t * a.d;
        const uint32_t *off = a.meta, *flo = a.meta + a.d, *fhi = a.meta + a.d + KS;
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            uint64_t v = 0;
            for (uint32_t ft = flo[k]; ft < fhi[k]; ++ft) {
                const uint32_t c = row[ft];
                ok &= c < a.nbins[ft];
                const uint32_t bit = off[ft] + c;
                if ((bit >> 6) == (uint32_t)k) v |= 1ull << (bit & 63);
            }
            wd[k] = v;
        }
    } else {
#pragma unroll
        for (int k = 0; k < KS; ++k) wd[k] = (act && k < (int)a.K) ? a.words[(size_t)t * a.K + k] : 0ull;
    }
#pragma unroll
    for (int k = 0; k < KS; ++k) {
        // NOT t; an inactive or invalid flow is the empty set, which contains no pattern.
        // The spare token is 1 in every flow (it carries the count's starting +1).
        uint64_t nt = ok ? ~wd[k] : ~0ull;
        if (SF == SF_SPARE && k == KS - 1) nt |= 1ull << 63;
        const uint32_t dwd = (uint32_t)(nt >> (32 * half));
        b[k] = v8i_t{(int)spread8(dwd), (int)spread8(dwd >> 8), (int)spread8(dwd >> 16), (int)spread8(dwd >> 24),
                     0, 0, 0, 0};
    }
    return ok;
}

// One 32-pattern tile against the wave's column sets: the containment counts on
// the fp4 matrix cores, then the weighting product adds the weight chunks of the
// patterns inside each flow to C.
template <int KS, int SF>
__device__ __forceinline__ void score_tile(const uint4 *tile, int lane, const v8i_t (&b)[MF_FB][KS],
                                           v16i_t (&C)[MF_FB]) {
    // the count starts at +1: from the spare token or the bias slots, or here
    v16f_t acc[MF_FB];
#pragma unroll
    for (int f = 0; f < MF_FB; ++f)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[f][r] = SF == SF_PLAIN ? 1.0f : 0.0f;
#pragma unroll
    for (int w = 0; w < KS; ++w) {
        const uint4 a4 = tile[w * 64 + lane];
        const v8i_t av = {(int)a4.x, (int)a4.y, (int)a4.z, (int)a4.w, 0, 0, 0, 0};
#pragma unroll
        for (int f = 0; f < MF_FB; ++f)
            acc[f] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av, b[f][w], acc[f], 4, 4, 0, 127, 0, 127);
    }
    // weight chunks of this tile as the A operand (lanes 32 h + c, c < 4; the
    // other lanes zero)
    const uint4 q = tile[KS * 64 + (lane >> 5) * 4 + (lane & 3)];
    const bool wl = (lane & 31) < 4;
    const v4i_t wa = {wl ? (int)q.x : 0, wl ? (int)q.y : 0, wl ? (int)q.z : 0, wl ? (int)q.w : 0};
#pragma unroll
    for (int f = 0; f < MF_FB; ++f) {
        // inside = max(acc, 0) as a byte (1 or 0), accumulator r -> byte r
        v4i_t z;
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
            uint32_t d = __builtin_amdgcn_cvt_pk_u8_f32(acc[f][4 * qq], 0, 0u);
            d = __builtin_amdgcn_cvt_pk_u8_f32(acc[f][4 * qq + 1], 1, d);
            d = __builtin_amdgcn_cvt_pk_u8_f32(acc[f][4 * qq + 2], 2, d);
            d = __builtin_amdgcn_cvt_pk_u8_f32(acc[f][4 * qq + 3], 3, d);
            z[qq] = (int)d;
        }
        C[f] = __builtin_amdgcn_mfma_i32_32x32x32_i8(wa, z, C[f], 0, 0, 0);
    }
}

// Adds the weighting sums of the wave's valid flows to their column of out (A from
// class 1, N from class 0).
__device__ __forceinline__ void score_flush(int64_t *out, int cls, int half, const v16i_t (&C)[MF_FB],
                                            const uint32_t (&tf)[MF_FB], const bool (&valid)[MF_FB]) {
    const int colsel = cls == 1 ? 0 : 1;
#pragma unroll
    for (int f = 0; f < MF_FB; ++f) {
        uint64_t v = 0;
#pragma unroll
        for (int c = 0; c < 4; ++c) v += (uint64_t)(uint32_t)C[f][c] << (7 * c);
        if (half == 0 && valid[f] && v)
            atomicAdd(reinterpret_cast<unsigned long long *>(out + 2 * (size_t)tf[f] + colsel),
                      (unsigned long long)v);
    }
}

// Workgroup (range, flow block): the fblocks workgroups that read the same range
// of pattern tiles get ids that differ by multiples of 8, so they are dispatched
// to one XCD and share its L2.  The ranges split the tiles of both classes, taken
// one after the other, into equal parts; a range that holds tiles of both classes
// scans them as two segments and adds each class's sums to its own column.
template <int KS, int SF>
__global__ __launch_bounds__(SC_NT, SC_WPS) void k_score_mfma(ScoreMfmaArgs a) {
    constexpr int G = sc_group<KS>();
    constexpr int TW = KS * 64 + 8;
    __shared__ uint4 lds[ring_lds<TW, G, SC_NB>()];
    const uint32_t id = blockIdx.x, xcd = id % 8, seq = id / 8;
    const uint32_t range = (seq / a.fblocks) * 8 + xcd, fb = seq % a.fblocks;
    if (range >= a.ranges) return;   // uniform over the workgroup
    const uint64_t T = (uint64_t)a.ntiles[0] + a.ntiles[1];
    const uint32_t u0 = (uint32_t)(T * range / a.ranges), u1 = (uint32_t)(T * (range + 1) / a.ranges);
    if (u0 >= u1) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, half = lane >> 5, col = lane & 31;
    v8i_t b[MF_FB][KS];
    uint32_t tf[MF_FB];
    bool valid[MF_FB];   // active, with every code in range (the others keep their -1)
#pragma unroll
    for (int f = 0; f < MF_FB; ++f) {
        const uint32_t t = fb * SC_COLS + wave * (MF_FB * 32) + f * 32 + col;
        tf[f] = t;
        valid[f] = flow_operand<KS, SF>(a, t, t < a.n_flows, half, b[f]);
    }
    // C[f]: running weighting products; row c < 4 of column `col` (lane half 0,
    // accumulators 0..3) sums chunk c of the weights of the patterns inside the flow
    v16i_t C[MF_FB];
#pragma nounroll
    for (int cls = 0; cls < 2; ++cls) {
        const uint32_t lo = cls ? a.ntiles[0] : 0u, hi = lo + a.ntiles[cls];
        const uint32_t s0 = u0 > lo ? u0 : lo, s1 = u1 < hi ? u1 : hi;
        if (s0 >= s1) continue;
        // the class-0 segment's last group may still be read from the ring
        if (cls == 1 && u0 < lo) __syncthreads();
#pragma unroll
        for (int f = 0; f < MF_FB; ++f) C[f] = v16i_t{0};
        stream_tiles<TW, G, SC_NB, SC_NT>(a.frag[cls], s0 - lo, s1 - lo, lds, [&](const uint4 *tile) __attribute__((always_inline)) {
            score_tile<KS, SF>(tile, lane, b, C);
        });
        score_flush(a.out, cls, half, C, tf, valid);
    }
}

// Pruned scoring: a pattern can lie inside a flow only when the flow holds every
// token of it, in particular the pattern's bucket token (one token of each pattern,
// chosen when the model was built; the tiles of each class are grouped by it).
// A work unit is (class, bucket u, a range of at most p.rt of the bucket's tiles,
// a block of SC_COLS of the flows holding token u); its flows are tested against
// those tiles only.  Workgroups take units from a queue until it runs dry.  Every
// flow in the lists is valid; the launcher initialised out.  The flows' operands
// are built once per call (k_flow_operands) and loaded by each unit.
struct PruneArgs {
    const uint32_t *btile[2];   // [L + 1]: first tile of each bucket, per class
    const uint32_t *fcnt;       // [L]: flows holding token u
    const uint32_t *foff;       // [L + 1]: start of the list of flows holding token u
    const uint32_t *flist;      // flow ids grouped by token
    const uint32_t *uoff;       // [2L + 1]: first unit of (class, bucket) c * L + u
    const uint4 *ops;           // [n_flows][2][KS]: B operand of each flow and lane half
    uint32_t *queue;            // next unit to take (zero at launch)
    uint32_t L, rt;
};

// B operands of every flow, one thread per (flow, lane half): ops[(t * 2 + half) *
// KS + k] = the four used dwords of word k's operand.
template <int KS, int SF>
__global__ __launch_bounds__(256) void k_flow_operands(ScoreMfmaArgs a, uint4 *__restrict__ ops) {
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= 2 * a.n_flows) return;
    v8i_t b[KS];
    flow_operand<KS, SF>(a, g >> 1, true, (int)(g & 1), b);
#pragma unroll
    for (int k = 0; k < KS; ++k)
        ops[(size_t)g * KS + k] = uint4{(uint32_t)b[k][0], (uint32_t)b[k][1], (uint32_t)b[k][2], (uint32_t)b[k][3]};
}

template <int KS, int SF>
__global__ __launch_bounds__(SC_NT, SC_WPS) void k_score_mfma_pruned(ScoreMfmaArgs a, PruneArgs p) {
    constexpr int G = sp_group<KS>();
    constexpr int TW = KS * 64 + 8;
    __shared__ uint4 lds[ring_lds<TW, G, SP_NB>()];
    __shared__ uint32_t s_unit[2], s_owner[2];
    const uint32_t total = p.uoff[2 * p.L];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, half = lane >> 5, col = lane & 31;
    // the operand of an inactive column (no flow): no pattern lies inside it
    v8i_t bz[KS];
    flow_operand<KS, SF>(a, 0u, false, half, bz);
    // thread 0 takes the next unit one unit ahead, so the queue's latency overlaps work
    uint32_t next = 0;
    if (threadIdx.x == 0) next = atomicAdd(p.queue, 1u);
    for (uint32_t it = 0;; ++it) {
        if (wave == 0) {
            const uint32_t unit = __builtin_amdgcn_readfirstlane(next);
            const uint32_t owner = unit < total ? unit_owner(p.uoff, 2 * p.L, unit) : 0u;
            if (threadIdx.x == 0) {
                s_unit[it & 1] = unit;
                s_owner[it & 1] = owner;
                if (unit < total) next = atomicAdd(p.queue, 1u);
            }
        }
        // the unit is published; every wave is done with the previous unit's ring.
        // (slot it & 1 is rewritten two units later, after the next barrier, by which
        // time every thread has read it)
        __syncthreads();
        const uint32_t unit = s_unit[it & 1], lo = s_owner[it & 1];
        if (unit >= total) break;   // uniform over the workgroup
        const int cls = lo >= p.L ? 1 : 0;
        const uint32_t u = lo - (uint32_t)cls * p.L;
        const uint32_t nf = p.fcnt[u], nb = (nf + SC_COLS - 1) / SC_COLS;
        const uint32_t local = unit - p.uoff[lo], r = local / nb, fb = local % nb;
        const uint32_t t0 = p.btile[cls][u] + r * p.rt, tend = p.btile[cls][u + 1];
        const uint32_t t1 = t0 + p.rt < tend ? t0 + p.rt : tend;
        const uint32_t wave0 = fb * SC_COLS + wave * (MF_FB * 32);   // first slot of the wave
        // a wave without flows in this block only helps to stream the tiles (it takes
        // the same loads and barriers, and skips the products)
        if (__builtin_amdgcn_readfirstlane(wave0 < nf ? 1 : 0)) {
            v8i_t b[MF_FB][KS];
            uint32_t tf[MF_FB];
            bool valid[MF_FB];
            v16i_t C[MF_FB];
            stream_tiles_after<TW, G, SP_NB, SC_NT>(
                a.frag[cls], t0, t1, lds,
                [&]() __attribute__((always_inline)) {
                    const uint32_t *fl = p.flist + p.foff[u];
#pragma unroll
                    for (int f = 0; f < MF_FB; ++f) {
                        const uint32_t slot = wave0 + f * 32 + col;
                        valid[f] = slot < nf;
                        tf[f] = valid[f] ? fl[slot] : 0u;
                    }
#pragma unroll
                    for (int f = 0; f < MF_FB; ++f)
#pragma unroll
                        for (int k = 0; k < KS; ++k) {
                            const uint4 q = p.ops[((size_t)tf[f] * 2 + half) * KS + k];
                            b[f][k] = valid[f] ? v8i_t{(int)q.x, (int)q.y, (int)q.z, (int)q.w, 0, 0, 0, 0} : bz[k];
                        }
#pragma unroll
                    for (int f = 0; f < MF_FB; ++f) C[f] = v16i_t{0};
                },
                [&](const uint4 *tile) __attribute__((always_inline)) { score_tile<KS, SF>(tile, lane, b, C); });
            score_flush(a.out, cls, half, C, tf, valid);
        } else {
            stream_tiles<TW, G, SP_NB, SC_NT>(a.frag[cls], t0, t1, lds,
                                              [&](const uint4 *) __attribute__((always_inline)) {});
        }
    }
}

void launch_mfma_patterns(const uint64_t *W, const int64_t *S, uint32_t m, uint32_t KS, bool spare, bool tern,
                          uint4 *frag, hipStream_t s, const uint32_t *perm, const uint32_t *bt, const uint32_t *brow,
                          uint32_t L, uint32_t ntiles) {
    if (!bt) ntiles = (m + 31) / 32;
    if (!ntiles) return;
    IG_REQUIRE(KS >= 1 && KS <= 8, IG_E_UNSUPPORTED, "matrix-core scoring operands of more than 8 words");
    IG_REQUIRE(!bt || (brow && L >= 1), IG_E_INVAL, "bucket tiles without bucket rows");
    IG_REQUIRE(!(spare && tern), IG_E_INVAL, "ternary scoring operands take no spare token");
    Scratch<uint2> tr;
    if (bt) {
        tr.reset(ntiles, s);
        hipLaunchKernelGGL(k_tile_bucket, dim3((ntiles + 255) / 256), dim3(256), 0, s, bt, brow, L, ntiles, tr.get());
        IG_HIP(hipGetLastError());
    }
    const dim3 grid((ntiles + 3) / 4);
    switch (KS) {
#define IG_MP(V)                                                                                                  \
    case V:                                                                                                       \
        hipLaunchKernelGGL(k_mfma_patterns<V>, grid, dim3(256), 0, s, W, S, m, ntiles, spare, tern, perm, bt, tr.get(), \
                           frag);                                                                                 \
        break;
        IG_MP(1) IG_MP(2) IG_MP(3) IG_MP(4) IG_MP(5) IG_MP(6) IG_MP(7) IG_MP(8)
#undef IG_MP
        default: break;
    }
    IG_HIP(hipGetLastError());
}

uint32_t mfma_record_tiles(uint32_t n) { return (n + 31) / 32; }

void launch_mfma_records_signed(const uint64_t *FR, uint32_t n, const FactorView &fv, uint4 *frag, hipStream_t s) {
    const uint32_t KO = fv.KF, ntiles = mfma_record_tiles(n);
    const size_t total = (size_t)ntiles * KO * 64;
    if (!total) return;
    IG_REQUIRE(fv.tok && fv.fbit, IG_E_DEVICE, "signed record operands without a token table");
    hipLaunchKernelGGL(k_mfma_records_signed, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, FR, n, KO,
                       ntiles, fv, frag);
    IG_HIP(hipGetLastError());
}

void launch_mfma_records_ternary(const uint64_t *FR, uint32_t n, uint32_t KO, uint32_t T, uint4 *frag,
                                 hipStream_t s) {
    const uint32_t ntiles = mfma_record_tiles(n), nslots = tern_bias_slots(T);
    IG_REQUIRE(KO >= 1 && T + nslots <= 64 * KO && nslots <= 32, IG_E_INVAL, "ternary tokens overlap the bias slots");
    const size_t total = (size_t)ntiles * KO * 64;
    if (!total) return;
    hipLaunchKernelGGL(k_mfma_records_ternary, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, FR, n, KO,
                       ntiles, nslots, frag);
    IG_HIP(hipGetLastError());
}

void launch_mfma_records_ternary_lists(const uint64_t *FR, uint32_t KO, uint32_t T, const uint32_t *list,
                                       const uint32_t *ro, const uint32_t *bt, const uint32_t *brec, uint32_t nb,
                                       uint32_t ntiles, uint4 *frag, hipStream_t s) {
    const uint32_t nslots = tern_bias_slots(T);
    IG_REQUIRE(KO >= 1 && T + nslots <= 64 * KO && nslots <= 32, IG_E_INVAL, "ternary tokens overlap the bias slots");
    const size_t total = (size_t)ntiles * KO * 64;
    if (!total) return;
    hipLaunchKernelGGL(k_mfma_records_ternary_lists, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, FR, KO,
                       ntiles, nslots, list, ro, bt, brec, nb, frag);
    IG_HIP(hipGetLastError());
}

void launch_mfma_records(const uint64_t *NX, uint32_t n, uint32_t KS, uint4 *frag, hipStream_t s) {
    const uint32_t ntiles = mfma_record_tiles(n);
    const size_t total = (size_t)ntiles * KS * 64;
    if (!total) return;
    hipLaunchKernelGGL(k_mfma_records, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, NX, n, KS, ntiles,
                       frag);
    IG_HIP(hipGetLastError());
}

// -------------------------------------------------------------- support ----
template <int KS, int CPL>
__global__ __launch_bounds__(256) void k_support(const uint64_t *__restrict__ Wrows, size_t m,
                                                const uint64_t *__restrict__ NX, uint32_t n,
                                                uint32_t *__restrict__ f_out, int64_t *__restrict__ S_out) {
    constexpr int W = 2 * KS;
    const size_t base = (size_t)blockIdx.x * (256 * CPL);
    uint32_t b[CPL][W];
    uint32_t cnt[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        size_t e = base + (size_t)c * 256 + threadIdx.x;
        bool act = e < m;
        const uint32_t *row = reinterpret_cast<const uint32_t *>(Wrows + (act ? e : 0) * KS);
#pragma unroll
        for (int k = 0; k < W; ++k) b[c][k] = act ? row[k] : 0u;
        cnt[c] = 0;
    }
    cptr32 R = (cptr32)(const void *)NX;
    for (uint32_t r = 0; r < n; ++r) {
        cptr32 rr = R + (size_t)r * W;
#pragma unroll
        for (int c = 0; c < CPL; ++c) cnt[c] += masked_or<W>(rr, b[c]) == 0u;
    }
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        size_t e = base + (size_t)c * 256 + threadIdx.x;
        if (e < m) {
            uint32_t len = 0;
#pragma unroll
            for (int k = 0; k < W; ++k) len += __popc(b[c][k]);
            f_out[e] = cnt[c];
            S_out[e] = (int64_t)cnt[c] * (int64_t)len * (int64_t)len;
        }
    }
}

// ---------------------------------------------------------------- score ----
struct ScoreArgs {
    const uint64_t *P[2];
    const int64_t *S[2];
    uint64_t np[2];
    uint64_t chunk[2];          // patterns per y-block
    const uint16_t *codes;      // [n][d] or null
    const uint64_t *words;      // [n][K] or null
    const uint32_t *meta;       // off[d] | flo[KS] | fhi[KS]
    const uint16_t *nbins;
    int64_t *out;               // [n][2] = (A, N)
    uint32_t n_flows, d, K;
    uint32_t narrow[2];         // all weights of the class below 2^31
    uint32_t flush[2];          // patterns per 32-bit partial sum
};

template <int KS>
__device__ __forceinline__ bool load_flow(const ScoreArgs &a, uint32_t t, uint32_t (&nt)[2 * KS]) {
    uint64_t w[KS];
    bool ok = true;
    if (a.codes) {
        const uint16_t *row = a.codes + (size_t)t * a.d;
        const uint32_t *off = a.meta, *flo = a.meta + a.d, *fhi = a.meta + a.d + KS;
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            uint64_t v = 0;
            for (uint32_t f = flo[k]; f < fhi[k]; ++f) {
                uint32_t c = row[f];
                ok &= c < a.nbins[f];
                uint32_t bit = off[f] + c;
                if ((bit >> 6) == (uint32_t)k) v |= 1ull << (bit & 63);
            }
            w[k] = v;
        }
    } else {
        const uint64_t *row = a.words + (size_t)t * a.K;
#pragma unroll
        for (int k = 0; k < KS; ++k) w[k] = k < (int)a.K ? row[k] : 0ull;
    }
#pragma unroll
    for (int k = 0; k < KS; ++k) {
        // complement; an invalid flow contains nothing, so no pattern matches it
        uint64_t c = ok ? ~w[k] : ~0ull;
        nt[2 * k] = (uint32_t)c;
        nt[2 * k + 1] = (uint32_t)(c >> 32);
    }
    return ok;
}

__global__ void k_score_init(ScoreArgs a) {
    uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.n_flows) return;
    bool ok = true;
    if (a.codes) {
        const uint16_t *row = a.codes + (size_t)t * a.d;
        for (uint32_t f = 0; f < a.d; ++f) ok &= row[f] < a.nbins[f];
    }
    int64_t v = ok ? 0 : -1;
    a.out[2 * (size_t)t] = v;
    a.out[2 * (size_t)t + 1] = v;
}

template <int KS, int FPL>
__global__ __launch_bounds__(256) void k_score(ScoreArgs a) {
    constexpr int W = 2 * KS;
    const int cls = blockIdx.z;
    const uint64_t np = a.np[cls];
    const uint64_t p0 = (uint64_t)blockIdx.y * a.chunk[cls];
    if (p0 >= np) return;
    const uint64_t p1 = p0 + a.chunk[cls] < np ? p0 + a.chunk[cls] : np;
    uint32_t nt[FPL][W];
    uint64_t sum[FPL];
    bool act[FPL];
#pragma unroll
    for (int c = 0; c < FPL; ++c) {
        uint32_t t = (blockIdx.x * FPL + c) * 256 + threadIdx.x;
        act[c] = t < a.n_flows;
        load_flow<KS>(a, act[c] ? t : 0, nt[c]);
        sum[c] = 0;
    }
    cptr32 P = (cptr32)(const void *)a.P[cls] + p0 * W;
    cptr64 S = (cptr64)(const void *)a.S[cls] + p0;
    const uint32_t cnt = (uint32_t)(p1 - p0);
    if (a.narrow[cls]) {
        // every weight < 2^31: 32-bit partial sums, flushed before they can wrap
        const uint32_t flush = a.flush[cls];
        for (uint32_t q0 = 0; q0 < cnt; q0 += flush) {
            const uint32_t q1 = q0 + flush < cnt ? q0 + flush : cnt;
            uint32_t lo[FPL];
#pragma unroll
            for (int c = 0; c < FPL; ++c) lo[c] = 0;
            for (uint32_t q = q0; q < q1; ++q) {
                cptr32 pp = P + (size_t)q * W;
                const uint32_t s = (uint32_t)S[q];
#pragma unroll
                for (int c = 0; c < FPL; ++c)
                    if (masked_or<W>(pp, nt[c]) == 0u) lo[c] += s;
            }
#pragma unroll
            for (int c = 0; c < FPL; ++c) sum[c] += lo[c];
        }
    } else {
        for (uint32_t q = 0; q < cnt; ++q) {
            cptr32 pp = P + (size_t)q * W;
            const int64_t s = S[q];
#pragma unroll
            for (int c = 0; c < FPL; ++c)
                if (masked_or<W>(pp, nt[c]) == 0u) sum[c] += (uint64_t)s;
        }
    }
    const int col = cls == 1 ? 0 : 1;   // A from class 1, N from class 0
#pragma unroll
    for (int c = 0; c < FPL; ++c) {
        uint32_t t = (blockIdx.x * FPL + c) * 256 + threadIdx.x;
        if (act[c] && sum[c]) atomicAdd(reinterpret_cast<unsigned long long *>(a.out + 2 * (size_t)t + col),
                                        (unsigned long long)sum[c]);
    }
}

// largest S and total of S (for the int64 overflow bound of Eq. 4 sums); a
// bounded grid strides over S and adds one atomic pair per workgroup
__global__ __launch_bounds__(256) void k_maxsum(const int64_t *__restrict__ S, size_t m,
                                               unsigned long long *__restrict__ ms) {
    __shared__ unsigned long long smx[4], ssm[4];
    unsigned long long mx = 0, sm = 0;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (size_t)gridDim.x * blockDim.x) {
        unsigned long long v = (unsigned long long)S[e];
        mx = v > mx ? v : mx;
        sm += v;
    }
    for (int o = 32; o > 0; o >>= 1) {
        unsigned long long u = __shfl_xor(mx, o, 64);
        mx = u > mx ? u : mx;
        sm += __shfl_xor(sm, o, 64);
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { smx[wave] = mx; ssm[wave] = sm; }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long a = smx[0], b = ssm[0];
        for (int w = 1; w < 4; ++w) { a = smx[w] > a ? smx[w] : a; b += ssm[w]; }
        atomicMax(&ms[0], a);
        atomicAdd(&ms[1], b);
    }
}

// ---------------------------------------------------------- dispatching ----
#define IG_FOR_EACH_KS(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(10) X(12) X(14) X(16) X(20) X(24) X(28) X(32) X(40) X(48) X(56) X(64)

int storage_words(int K) {
    static const int ks[] = {1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16, 20, 24, 28, 32, 40, 48, 56, 64};
    for (int v : ks)
        if (K <= v) return v;
    return -1;
}

uint32_t device_cus() {
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cached[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            cached[dev] = v;
        else
            cached[dev] = 256;
    }
    return (uint32_t)cached[dev];
}

// Workgroups of `kernel` (threads each, static LDS only) that one XCD runs at once:
// its eighth of the compute units times the workgroups per compute unit.
static uint32_t xcd_slots(const void *kernel, int threads) {
    int per_cu = 0;
    IG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0));
    const uint32_t cus = device_cus();
    const uint32_t s = (cus >= 8 ? cus / 8 : 1) * (uint32_t)(per_cu > 0 ? per_cu : 1);
    return s ? s : 1;
}

uint32_t coherence_grid(uint32_t grid_per_cu) {
    const uint32_t cus = device_cus();
    if (grid_per_cu < 1) grid_per_cu = 1;
    if (grid_per_cu > 32) grid_per_cu = 32;
    return (uint32_t)cus * grid_per_cu;   // persistent workgroups of 4 waves
}

void launch_coherence(int KS, int cpl, const CohSeg *segs_dev, uint32_t nseg, uint32_t r_begin, uint32_t r_end,
                      uint32_t *queue, uint32_t grid, hipStream_t s) {
    launch_fill_u32(queue, 0u, 1, s);
#define IG_COH(V)                                                                                              \
    case V:                                                                                                    \
        if (cpl == 2 && V <= 16)                                                                               \
            hipLaunchKernelGGL((k_coherence<V, 2>), dim3(grid), dim3(256), 0, s, segs_dev, nseg, r_begin, r_end, queue); \
        else                                                                                                   \
            hipLaunchKernelGGL((k_coherence<V, 1>), dim3(grid), dim3(256), 0, s, segs_dev, nseg, r_begin, r_end, queue); \
        break;
    switch (KS) {
        IG_FOR_EACH_KS(IG_COH)
        default: throw Error(IG_E_UNSUPPORTED, "unsupported word count");
    }
#undef IG_COH
    IG_HIP(hipGetLastError());
}

void launch_support(int KS, int cpl, const uint64_t *W, size_t m, const uint64_t *NX, uint32_t n, uint32_t *f,
                    int64_t *S, hipStream_t s) {
    if (!m) return;
    const int c = (cpl == 2 && KS <= 16) ? 2 : 1;
    dim3 grid((unsigned)((m + 256 * c - 1) / (256 * c)));
#define IG_SUP(V)                                                                                     \
    case V:                                                                                           \
        if (c == 2)                                                                                   \
            hipLaunchKernelGGL((k_support<V, 2>), grid, dim3(256), 0, s, W, m, NX, n, f, S);          \
        else                                                                                          \
            hipLaunchKernelGGL((k_support<V, 1>), grid, dim3(256), 0, s, W, m, NX, n, f, S);          \
        break;
    switch (KS) {
        IG_FOR_EACH_KS(IG_SUP)
        default: throw Error(IG_E_UNSUPPORTED, "unsupported word count");
    }
#undef IG_SUP
    IG_HIP(hipGetLastError());
}

void launch_score(const ScoreModel &m, const uint16_t *codes, const uint64_t *words, uint32_t K, uint32_t n_flows,
                  uint32_t d, const uint32_t *meta, const uint16_t *nbins, int64_t *out, int fpl, hipStream_t s) {
    if (!n_flows) return;
    ScoreArgs a{};
    for (int c = 0; c < 2; ++c) {
        a.P[c] = m.P[c];
        a.S[c] = m.S[c];
        a.np[c] = m.np[c];
    }
    a.codes = codes;
    a.words = words;
    a.meta = meta;
    a.nbins = nbins;
    a.out = out;
    a.n_flows = n_flows;
    a.d = d;
    a.K = K;
    for (int c = 0; c < 2; ++c) {
        const uint64_t mx = m.maxS[c] > 0 ? (uint64_t)m.maxS[c] : 1ull;
        a.narrow[c] = mx < (1ull << 31);
        uint64_t fl = 0xffffffffull / mx;
        a.flush[c] = (uint32_t)(fl < 1 ? 1 : (fl > (1u << 30) ? (1u << 30) : fl));
    }
    hipLaunchKernelGGL(k_score_init, dim3((n_flows + 255) / 256), dim3(256), 0, s, a);
    IG_HIP(hipGetLastError());
    const int KS = (int)m.KS;
    const int f = (fpl == 2 && KS <= 16) ? 2 : 1;
    const uint32_t fblocks = (n_flows + 256 * f - 1) / (256 * f);
    // enough workgroups to fill the chip: split the pattern range into chunks
    const uint64_t target_blocks = 256ull * 32ull;   // ~8 waves per SIMD
    uint64_t npmax = m.np[0] > m.np[1] ? m.np[0] : m.np[1];
    if (npmax == 0) return;
    uint64_t ychunks = (target_blocks + 2ull * fblocks - 1) / (2ull * fblocks);
    if (ychunks < 1) ychunks = 1;
    for (int c = 0; c < 2; ++c) {
        uint64_t ch = (m.np[c] + ychunks - 1) / ychunks;
        if (ch < 64) ch = 64;
        a.chunk[c] = ch;
    }
    uint64_t ny0 = (m.np[0] + a.chunk[0] - 1) / a.chunk[0], ny1 = (m.np[1] + a.chunk[1] - 1) / a.chunk[1];
    uint64_t ny = ny0 > ny1 ? ny0 : ny1;
    if (ny > 65535) {   // grid.y limit: enlarge the chunks
        for (int c = 0; c < 2; ++c) a.chunk[c] = (m.np[c] + 65534) / 65535;
        ny = 65535;
    }
    dim3 grid(fblocks, (unsigned)ny, 2);
#define IG_SC(V)                                                                          \
    case V:                                                                               \
        if (f == 2)                                                                       \
            hipLaunchKernelGGL((k_score<V, 2>), grid, dim3(256), 0, s, a);                \
        else                                                                              \
            hipLaunchKernelGGL((k_score<V, 1>), grid, dim3(256), 0, s, a);                \
        break;
    switch (KS) {
        IG_FOR_EACH_KS(IG_SC)
        default: throw Error(IG_E_UNSUPPORTED, "unsupported word count");
    }
#undef IG_SC
    IG_HIP(hipGetLastError());
}

// Digest: sum over rows e of mix(e, row words, f, S).  Addition modulo 2^64 makes the
// result independent of thread order; mixing in e makes it depend on row order.
__device__ __forceinline__ uint64_t dmix(uint64_t h) {
    h ^= h >> 33;
    h *= 0xff51afd7ed558ccdull;
    h ^= h >> 33;
    h *= 0xc4ceb9fe1a85ec53ull;
    h ^= h >> 33;
    return h;
}

__global__ __launch_bounds__(256) void k_digest(const uint64_t *__restrict__ W, const uint32_t *__restrict__ f,
                                               const int64_t *__restrict__ S, size_t m, uint32_t KS, uint32_t K,
                                               unsigned long long *__restrict__ out) {
    __shared__ unsigned long long part[4];
    unsigned long long acc = 0;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (size_t)gridDim.x * blockDim.x) {
        uint64_t h = 0x9e3779b97f4a7c15ull;   // no position: a digest of the set
        for (uint32_t k = 0; k < K; ++k) h = dmix(h ^ W[e * KS + k]);
        h = dmix(h ^ f[e]);
        h = dmix(h ^ (uint64_t)S[e]);
        acc += h;
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(out, part[0] + part[1] + part[2] + part[3]);
}

void launch_digest(const uint64_t *W, const uint32_t *f, const int64_t *S, size_t m, uint32_t KS, uint32_t K,
                   unsigned long long *out, hipStream_t s) {
    launch_fill_u64(reinterpret_cast<uint64_t *>(out), 0ull, 1, s);
    if (!m) return;
    unsigned g = (unsigned)((m + 255) / 256);
    if (g > 2048) g = 2048;
    hipLaunchKernelGGL(k_digest, dim3(g), dim3(256), 0, s, W, f, S, m, KS, K, out);
    IG_HIP(hipGetLastError());
}

void launch_reduce_maxsum(const int64_t *S, size_t m, unsigned long long *d_max_sum, hipStream_t s) {
    launch_fill_u64(reinterpret_cast<uint64_t *>(d_max_sum), 0ull, 2, s);
    if (!m) return;
    unsigned g = (unsigned)((m + 255) / 256);
    if (g > 1024) g = 1024;
    hipLaunchKernelGGL(k_maxsum, dim3(g), dim3(256), 0, s, S, m, d_max_sum);
    IG_HIP(hipGetLastError());
}

// The form of a model's scoring operands (SF_*).  Ternary operands: the flows carry
// the constants of a record tile row in the bias slots (launch_mfma_records_ternary).
static int score_form(const ScoreModel &m, ScoreMfmaArgs &a) {
    if (!m.fv.ternary) return m.spare ? SF_SPARE : SF_PLAIN;
    IG_REQUIRE(m.fv.KF == m.KO && m.tslots >= 1 && m.tslots <= 32, IG_E_DEVICE,
               "ternary scoring operands without bias slots");
    uint64_t q[2] = {0, 0};
    for (uint32_t sl = 0; sl < m.tslots; ++sl) {
        const uint32_t nib = 31 - sl;   // of the upper half of the last word
        q[nib / 16] |= (uint64_t)(sl ? 0x7u : 0x2u) << (4 * (nib % 16));
    }
    a.tbias[0] = q[0];
    a.tbias[1] = q[1];
    return SF_TERN;
}

void launch_score_mfma(const ScoreModel &m, const uint16_t *codes, const uint64_t *words, uint32_t K,
                       uint32_t n_flows, uint32_t d, const uint32_t *meta, const uint16_t *nbins, int64_t *out,
                       hipStream_t s) {
    if (!n_flows) return;
    ScoreArgs ia{};
    ia.codes = codes;
    ia.words = words;
    ia.meta = meta;
    ia.nbins = nbins;
    ia.out = out;
    ia.n_flows = n_flows;
    ia.d = d;
    ia.K = K;
    hipLaunchKernelGGL(k_score_init, dim3((n_flows + 255) / 256), dim3(256), 0, s, ia);
    IG_HIP(hipGetLastError());
    ScoreMfmaArgs a{};
    for (int c = 0; c < 2; ++c) {
        a.frag[c] = m.frag[c];
        a.ntiles[c] = m.ftiles[c];
    }
    a.codes = codes;
    a.words = words;
    a.meta = meta;
    a.nbins = nbins;
    a.out = out;
    a.n_flows = n_flows;
    a.d = d;
    a.K = K;
    a.fv = m.fv;
    IG_REQUIRE(!m.fv.KF || codes, IG_E_UNSUPPORTED, "factored matrix-core operands score flows given as codes");
    a.fblocks = (n_flows + SC_COLS - 1) / SC_COLS;
    const uint64_t tiles = (uint64_t)a.ntiles[0] + a.ntiles[1];
    if (!tiles) return;
    IG_REQUIRE(m.KO >= 1 && m.KO <= 8, IG_E_UNSUPPORTED, "the matrix-core scoring path handles up to 8 words");
    const void *kernels[8][3] = {
#define IG_SCK(V) {(const void *)k_score_mfma<V, SF_PLAIN>, (const void *)k_score_mfma<V, SF_SPARE>, \
                   (const void *)k_score_mfma<V, SF_TERN>},
        IG_SCK(1) IG_SCK(2) IG_SCK(3) IG_SCK(4) IG_SCK(5) IG_SCK(6) IG_SCK(7) IG_SCK(8)
#undef IG_SCK
    };
    const int form = score_form(m, a);
    const void *kern = kernels[m.KO - 1][form];
    // Equal ranges, 8 r of them (r per XCD): the r * fblocks workgroups of an XCD
    // run in ceil(r * fblocks / slots) rounds of (tiles / 8 r) tiles each, plus a
    // set-up per workgroup (the flows' operands and the ring's first loads, taken
    // as kSetupTiles tiles).  r is chosen to minimise that time: workgroup counts
    // that fill the last round, without making ranges shorter than needed.
    constexpr double kSetupTiles = 32.0;
    static std::atomic<uint32_t> slot_cache[8][3] = {};
    uint32_t slots = slot_cache[m.KO - 1][form].load(std::memory_order_relaxed);
    if (!slots) {
        slots = xcd_slots(kern, SC_NT);
        slot_cache[m.KO - 1][form].store(slots, std::memory_order_relaxed);
    }
    // a few recent choices are kept per thread: serving batches cycle through a small set of
    // flow-block counts over one pattern set, and the search below is up to 4,096 steps
    constexpr int kMemo = 16;
    thread_local uint64_t memo_key[kMemo][3] = {}, memo_r[kMemo] = {};
    thread_local int memo_next = 0;
    // the int32 weighting sums stay exact: at most 2^18 tiles x 32 rows x 127 per range
    const uint64_t rmin = (tiles + 8 * (1ull << 18) - 1) / (8 * (1ull << 18));
    uint64_t rmax = (tiles + 7) / 8;
    if (rmax > 4096) rmax = 4096;
    if (rmax < rmin) rmax = rmin;
    uint64_t best_r = 0;
    for (int i = 0; i < kMemo; ++i)
        if (memo_r[i] && memo_key[i][0] == tiles && memo_key[i][1] == a.fblocks && memo_key[i][2] == slots) {
            best_r = memo_r[i];
            break;
        }
    if (!best_r) {
        best_r = rmin;
        double best = -1.0;
        for (uint64_t r = rmin; r <= rmax; ++r) {
            const uint64_t rounds = (r * a.fblocks + slots - 1) / slots;
            const double t = (double)rounds * ((double)tiles / (8.0 * (double)r) + kSetupTiles);
            if (best < 0.0 || t < best * (1.0 - 1e-9)) {
                best = t;
                best_r = r;
            }
        }
        memo_key[memo_next][0] = tiles;
        memo_key[memo_next][1] = a.fblocks;
        memo_key[memo_next][2] = slots;
        memo_r[memo_next] = best_r;
        memo_next = (memo_next + 1) % kMemo;
    }
    IG_REQUIRE(8 * best_r * a.fblocks < (1ull << 31), IG_E_UNSUPPORTED, "too many flows for one scoring launch");
    a.ranges = (uint32_t)(8 * best_r);
    const dim3 grid((unsigned)(a.ranges * a.fblocks));
    void *args[] = {&a};
    IG_HIP(hipLaunchKernel(kern, grid, dim3(SC_NT), args, 0, s));
}

// Tiles per work unit of pruned scoring: long enough to cover a unit's set-up (the
// flows' operands and the ring's first loads), short enough that the units of a
// large bucket spread over many workgroups.
#ifndef IG_PRUNE_RT
#define IG_PRUNE_RT 128
#endif

bool launch_score_mfma_pruned(const ScoreModel &m, const uint16_t *codes, uint32_t n_flows, uint32_t d,
                              const uint32_t *meta, const uint16_t *nbins, int64_t *out, uint32_t *ws, hipStream_t s) {
    IG_REQUIRE(m.btile[0] && m.btile[1] && m.nbucket, IG_E_INVAL, "model tiles are not grouped by token");
    IG_REQUIRE(m.KO >= 1 && m.KO <= 8, IG_E_UNSUPPORTED, "the matrix-core scoring path handles up to 8 words");
    if (!n_flows) return true;
    const uint32_t L = m.nbucket, rt = IG_PRUNE_RT;
    // every unit count and the queue stay below 2^32
    const uint64_t tiles = (uint64_t)m.ftiles[0] + m.ftiles[1];
    const uint64_t bound = (tiles / rt + 2ull * L) * ((uint64_t)n_flows / SC_COLS + 1);
    if (bound >= (1ull << 31)) return false;
    PruneWork w = prune_work(ws, L, n_flows, d);
    IG_REQUIRE(((uintptr_t)w.ops & 15u) == 0, IG_E_INVAL, "scoring scratch must be 16-byte aligned");
    launch_prune_lists(codes, n_flows, d, meta, nbins, L, m.btile[0], m.btile[1], rt, SC_COLS, out, w, s);
    if (!tiles) return true;
    ScoreMfmaArgs a{};
    for (int c = 0; c < 2; ++c) {
        a.frag[c] = m.frag[c];
        a.ntiles[c] = m.ftiles[c];
    }
    a.codes = codes;
    a.meta = meta;
    a.nbins = nbins;
    a.out = out;
    a.n_flows = n_flows;
    a.d = d;
    a.fv = m.fv;
    PruneArgs p{};
    p.btile[0] = m.btile[0];
    p.btile[1] = m.btile[1];
    p.fcnt = w.cnt;
    p.foff = w.foff;
    p.flist = w.list;
    p.uoff = w.uoff;
    p.queue = w.queue;
    p.L = L;
    p.rt = rt;
    const void *kernels[8][3] = {
#define IG_SCP(V) {(const void *)k_score_mfma_pruned<V, SF_PLAIN>, (const void *)k_score_mfma_pruned<V, SF_SPARE>, \
                   (const void *)k_score_mfma_pruned<V, SF_TERN>},
        IG_SCP(1) IG_SCP(2) IG_SCP(3) IG_SCP(4) IG_SCP(5) IG_SCP(6) IG_SCP(7) IG_SCP(8)
#undef IG_SCP
    };
    const int form = score_form(m, a);
    const void *kern = kernels[m.KO - 1][form];
    const void *opk[8][3] = {
#define IG_FOP(V) {(const void *)k_flow_operands<V, SF_PLAIN>, (const void *)k_flow_operands<V, SF_SPARE>, \
                   (const void *)k_flow_operands<V, SF_TERN>},
        IG_FOP(1) IG_FOP(2) IG_FOP(3) IG_FOP(4) IG_FOP(5) IG_FOP(6) IG_FOP(7) IG_FOP(8)
#undef IG_FOP
    };
    {
        uint4 *ops = w.ops;
        void *oargs[] = {&a, &ops};
        IG_HIP(hipLaunchKernel(opk[m.KO - 1][form], dim3((unsigned)((2ull * n_flows + 255) / 256)), dim3(256), oargs,
                               0, s));
    }
    p.ops = w.ops;
    static std::atomic<uint32_t> slot_cache[8][3] = {};
    uint32_t slots = slot_cache[m.KO - 1][form].load(std::memory_order_relaxed);
    if (!slots) {
        slots = xcd_slots(kern, SC_NT);
        slot_cache[m.KO - 1][form].store(slots, std::memory_order_relaxed);
    }
    // a persistent grid: every resident workgroup drains the queue; no more
    // workgroups than units can exist
    uint64_t grid = 8ull * slots;
    if (grid > bound) grid = bound ? bound : 1;
    void *args[] = {&a, &p};
    IG_HIP(hipLaunchKernel(kern, dim3((unsigned)grid), dim3(SC_NT), args, 0, s));
    return true;
}

}  // namespace ig
