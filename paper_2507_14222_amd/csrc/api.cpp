// libig host runtime: the C ABI of include/ig.h.
//
// Fit pipeline (per fit, both classes in one pass where memory allows):
//   validate + class split + pack (Eq. 5, rows stacked by class)
//   pair space chunked -> (hash, pair id) per candidate (Eq. 1)
//   radix sort by (class, hash) -> exact de-duplication by full compare
//   coherence filter of the distinct candidates (Eq. 3 / Eq. 6)
//   canonical order of the coherent set (LSD radix sort on the words)
//   support and weight of each pattern (Eq. 2)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "common.h"
#include "kernels.h"
#include "../../include/ig_probe.h"

namespace ig {

static thread_local std::string g_last_error;

void set_error(const std::string &m) { g_last_error = m; }

// --------------------------------------------------------------- the model ----
struct DevModel {
    int device = 0;
    ig_allocator user{};                   // the caller allocator the buffers came from
    bool has_user = false;                 //   (else the library's arena)
    uint32_t K = 0, KS = 0, L = 0, d = 0;
    uint64_t np[2] = {0, 0};
    uint64_t *W[2] = {nullptr, nullptr};
    uint32_t *f[2] = {nullptr, nullptr};
    int64_t *S[2] = {nullptr, nullptr};
    int64_t maxS[2] = {0, 0};
    uint32_t *meta = nullptr;    // off[d] | flo[KS] | fhi[KS]
    uint16_t *nbins = nullptr;
    uint4 *frag[2] = {nullptr, nullptr};   // matrix-core scoring operands (KS <= 8)
    uint32_t ftiles[2] = {0, 0};           // 32-row tiles of frag
    uint32_t *btile[2] = {nullptr, nullptr};   // [L + 1] first tile of each token bucket (fits from codes)
    uint32_t *brow[2] = {nullptr, nullptr};    // [L + 1] first position of each bucket in bperm
    uint32_t *bperm[2] = {nullptr, nullptr};   // [np] rows of the class grouped by bucket
    KeyPiece *pieces = nullptr;            // compressed sort keys (fits from codes), or null
    uint32_t npieces = 0, nkeys = 0;
    void *fac = nullptr;                   // factored-token table (one device block)
    FactorView fv;                         // fv.KF = 0: matrix-core operands stay one-hot
    void *tfac = nullptr;                  // the ternary (bit tokens only) table
    FactorView tv;                         // of the coherence and support contractions
    uint32_t fac_tokens = 0;               // tokens of the factored form
    uint32_t fac_tokens_last = 0;          // of them, in its last word
    uint32_t tern_tokens = 0;              // tokens of the ternary form
    uint32_t fit_tokens = 0, fit_words = 0;    // operand rows of the fit's contractions
    bool fit_buckets = false;              // the fit's contractions used token buckets
    bool score_factored = false;           // frag holds factored operand rows
    bool score_ternary = false;            // ... of the ternary view (tv)
    bool score_spare = false;              // frag carries the +1 at the spare last token
    int score_pref = -1;                   // scoring view: -1 automatic, 0 presence tokens, 1 ternary
    // [L + 2] first pattern of each bucket when the fit grouped class c's patterns
    // by token bucket (empty otherwise)
    std::vector<uint32_t> sgroup[2];
    ig_stats stats{};


    void release(void *p) const noexcept { device_free(p, device, has_user ? &user : nullptr); }

    ~DevModel() {
        for (int c = 0; c < 2; ++c) {
            release(W[c]);
            release(f[c]);
            release(S[c]);
            release(frag[c]);
            release(btile[c]);
            release(brow[c]);
            release(bperm[c]);
        }
        release(meta);
        release(nbins);
        release(pieces);
        release(fac);
        release(tfac);
    }
};

// A model buffer of `count` T, from the allocator of the running call (the caller's,
// or the library's arena); DevModel::release hands it back.
template <class T>
static T *dev_alloc(size_t count) {
    return static_cast<T *>(device_alloc((count ? count : 1) * sizeof(T), nullptr, current_user_allocator()));
}

// Token layout tables for codes with the given bins: off[f], and per storage
// word k the features [flo[k], fhi[k]) whose token ranges meet word k.
static std::vector<uint32_t> token_tables(const uint16_t *nbins, uint32_t d, uint32_t KS) {
    std::vector<uint32_t> t(d + 2 * KS, 0);
    uint32_t acc = 0;
    for (uint32_t f = 0; f < d; ++f) {
        t[f] = acc;
        acc += nbins[f];
    }
    for (uint32_t k = 0; k < KS; ++k) {
        uint32_t lo = 64 * k, hi = 64 * (k + 1);
        uint32_t flo = d, fhi = 0;
        for (uint32_t f = 0; f < d; ++f) {
            uint32_t a = t[f], b = t[f] + nbins[f];
            if (a < hi && b > lo) {
                flo = std::min(flo, f);
                fhi = std::max(fhi, f + 1);
            }
        }
        if (flo >= fhi) flo = fhi = 0;
        t[d + k] = flo;
        t[d + KS + k] = fhi;
    }
    return t;
}

// Pieces of the compressed sort keys (see KeyPiece): every (feature, word) overlap,
// most significant first -- words ascending, higher bits first within a word --
// each taking ceil(log2(width + 1)) key bits; a piece never straddles key words.
// Returns the number of key words, or 0 when compression would not save a word.
static uint32_t key_pieces(const uint16_t *nbins, uint32_t d, uint32_t K, std::vector<KeyPiece> &out) {
    out.clear();
    uint32_t off = 0;
    for (uint32_t f = 0; f < d; ++f) {
        const uint32_t a = off, b = off + nbins[f];
        for (uint32_t t = a; t < b;) {
            const uint32_t w = t / 64, hi = std::min(b, 64 * (w + 1));
            KeyPiece p{};
            p.word = (uint8_t)w;
            p.lo = (uint8_t)(t % 64);
            p.width = (uint8_t)(hi - t);
            out.push_back(p);
            t = hi;
        }
        off = b;
    }
    std::sort(out.begin(), out.end(), [](const KeyPiece &x, const KeyPiece &y) {
        return x.word != y.word ? x.word < y.word : x.lo > y.lo;
    });
    uint32_t kw = 0, used = 0;
    for (KeyPiece &p : out) {
        const uint32_t cb = 32 - __builtin_clz((uint32_t)p.width);   // codes 0..width
        if (used + cb > 64) { ++kw; used = 0; }
        p.kw = (uint8_t)kw;
        p.shift = (uint8_t)(64 - used - cb);
        used += cb;
    }
    const uint32_t nk = out.empty() ? 0 : kw + 1;
    return nk < K ? nk : 0;
}

static void set_key_pieces(DevModel &m, const uint16_t *h_nbins, uint32_t d, hipStream_t s) {
    std::vector<KeyPiece> pc;
    const uint32_t nk = key_pieces(h_nbins, d, m.K, pc);
    if (!nk) return;
    m.pieces = dev_alloc<KeyPiece>(pc.size());
    upload(m.pieces, pc.data(), pc.size() * sizeof(KeyPiece), s);
    m.npieces = (uint32_t)pc.size();
    m.nkeys = nk;
}

// Signed-bit tokens of a feature with nb bins (nb >= 2): m = ceil(log2 nb) tokens
// for the bits of the bin index and p presence tokens, p = 1 when m <= 4 and 2 when
// 5 <= m <= 10.  The record side carries the popcount of its bin index on them, in
// parts that e2m1 holds exactly: the first min(popcount, 4), or 6 when the popcount
// is 6 or more, the second what is left (at most 4).  Returns m + p with *bits = m;
// 0 for one bin; ~0 beyond 1024 bins.
static uint32_t feature_tokens(uint32_t nb, uint32_t *bits) {
    uint32_t mb = 0;
    while ((1u << mb) < nb) ++mb;
    *bits = mb;
    if (mb == 0) return 0;
    if (mb > 10) return ~0u;
    return mb + (mb <= 4 ? 1u : 2u);
}

// Factored-token table of a fit from codes (see FactorView), used when it needs at
// most 16 words and fewer words than the one-hot packing.  A pattern (or candidate)
// sets, for each feature it holds, the bits of the bin index and the presence
// tokens; the other side (a record, or a flow in scoring) holds every feature and
// carries +1 on a bit token whose bit is 0, -1 where it is 1, and the popcount of
// its bin index on the presence tokens.  Their product summed over a feature's
// tokens is the number of bits in which the two bin indices differ (0 when the
// pattern lacks the feature), so the contraction is zero exactly when the pattern
// lies inside (Eq. 6).  Tokens are laid out feature after feature; a feature may
// cross a word boundary, so its tokens touch at most two words.
//
// ternary: the table of the bit tokens alone (no presence tokens), for the
// contractions of the fit (see FactorView::ternary); stored in m.tv / m.tfac.
static void set_factor_table(DevModel &m, const uint16_t *h_nbins, uint32_t d, hipStream_t s, bool ternary = false) {
    std::vector<FacFeature> feat(d);
    std::vector<uint64_t> mask;
    std::vector<uint64_t> fbit(2 * (size_t)d, 0);   // bit tokens of each feature, words w0 and w0 + 1
    std::vector<uint32_t> tokdesc;                  // per token: kind | bit index << 8 | feature << 16
    std::vector<uint64_t> bitw(16, 0);              // bit tokens per word
    std::vector<uint32_t> ptok(d, ~0u);             // first presence token | count << 24
    uint32_t off = 0, tokens = 0, used = 0, word = 0;
    for (uint32_t f = 0; f < d; ++f) {
        const uint32_t nb = h_nbins[f];
        uint32_t mb = 0;
        uint32_t nt = feature_tokens(nb, &mb);
        if (nt == ~0u) return;   // a feature beyond 1024 bins: stay one-hot
        if (ternary) nt = mb;
        if (f >= (1u << 16)) return;
        FacFeature ft{};
        ft.off = (uint16_t)off;
        ft.nb = (uint16_t)nb;
        ft.mask = (uint32_t)mask.size();
        if (nt) {
            const uint32_t t0 = tokens, t1 = tokens + nt;   // tokens [t0, t1)
            if ((t1 - 1) / 64 >= 16) return;                 // more than 16 words
            ft.w0 = (uint8_t)(t0 / 64);
            ft.nw = (uint8_t)((t1 - 1) / 64 - t0 / 64 + 1);
            for (uint32_t t = t0; t < t1; ++t) {
                const uint32_t k = t - t0;
                const uint32_t desc = k < mb ? (1u | k << 8) : (k == mb ? 2u : 3u);
                tokdesc.push_back(desc | f << 16);
                if (k < mb) {
                    fbit[2 * f + (t / 64 - ft.w0)] |= 1ull << (t % 64);
                    bitw[t / 64] |= 1ull << (t % 64);
                }
            }
            if (!ternary) ptok[f] = (t0 + mb) | (nt - mb) << 24;
            for (uint32_t c = 0; c < nb; ++c) {
                uint64_t part[2] = {0, 0};
                for (uint32_t t = t0; t < t1; ++t) {
                    const uint32_t k = t - t0;
                    if (k >= mb || ((c >> k) & 1u)) part[t / 64 - ft.w0] |= 1ull << (t % 64);
                }
                for (uint32_t w = 0; w < ft.nw; ++w) mask.push_back(part[w]);
            }
            tokens = t1;
            word = (t1 - 1) / 64;
            used = t1 - 64 * word;
        }
        feat[f] = ft;
        off += nb;
    }
    // a ternary view keeps the top tokens of its last word for the bias slots
    const uint32_t KF = !tokens ? 0 : ternary ? (tokens + tern_bias_slots(tokens) + 63) / 64 : word + 1;
    if (KF == 0 || KF >= m.K || KF > 16) return;
    // pieces: each feature cut at one-hot word boundaries
    std::vector<std::vector<FacPiece>> by_word(m.K);
    for (uint32_t f = 0; f < d; ++f) {
        const FacFeature &ft = feat[f];
        if (!ft.nw) continue;
        for (uint32_t t = ft.off; t < (uint32_t)ft.off + ft.nb;) {
            const uint32_t w = t / 64, hi = std::min<uint32_t>(ft.off + ft.nb, 64 * (w + 1));
            FacPiece p{};
            p.lo = (uint8_t)(t % 64);
            p.width = (uint8_t)(hi - t);
            p.w0 = ft.w0;
            p.nw = ft.nw;
            p.base = (uint16_t)(t - ft.off);
            p.mask = ft.mask;
            p.pad2 = f;   // the feature (ternary views read its tokens, fbit, as P)
            by_word[w].push_back(p);
            t = hi;
        }
    }
    // one range per storage word (KS >= K): the kernels walk every word they hold,
    // and the padding words K .. KS - 1 have no pieces
    std::vector<FacPiece> piece;
    std::vector<uint32_t> pbeg(m.KS + 1, 0);
    for (uint32_t w = 0; w < m.KS; ++w) {
        pbeg[w] = (uint32_t)piece.size();
        if (w < m.K) piece.insert(piece.end(), by_word[w].begin(), by_word[w].end());
    }
    pbeg[m.KS] = (uint32_t)piece.size();
    std::vector<uint32_t> fbeg(KF + 1, d), fend(KF + 1, 0);
    for (uint32_t f = 0; f < d; ++f)
        for (uint32_t w = feat[f].w0; w < (uint32_t)feat[f].w0 + feat[f].nw; ++w) {
            fbeg[w] = std::min(fbeg[w], f);
            fend[w] = std::max(fend[w], f + 1);
        }
    for (uint32_t w = 0; w <= KF; ++w)
        if (fbeg[w] >= fend[w]) fbeg[w] = fend[w] = 0;
    // token ranges per output word (rows of record pairs): every bin's tokens
    // of a feature, one entry per word it touches; a feature on two words gets the
    // next bit of the spanning mask
    std::vector<std::vector<uint32_t>> wq(KF);   // 4 dwords per entry
    uint32_t nspan = 0;
    for (uint32_t f = 0; f < d; ++f) {
        const FacFeature &ft = feat[f];
        if (!ft.nw) continue;
        const uint32_t bit = ft.nw > 1 ? nspan++ : 0u;
        for (uint32_t k = 0; k < ft.nw; ++k) {
            uint64_t rg = 0;
            for (uint32_t c = 0; c < ft.nb; ++c) rg |= mask[ft.mask + c * ft.nw + k];
            wq[ft.w0 + k].insert(wq[ft.w0 + k].end(),
                                 {bit, ft.nw > 1 ? 1u : 0u, (uint32_t)rg, (uint32_t)(rg >> 32)});
        }
    }
    if (nspan > 32) return;   // cannot happen: a spanning feature per word boundary, KF <= 16
    std::vector<uint32_t> wfe, wbeg(KF + 1, 0);
    for (uint32_t w = 0; w < KF; ++w) {
        wbeg[w] = (uint32_t)(wfe.size() / 4);
        wfe.insert(wfe.end(), wq[w].begin(), wq[w].end());
    }
    wbeg[KF] = (uint32_t)(wfe.size() / 4);
    // one device block: range entries | masks | features | pieces | fbeg | fend | pbeg | wbeg
    // (16-byte aligned parts; the entries and pieces are read as 16-byte scalar loads)
    tokdesc.resize((size_t)KF * 64, 0u);   // tokens past the last feature: kind 0
    bitw.resize(KF);
    auto al16 = [](size_t b) { return (b + 15) / 16 * 16; };
    const size_t eb = al16(wfe.size() * 4), mb = al16(mask.size() * 8),
                 fb = al16(feat.size() * sizeof(FacFeature)), pb = al16(piece.size() * sizeof(FacPiece)),
                 ib = al16((KF + 1) * 4), kb = al16((m.KS + 1) * 4), tb = al16(tokdesc.size() * 4),
                 bb = al16(fbit.size() * 8), wb = al16(bitw.size() * 8), qb = al16(ptok.size() * 4);
    std::vector<char> host(eb + mb + fb + pb + 3 * ib + kb + tb + bb + wb + qb, 0);
    size_t at = 0;
    auto put = [&](const void *src, size_t bytes, size_t span) {
        std::memcpy(host.data() + at, src, bytes);
        const size_t here = at;
        at += span;
        return here;
    };
    const size_t o_wfe = put(wfe.data(), wfe.size() * 4, eb);
    const size_t o_mask = put(mask.data(), mask.size() * 8, mb);
    const size_t o_feat = put(feat.data(), feat.size() * sizeof(FacFeature), fb);
    const size_t o_piece = put(piece.data(), piece.size() * sizeof(FacPiece), pb);
    const size_t o_fbeg = put(fbeg.data(), (KF + 1) * 4, ib);
    const size_t o_fend = put(fend.data(), (KF + 1) * 4, ib);
    const size_t o_pbeg = put(pbeg.data(), (m.KS + 1) * 4, kb);
    const size_t o_wbeg = put(wbeg.data(), (KF + 1) * 4, ib);
    const size_t o_tok = put(tokdesc.data(), tokdesc.size() * 4, tb);
    const size_t o_fbit = put(fbit.data(), fbit.size() * 8, bb);
    const size_t o_bitw = put(bitw.data(), bitw.size() * 8, wb);
    const size_t o_ptok = put(ptok.data(), ptok.size() * 4, qb);
    char *dev = dev_alloc<char>(host.size());
    (ternary ? m.tfac : m.fac) = dev;
    upload(dev, host.data(), host.size(), s);
    FactorView &v = ternary ? m.tv : m.fv;
    v.mask = reinterpret_cast<const uint64_t *>(dev + o_mask);
    v.feat = reinterpret_cast<const FacFeature *>(dev + o_feat);
    v.piece = reinterpret_cast<const FacPiece *>(dev + o_piece);
    v.fbeg = reinterpret_cast<const uint32_t *>(dev + o_fbeg);
    v.fend = reinterpret_cast<const uint32_t *>(dev + o_fend);
    v.pbeg = reinterpret_cast<const uint32_t *>(dev + o_pbeg);
    v.wfe = reinterpret_cast<const uint4 *>(dev + o_wfe);
    v.wbeg = reinterpret_cast<const uint32_t *>(dev + o_wbeg);
    v.tok = reinterpret_cast<const uint32_t *>(dev + o_tok);
    v.fbit = reinterpret_cast<const uint64_t *>(dev + o_fbit);
    v.bitw = reinterpret_cast<const uint64_t *>(dev + o_bitw);
    v.ptok = reinterpret_cast<const uint32_t *>(dev + o_ptok);
    v.d = d;
    v.KF = KF;
    v.nmask = (uint32_t)mask.size();
    v.npiece = (uint32_t)piece.size();
    v.nwords = m.KS;
    v.ternary = ternary ? 1u : 0u;
    if (!ternary) {
        m.fac_tokens_last = used;
        m.fac_tokens = tokens;
    } else {
        m.tern_tokens = tokens;
    }
}

// The view of the scoring operands: that of the fit's contractions when they used
// factored tokens (ternary or with presence tokens), else the ternary bit tokens
// when they take fewer words than the presence tokens, else the presence tokens
// (fv.KF = 0: the one-hot words).  Ternary views of more than 8 words give way.
static const FactorView &score_view(const DevModel &m) {
    const bool tern = m.tv.KF && m.tv.KF <= 8 &&
                      (m.score_pref == 1 || (m.score_pref < 0 && (!m.fv.KF || m.tv.KF < m.fv.KF)));
    return tern ? m.tv : m.fv;
}

static void check_nbins(const uint16_t *h_nbins, uint32_t d, uint32_t &L, uint32_t &K) {
    IG_REQUIRE(d >= 1 && d <= 4096, IG_E_INVAL, "d must be in 1..4096");
    IG_REQUIRE(h_nbins != nullptr, IG_E_INVAL, "nbins is NULL");
    uint64_t s = 0;
    for (uint32_t f = 0; f < d; ++f) {
        IG_REQUIRE(h_nbins[f] >= 1 && h_nbins[f] < IG_ABSENT, IG_E_INVAL,
                   "nbins[" + std::to_string(f) + "] must be in 1..65534");
        s += h_nbins[f];
    }
    IG_REQUIRE(s <= 4096, IG_E_UNSUPPORTED, "token universe L = " + std::to_string(s) + " exceeds 4096");
    L = (uint32_t)s;
    K = (L + 63) / 64;
}

// n words from the device after the work queued on s (a copy that returns when it
// is done, so the stream has reached it: no separate synchronisation)
static std::vector<uint32_t> host_read_u32(const uint32_t *d, size_t n, hipStream_t s) {
    std::vector<uint32_t> h(n);
    if (n) IG_HIP(hipMemcpyWithStream(h.data(), d, n * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    else IG_HIP(hipStreamSynchronize(s));
    return h;
}

// ----------------------------------------------------------- fit from rows ----
struct Timer {
    hipEvent_t ev[9] = {};
    bool marked[9] = {};
    bool on = false;
    hipStream_t s;
    explicit Timer(hipStream_t st) : s(st) {
        on = true;
        for (auto &e : ev)
            if (hipEventCreate(&e) != hipSuccess) on = false;
        (void)hipGetLastError();
    }
    void mark(int i) {
        if (on && hipEventRecord(ev[i], s) == hipSuccess) marked[i] = true;
    }
    // milliseconds between two recorded events (false when either was not recorded)
    bool elapsed(int a, int b, float &ms) const {
        if (!on || !marked[a] || !marked[b]) return false;
        return hipEventElapsedTime(&ms, ev[a], ev[b]) == hipSuccess;
    }
    ~Timer() {
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

struct Tuning {
    int cpl = 1;               // coherence: candidates per lane (one measured fastest at 15k)
    uint32_t grid_per_cu = 8;  // coherence: persistent workgroups per CU
    int support_cpl = 2;       // support: patterns per lane
    int coh_sets = 0;          // matrix-core coherence: column sets per wave (0: default)
    int sup_sets = 0;          // matrix-core support: the same
};

// Launch shape for a problem stored with KS words and `pairs` same-class pairs:
// the matching row of the tuning table with the largest min_pairs (an exact KS
// match beats ks = 0), then the explicit filter_cpl override.
static Tuning tuning_for(const ig_fit_opts *o, uint32_t KS, uint64_t pairs) {
    Tuning t;
    if (o && o->tune && o->n_tune) {
        const ig_tune_entry *best = nullptr;
        for (uint32_t i = 0; i < o->n_tune; ++i) {
            const ig_tune_entry &e = o->tune[i];
            if (e.mfma_words || (e.ks != 0 && e.ks != KS) || e.min_pairs > pairs) continue;
            if (!best || (best->ks == 0 && e.ks != 0) ||
                ((best->ks != 0) == (e.ks != 0) && e.min_pairs > best->min_pairs))
                best = &e;
        }
        if (best) {
            if (best->filter_cpl == 1 || best->filter_cpl == 2) t.cpl = (int)best->filter_cpl;
            if (best->grid_per_cu >= 1 && best->grid_per_cu <= 32) t.grid_per_cu = best->grid_per_cu;
            if (best->support_cpl == 1 || best->support_cpl == 2) t.support_cpl = (int)best->support_cpl;
        }
    }
    if (o && (o->filter_cpl == 1 || o->filter_cpl == 2)) t.cpl = (int)o->filter_cpl;
    return t;
}

// The matrix-core contractions' shape for operands of KO words: the matching
// mfma_words row with the largest min_pairs not above `pairs`.
static void mfma_tuning(const ig_fit_opts *o, uint32_t KO, uint64_t pairs, Tuning &t) {
    if (!o || !o->tune || !o->n_tune) return;
    const ig_tune_entry *best = nullptr;
    for (uint32_t i = 0; i < o->n_tune; ++i) {
        const ig_tune_entry &e = o->tune[i];
        if (e.mfma_words != KO || e.min_pairs > pairs) continue;
        if (!best || e.min_pairs > best->min_pairs) best = &e;
    }
    if (!best) return;
    if (best->coherence_sets >= 1 && best->coherence_sets <= 3) t.coh_sets = (int)best->coherence_sets;
    if (best->support_sets >= 1 && best->support_sets <= 3) t.sup_sets = (int)best->support_sets;
}

struct ClassRows {
    Scratch<uint64_t> X, NX;
    uint32_t n = 0;
};

// Operand rows of a model's patterns (in the model's own token view), kept from the
// support step so that the scoring operands need not build them again.
struct PatternRows {
    Scratch<uint64_t> rows[2];
    bool valid[2] = {false, false};
};


// Canonical order (ascending w_0 .. w_{K-1}, unsigned, w_0 most significant) of
// `count` patterns: the pair ids `ids` into the class rows X [n][KS], or, with ids
// null, the rows X [count][KS] themselves.  Writes the sorting permutation to perm
// (perm[e] = index of the e-th pattern in order).  LSD radix sort of a permutation,
// on compressed keys when the model has them (fits from codes), else on the words.
static void canonical_permutation(const DevModel &m, const uint64_t *X, uint32_t n, const uint32_t *ids,
                                  size_t count, uint32_t *perm, hipStream_t s) {
    const uint32_t KS = m.KS, K = m.K;
    launch_iota(perm, count, s);
    if (count <= 1) return;
    auto byte_mask = [](unsigned long long orv, unsigned long long andv) {
        const uint64_t vary = orv ^ andv;   // bits that differ somewhere
        uint32_t mask = 0;
        for (int b = 0; b < 8; ++b)
            if ((vary >> (8 * b)) & 0xffull) mask |= 1u << b;
        return mask;
    };
    // key words (nk arrays of `count`), least significant first in the sort
    const uint32_t nk = m.pieces ? m.nkeys : K;
    Scratch<uint64_t> keys((size_t)nk * count, s);
    if (m.pieces) {
        launch_compress_keys(X, n, KS, ids, count, m.pieces, m.npieces, keys.get(), s);
    } else {
        Scratch<uint32_t> iota(count, s);
        launch_iota(iota.get(), count, s);
        for (uint32_t k = 0; k < K; ++k) {
            if (ids) launch_gather_word(X, n, KS, k, ids, count, keys.get() + (size_t)k * count, s);
            else launch_row_word(X, iota.get(), count, KS, k, keys.get() + (size_t)k * count, s);
        }
    }
    Scratch<unsigned long long> rng(2 * nk, s);
    launch_fill_u64(reinterpret_cast<uint64_t *>(rng.get()), 0ull, nk, s);
    launch_fill_u64(reinterpret_cast<uint64_t *>(rng.get() + nk), ~0ull, nk, s);
    launch_key_range(keys.get(), nk, count, rng.get(), rng.get() + nk, s);
    std::vector<unsigned long long> hr(2 * nk);
    IG_HIP(hipMemcpyAsync(hr.data(), rng.get(), 2 * nk * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    IG_HIP(hipStreamSynchronize(s));
    Scratch<uint32_t> palt(count, s);
    Scratch<uint64_t> k0(count, s), k1(count, s);
    uint32_t *pcur = perm, *pnext = palt.get();
    bool identity = true;   // pcur is still the identity permutation
    for (int k = (int)nk - 1; k >= 0; --k) {
        const uint32_t mask = byte_mask(hr[k], hr[nk + k]);
        if (!mask) continue;
        uint64_t *kin = keys.get() + (size_t)k * count;   // consumed: the sort may overwrite it
        if (!identity) {
            launch_permute_u64(kin, pcur, count, k0.get(), s);
            kin = k0.get();
        }
        const int where = radix_sort_pairs(kin, pcur, k1.get(), pnext, count, mask, s);
        if (where) std::swap(pcur, pnext);
        identity = false;
    }
    if (pcur != perm) IG_HIP(hipMemcpyAsync(perm, pcur, count * 4, hipMemcpyDeviceToDevice, s));
}

// Device times of launches, from event pairs read once the stream has passed
// them (collect), instead of a synchronisation per launch; host tables whose
// asynchronous copies precede those launches are kept until then.
struct KernelClock {
    struct Item {
        hipEvent_t a = nullptr, b = nullptr;
        float *to = nullptr;
    };
    std::deque<Item> items;   // references to items stay valid as more are opened
    std::vector<std::vector<uint32_t>> keep;
    Item &open(hipStream_t s, float *to) {
        items.emplace_back();
        Item &it = items.back();
        it.to = to;
        IG_HIP(hipEventCreate(&it.a));
        IG_HIP(hipEventCreate(&it.b));
        IG_HIP(hipEventRecord(it.a, s));
        return it;
    }
    void close(Item &it, hipStream_t s) { IG_HIP(hipEventRecord(it.b, s)); }
    void collect() {
        for (Item &it : items) {
            float ms = 0;
            if (hipEventSynchronize(it.b) == hipSuccess && hipEventElapsedTime(&ms, it.a, it.b) == hipSuccess &&
                it.to)
                *it.to += ms;
        }
        release();
    }
    void release() {
        for (Item &it : items) {
            if (it.a) (void)hipEventDestroy(it.a);
            if (it.b) (void)hipEventDestroy(it.b);
        }
        items.clear();
        keep.clear();
    }
    ~KernelClock() { release(); }
};

// The records of one class listed under each token they hold, with bucket L
// holding every record: the A tiles of the pruned contractions
// (k_contain_mfma_pruned).  A candidate's bucket is its token held by the fewest
// of these records (the lowest such token on ties): the token of lowest rank.
struct FitBuckets {
    std::vector<uint32_t> cnt;     // [L + 1] records per bucket (host copy)
    Scratch<uint16_t> rank;        // [L] rank of each token, then [L] the token of each rank
    Scratch<uint32_t> tab;         // [L + 2] tile starts bt, then [L + 1] records brec
    Scratch<uint4> frag;
    const uint16_t *inv() const { return rank.get() + cnt.size() - 1; }
};

struct MfmaFit {
    bool on = false;
    FactorView view;
    uint32_t KO = 0;
    uint32_t RW = 0;           // words per operand row: 2 KO for a ternary view
    Scratch<uint4> frag[2];
    Scratch<uint64_t> fr[2];   // factored rows of each class's records (factored view only)
    bool pruned = false;       // token buckets: bk[t] lists class t's records
    uint32_t L = 0, KSr = 0;
    FitBuckets bk[2];
    // class c's records with their tokens renumbered by the ranks of the coherence
    // (bk[1 - c]) and the support (bk[c]) buckets
    Scratch<uint64_t> xr_coh[2], xr_sup[2];
    KernelClock clock;         // device times of the pruned contractions
    // pairs the pruned contractions examined: coherence of class 0, 1, support of 0, 1
    Scratch<unsigned long long> dtests;
    unsigned long long htests[4] = {};
    // waits for the stream: copies dtests to htests when pruned (a copy that
    // returns when the stream has reached it), else synchronises
    void finish(hipStream_t s) {
        if (pruned) IG_HIP(hipMemcpyWithStream(htests, dtests.get(), sizeof(htests), hipMemcpyDeviceToHost, s));
        else IG_HIP(hipStreamSynchronize(s));
    }
    void put_tests(DevModel &m) const {
        if (!pruned) return;
        for (int c = 0; c < 2; ++c) {
            m.stats.tests[c] = htests[c];
            m.stats.support_tests[c] = htests[2 + c];
        }
    }
};

// Token buckets of both classes' records for the pruned contractions (ternary
// view), with one host round trip for both.
static void build_fit_buckets(const DevModel &m, const ClassRows cls[2], MfmaFit &mf, hipStream_t s) {
    const uint32_t L = m.L, d = m.d;
    Scratch<uint32_t> key[2], list[2], first(2 * ((size_t)L + 2), s);
    for (int t = 0; t < 2; ++t) {
        const uint32_t n = cls[t].n;
        const size_t nd = (size_t)n * d;
        key[t].reset(std::max<size_t>(nd, 1), s);
        list[t].reset(nd + n + 1, s);
        Scratch<uint32_t> ws(bucket_ws_words(nd, L), s);
        launch_group_records(cls[t].X.get(), n, m.KS, L, d, key[t].get(), list[t].get(), first.get() + t * (L + 2),
                             ws.get(), s);
        if (n) launch_iota(list[t].get() + nd, n, s);   // bucket L: every record
    }
    const std::vector<uint32_t> hf = host_read_u32(first.get(), 2 * ((size_t)L + 2), s);
    // per class: ranks and their tokens (u16 pairs), then list offsets ro [L + 2],
    // tile starts bt [L + 2] and records brec [L + 1]
    const size_t per = (size_t)L + (3 * (size_t)L + 5);
    std::vector<uint32_t> up(2 * per, 0);
    uint32_t ntiles[2];
    for (int t = 0; t < 2; ++t) {
        FitBuckets &b = mf.bk[t];
        const uint32_t *h = hf.data() + t * (L + 2);
        const uint32_t n = cls[t].n;
        const size_t nd = (size_t)n * d;
        // ranks: tokens by ascending records holding them, then token
        std::vector<uint32_t> order(L);
        for (uint32_t u = 0; u < L; ++u) order[u] = u;
        std::stable_sort(order.begin(), order.end(),
                         [&](uint32_t x, uint32_t y) { return h[x + 1] - h[x] < h[y + 1] - h[y]; });
        uint16_t *rank = reinterpret_cast<uint16_t *>(up.data() + t * per);
        for (uint32_t r = 0; r < L; ++r) {
            rank[order[r]] = (uint16_t)r;
            rank[L + r] = (uint16_t)order[r];
        }
        uint32_t *ro = up.data() + t * per + L, *bt = ro + L + 2, *brec = bt + L + 2;
        b.cnt.assign(L + 1, 0);
        for (uint32_t u = 0; u < L; ++u) {
            b.cnt[u] = h[u + 1] - h[u];
            ro[u] = h[u];
        }
        b.cnt[L] = n;
        ro[L] = (uint32_t)nd;
        for (uint32_t u = 0; u <= L; ++u) {
            bt[u + 1] = bt[u] + (b.cnt[u] + 31) / 32;
            brec[u] = b.cnt[u];
        }
        ntiles[t] = bt[L + 1];
    }
    Scratch<uint32_t> dup(up.size(), s);
    upload(dup.get(), up.data(), up.size() * 4, s);
    for (int t = 0; t < 2; ++t) {
        FitBuckets &b = mf.bk[t];
        const uint32_t *base = dup.get() + t * per;
        const uint32_t *hbase = up.data() + t * per;
        b.rank.reset(2 * (size_t)L, s);
        b.tab.reset(2 * (size_t)L + 3, s);
        // from the host tables through the staging ring (a device-to-device copy
        // here cost as much host time as a synchronisation)
        upload(b.rank.get(), hbase, 2 * (size_t)L * 2, s);
        upload(b.tab.get(), hbase + L + L + 2, (2 * (size_t)L + 3) * 4, s);
        b.frag.reset(std::max<size_t>((size_t)ntiles[t] * mf.KO * 64, 1), s);
        launch_mfma_records_ternary_lists(mf.fr[t].get(), mf.KO, m.tern_tokens, list[t].get(), base + L, b.tab.get(),
                                          b.tab.get() + L + 2, L + 1, ntiles[t], b.frag.get(), s);
    }
    mf.clock.keep.push_back(std::move(up));   // until its copy has run
}

// Candidates grouped by bucket (see launch_group_candidates): perm and first on
// the device (first [L + 2]: bucket starts).
struct CandGroups {
    Scratch<uint32_t> perm, first;
};

// Groups m candidates (pair ids `ids` of the records Xr [n][KSr], renumbered by the
// ranks of the buckets b, or rows W [m][KS] of one-hot words when ids is null) by
// bucket.
// need_perm: also the permutation (position -> candidate); without it only the
// grouped ids (ids_out) and the bucket starts.
static void group_candidates(const MfmaFit &mf, const FitBuckets &b, const uint64_t *Xr, uint32_t n, uint32_t KS,
                             const uint32_t *ids, const uint64_t *W, size_t m, CandGroups &g, hipStream_t s,
                             uint32_t *ids_out = nullptr, bool need_perm = true) {
    IG_REQUIRE(m < (1ull << 32), IG_E_UNSUPPORTED, "more than 2^32 candidates in one contraction");
    IG_REQUIRE(need_perm || ids_out, IG_E_INVAL, "grouping with neither a permutation nor grouped ids");
    const uint32_t L = mf.L;
    Scratch<uint32_t> key(std::max<size_t>(m, 1), s), ws(bucket_ws_words(m, L), s);
    if (need_perm) g.perm.reset(std::max<size_t>(m, 1), s);
    g.first.reset(L + 2, s);
    launch_group_candidates(Xr, n, mf.KSr, ids, W, KS, m, L, b.rank.get(), b.inv(), key.get(), g.perm.get(),
                            g.first.get(), ws.get(), s, ids_out);
}

// The m grouped candidates (perm: position -> row of B and of out, null for the
// identity; first: bucket starts on the device) whose operand rows are B, tested on
// the matrix cores against the records of their buckets in b only: out[e] as
// launch_contain_mfma's (coherence flags, or support counts).  The work units are
// counted on the device (no host round trip); the (candidate, record) pairs tested
// are added to *tests (device), the contraction's device time to *kernel_ms.
static void pruned_contain(MfmaFit &mf, const FitBuckets &b, const uint32_t *perm, const uint32_t *first, size_t m,
                           const uint64_t *B, bool count, uint32_t *out, int sets, unsigned long long *tests,
                           float *kernel_ms, hipStream_t s, bool by_position = false) {
    // the support count takes 8 per record lacking a candidate in 32 bits
    IG_REQUIRE(b.cnt.back() < (1u << 28), IG_E_UNSUPPORTED, "more than 2^28 records in one class");
    if (!m) return;
    const uint32_t L = mf.L;
    const uint32_t cols = contain_pruned_cols((int)mf.KO, sets);
    // units: at most ceil(count_u / cols) <= count_u / cols + 1 per bucket
    const uint64_t bound = (m + cols - 1) / cols + L + 1;
    IG_REQUIRE(bound < (1ull << 31), IG_E_UNSUPPORTED, "too many work units in one contraction");
    Scratch<uint32_t> uo(L + 2, s);
    Scratch<uint4> desc(2 * bound, s);
    launch_contain_plan(first, b.tab.get() + L + 2, L + 1, cols, uo.get(), tests, s, b.tab.get(), (uint32_t)bound,
                        desc.get());
    ContainBuckets k{};
    k.perm = perm;
    k.desc = desc.get();
    k.by_position = by_position;
    KernelClock::Item &it = mf.clock.open(s, kernel_ms);
    launch_contain_mfma_pruned((int)mf.KO, count, B, b.frag.get(), k, (uint32_t)bound, out, s, sets);
    mf.clock.close(it, s);
}

// Rows of the coherent pair ids `ids` of one class (in the order given; in
// canonical order first when the pair space was chunked, which merges the repeats
// across chunks), then support and weights.  Fills model class c.
static void order_and_weigh(DevModel &m, int c, const ClassRows &cls, uint32_t *ids, size_t count,
                            bool may_repeat, const Tuning &tu, hipStream_t s, Timer *tm = nullptr,
                            int support_mark = -1, const uint4 *own_frag = nullptr,
                            const FactorView &mfma_view = FactorView{}, PatternRows *keep = nullptr,
                            Scratch<uint64_t> *pre_rows = nullptr, MfmaFit *pmf = nullptr,
                            const uint32_t *pre_idx = nullptr) {
    const uint32_t KS = m.KS;
    if (count == 0) {
        m.np[c] = 0;
        m.W[c] = dev_alloc<uint64_t>(KS);
        m.f[c] = dev_alloc<uint32_t>(1);
        m.S[c] = dev_alloc<int64_t>(1);
        return;
    }
    Scratch<uint32_t> sorted_ids;
    uint32_t *vcur = ids;
    // token buckets: the patterns grouped by support bucket before they are
    // materialised, so that support and the scoring tiles (which take the same
    // buckets) read them in order
    CandGroups sg;
    Scratch<uint64_t> built;   // operand rows built here in the grouped order
    const bool grouped = pmf && pmf->pruned && own_frag && !may_repeat;
    if (grouped) {
        sorted_ids.reset(count, s);
        // the rows are built in the grouped order below when the view is factored; the
        // permutation is needed only to gather the coherence step's rows otherwise
        const bool build_rows = mfma_view.KF && pmf->fr[c].get();
        group_candidates(*pmf, pmf->bk[c], pmf->xr_sup[c].get(), cls.n, KS, ids, nullptr, count, sg, s,
                         sorted_ids.get(), !build_rows);
        vcur = sorted_ids.get();
        if (build_rows) {
            // the pairs' operand rows in this order, from the class's factored rows (as
            // the coherence step built them): cheaper than gathering those at random
            built.reset(count * (mfma_view.ternary ? 2 * mfma_view.KF : mfma_view.KF), s);
            launch_pair_rows_factored(pmf->fr[c].get(), cls.n, vcur, count, mfma_view, built.get(), s);
            pre_idx = nullptr;
        } else if (pre_rows) {
            // row of position p: pre_rows[pre_idx[perm[p]]] (pre_idx: the coherent
            // candidates' rows among all of the coherence step's), or pre_rows[perm[p]]
            const uint32_t RWp = mfma_view.ternary ? 2 * mfma_view.KF : (mfma_view.KF ? mfma_view.KF : KS);
            Scratch<uint64_t> B2(count * RWp, s);
            launch_gather_rows(pre_rows->get(), sg.perm.get(), count, RWp, RWp, B2.get(), nullptr, nullptr, s,
                               pre_idx);
            *pre_rows = std::move(B2);
            pre_idx = nullptr;
        }
    }
    if (may_repeat) {
        // the chunks' survivors may repeat a pattern: canonical order puts repeats side by side
        Scratch<uint32_t> perm(count, s);
        canonical_permutation(m, cls.X.get(), cls.n, ids, count, perm.get(), s);
        sorted_ids.reset(count, s);
        launch_permute_u32(ids, perm.get(), count, sorted_ids.get(), s);
        vcur = sorted_ids.get();
    }
    Scratch<uint64_t> Wtmp;
    Scratch<uint32_t> flag, plen;   // plen: the patterns' token counts, for S = f |b|^2
    bool have_len = false;
    uint64_t *Wd = dev_alloc<uint64_t>(count * KS);
    size_t final_count = count;
    try {
        if (may_repeat) {
            Wtmp.reset(count * KS, s);
            flag.reset(count, s);
            launch_materialize(cls.X.get(), cls.n, KS, vcur, count, Wtmp.get(), flag.get(), s);
            Scratch<uint32_t> pos(count, s), tot(1, s);
            scan_exclusive_u32(flag.get(), pos.get(), count, tot.get(), s);
            launch_compact_rows(Wtmp.get(), flag.get(), pos.get(), count, KS, Wd, s);
            final_count = host_read_u32(tot.get(), 1, s)[0];
        } else {
            plen.reset(count, s);
            have_len = launch_materialize(cls.X.get(), cls.n, KS, vcur, count, Wd, nullptr, s, plen.get());
        }
        m.W[c] = Wd;
        m.np[c] = final_count;
        m.f[c] = dev_alloc<uint32_t>(final_count);
        m.S[c] = dev_alloc<int64_t>(final_count);
    } catch (...) {
        if (Wd && m.W[c] != Wd) m.release(Wd);
        throw;
    }
    if (tm && support_mark >= 0) tm->mark(support_mark);
    if (own_frag) {
        // f on the matrix cores against the class's own records, then S = f |b|^2
        const uint32_t KO = mfma_view.KF ? mfma_view.KF : KS;
        const uint32_t RW = mfma_view.ternary ? 2 * KO : KO;
        Scratch<uint64_t> B;
        if (built.get()) {
            B = std::move(built);
        } else if (pre_rows && !may_repeat && pre_idx) {
            // the coherence step's rows of these patterns, picked out in their order
            B.reset(final_count * RW, s);
            launch_gather_rows(pre_rows->get(), pre_idx, final_count, RW, RW, B.get(), nullptr, nullptr, s);
        } else if (pre_rows && !may_repeat) {
            B = std::move(*pre_rows);   // the coherence step's rows of these patterns, same order
        } else {
            B.reset(final_count * RW, s);
            launch_operand_rows(nullptr, 0, nullptr, m.W[c], KS, final_count, mfma_view, false, B.get(), s);
        }
        hipEvent_t ke[2];
        IG_HIP(hipEventCreate(&ke[0]));
        IG_HIP(hipEventCreate(&ke[1]));
        float tk = 0;
        hipError_t er = hipSuccess;
        if (pmf && pmf->pruned) {
            // the patterns against the class's records that hold their bucket token
            (void)hipEventDestroy(ke[0]);
            (void)hipEventDestroy(ke[1]);
            if (!grouped)   // the rows of a chunked fit, grouped here
                group_candidates(*pmf, pmf->bk[c], nullptr, cls.n, KS, nullptr, m.W[c], final_count, sg, s);
            pruned_contain(*pmf, pmf->bk[c], grouped ? nullptr : sg.perm.get(), sg.first.get(), final_count,
                           B.get(), true, m.f[c], tu.sup_sets, pmf->dtests.get() + 2 + c, &m.stats.kernel_ms[1], s);
            if (have_len) launch_weights_len(m.f[c], plen.get(), final_count, m.S[c], s);
            else launch_weights(m.W[c], m.f[c], final_count, KS, m.S[c], s);
            // the scoring tiles take these buckets when the patterns are in their order
            if (grouped) m.sgroup[c] = host_read_u32(sg.first.get(), pmf->L + 2, s);
        } else {
            m.stats.support_tests[c] = (uint64_t)final_count * cls.n;
            IG_HIP(hipEventRecord(ke[0], s));
            launch_contain_mfma((int)KO, true, B.get(), final_count, own_frag, cls.n, m.f[c], s, tu.sup_sets,
                                mfma_view.ternary != 0);
            IG_HIP(hipEventRecord(ke[1], s));
            if (have_len) launch_weights_len(m.f[c], plen.get(), final_count, m.S[c], s);
            else launch_weights(m.W[c], m.f[c], final_count, KS, m.S[c], s);
            er = hipEventSynchronize(ke[1]);
            if (er == hipSuccess) (void)hipEventElapsedTime(&tk, ke[0], ke[1]);
            (void)hipEventDestroy(ke[0]);
            (void)hipEventDestroy(ke[1]);
        }
        IG_HIP(er);
        m.stats.kernel_ms[1] += tk;
        // the scoring operands use the model's own view: keep the rows when it is this one
        const FactorView &sv = score_view(m);
        if (keep && mfma_view.KF && mfma_view.KF == sv.KF && mfma_view.ternary == sv.ternary) {
            keep->rows[c] = std::move(B);
            keep->valid[c] = true;
        }
    } else {
        m.stats.support_tests[c] = (uint64_t)final_count * cls.n;
        launch_support((int)KS, tu.support_cpl, m.W[c], final_count, cls.NX.get(), cls.n, m.f[c], m.S[c], s);
    }
}

// Matrix-core scoring operands of a finished model: when its rows fit the
// 8-word kernels and every weight is below 2^28 (sixteen of them sum without
// wrapping in 32 bits).  Otherwise scoring stays on the VALU kernel.
// Whether the last token of the scoring operands' last word is used by no pattern
// (factored tokens, or one-hot tokens, fewer than 64 per word on the last word).
static bool score_spare(const DevModel &m) {
    const uint32_t used = m.fv.KF ? m.fac_tokens_last : (m.L % 64 ? m.L % 64 : (m.KS > m.K ? 0u : 64u));
    return used < 64;
}

// Costs of the tokens for the choice of each pattern's bucket token (the lowest
// cost wins), [2][L], one row per class: the training records of the pattern's own
// class that hold the token (the buckets of the fit's pruned support, so that the
// patterns it grouped keep their order; such tokens are also held by few of the
// flows a model scores); for a model without records (imported) the tokens of
// features with more bins first.
static Scratch<uint32_t> token_costs(const DevModel &m, const ClassRows *cls, hipStream_t s) {
    Scratch<uint32_t> cost(2 * (size_t)m.L, s);
    if (cls) {
        launch_fill_u32(cost.get(), 0u, 2 * (size_t)m.L, s);
        for (int c = 0; c < 2; ++c)
            launch_token_counts(cls[c].X.get(), cls[c].n, m.KS, m.L, cost.get() + (size_t)c * m.L, s);
    } else {
        std::vector<uint16_t> nb(m.d);
        IG_HIP(hipMemcpyAsync(nb.data(), m.nbins, m.d * 2, hipMemcpyDeviceToHost, s));
        IG_HIP(hipStreamSynchronize(s));
        std::vector<uint32_t> h(2 * (size_t)m.L, 0);
        uint32_t t = 0;
        for (uint32_t f = 0; f < m.d; ++f)
            for (uint32_t c = 0; c < nb[f]; ++c) h[t++] = 65536u - nb[f];
        std::copy(h.begin(), h.begin() + m.L, h.begin() + m.L);
        upload(cost.get(), h.data(), 2 * (size_t)m.L * 4, s);
        IG_HIP(hipStreamSynchronize(s));
    }
    return cost;
}

// Scoring operands of class c with its tiles grouped by bucket token (every tile
// holds patterns of one bucket; a bucket's last tile is padded with empty rows of
// weight 0): m.frag[c], m.ftiles[c] and m.btile[c].
static void bucketed_operands(DevModel &m, int c, const uint64_t *rows, uint32_t KO, bool spare, bool tern,
                              const uint32_t *cost, hipStream_t s) {
    const size_t np = m.np[c];
    const uint32_t L = m.L;
    std::vector<uint32_t> bt(L + 1, 0), cnt(L, 0);
    const uint32_t *P = nullptr;   // position -> row (null: the rows are in bucket order)
    Scratch<uint64_t> key, key2;
    Scratch<uint32_t> perm, perm2;
    const std::vector<uint32_t> &g = m.sgroup[c];
    if (g.size() == L + 2 && g[L] == np && g[L + 1] == np) {
        // the fit left the patterns grouped by these buckets (none without a token)
        for (uint32_t u = 0; u < L; ++u) cnt[u] = g[u + 1] - g[u];
    } else {
        key.reset(np, s);
        key2.reset(np, s);
        perm.reset(np, s);
        perm2.reset(np, s);
        Scratch<uint32_t> err(1, s), first(L, s);
        launch_fill_u32(err.get(), 0u, 1, s);
        launch_bucket_keys(m.W[c], np, m.KS, L, cost, key.get(), err.get(), s);
        launch_iota(perm.get(), np, s);
        const uint32_t digits = L <= 256 ? 0x1u : 0x3u;
        const int where = radix_sort_pairs(key.get(), perm.get(), key2.get(), perm2.get(), np, digits, s);
        const uint64_t *sk = where ? key2.get() : key.get();
        P = where ? perm2.get() : perm.get();
        launch_fill_u32(first.get(), ~0u, L, s);
        launch_bucket_first(sk, np, first.get(), s);
        std::vector<uint32_t> hf = host_read_u32(first.get(), L, s);
        IG_REQUIRE(host_read_u32(err.get(), 1, s)[0] == 0, IG_E_DEVICE, "a pattern without a token");
        // bucket sizes from the first positions
        uint32_t next = (uint32_t)np;
        for (int u = (int)L - 1; u >= 0; --u) {
            if (hf[u] == ~0u) continue;
            cnt[u] = next - hf[u];
            next = hf[u];
        }
    }
    std::vector<uint32_t> br(L + 1, 0);
    for (uint32_t u = 0; u < L; ++u) {
        bt[u + 1] = bt[u] + (cnt[u] + 31) / 32;
        br[u + 1] = br[u] + cnt[u];
    }
    const uint32_t ntiles = bt[L];
    m.btile[c] = dev_alloc<uint32_t>(L + 1);
    upload(m.btile[c], bt.data(), (L + 1) * 4, s);
    // the rows of each bucket: for the tiles below and the evidence of a flow (ig_evidence)
    m.brow[c] = dev_alloc<uint32_t>(L + 1);
    upload(m.brow[c], br.data(), (L + 1) * 4, s);
    m.bperm[c] = dev_alloc<uint32_t>(np);
    if (P) IG_HIP(hipMemcpyAsync(m.bperm[c], P, np * 4, hipMemcpyDeviceToDevice, s));
    else launch_iota(m.bperm[c], np, s);
    m.ftiles[c] = ntiles;
    m.frag[c] = dev_alloc<uint4>((size_t)std::max<uint32_t>(ntiles, 1) * score_tile_words(KO));
    launch_mfma_patterns(rows, m.S[c], (uint32_t)np, KO, spare, tern, m.frag[c], s, P, m.btile[c], m.brow[c], L,
                         ntiles);
}

static void build_score_operands(DevModel &m, hipStream_t s, PatternRows *pr, const ClassRows *cls) {
    const FactorView &sv = score_view(m);
    const bool tern = sv.ternary != 0;
    const uint32_t KO = sv.KF ? sv.KF : m.KS, RW = tern ? 2 * KO : KO;
    if (KO > 8 || m.maxS[0] >= (1ll << 28) || m.maxS[1] >= (1ll << 28)) return;
    const bool spare = !tern && score_spare(m);
    // fits from codes and imported models group their tiles by token for pruned scoring
    const bool bucketed = m.d > 0 && m.L <= 4096;
    Scratch<uint32_t> cost;
    const auto grouped = [&](int c) { return m.sgroup[c].size() == m.L + 2 && m.sgroup[c][m.L + 1] == m.np[c]; };
    if (bucketed && !(grouped(0) && grouped(1))) cost = token_costs(m, cls, s);
    for (int c = 0; c < 2; ++c) {
        Scratch<uint64_t> own;
        const uint64_t *rows;
        if (pr && pr->valid[c]) {
            rows = pr->rows[c].get();
        } else {
            own.reset(std::max<uint64_t>(m.np[c], 1) * RW, s);
            launch_operand_rows(nullptr, 0, nullptr, m.W[c], m.KS, m.np[c], sv, false, own.get(), s);
            rows = own.get();
        }
        if (bucketed && m.np[c]) {
            bucketed_operands(m, c, rows, KO, spare, tern, cost.get() + (size_t)c * m.L, s);
            continue;
        }
        if (bucketed) {   // an empty class: no tiles or rows in any bucket
            m.btile[c] = dev_alloc<uint32_t>(m.L + 1);
            launch_fill_u32(m.btile[c], 0u, m.L + 1, s);
            m.brow[c] = dev_alloc<uint32_t>(m.L + 1);
            launch_fill_u32(m.brow[c], 0u, m.L + 1, s);
            m.bperm[c] = dev_alloc<uint32_t>(1);
        }
        const uint64_t ntiles = (m.np[c] + 31) / 32;
        m.ftiles[c] = (uint32_t)ntiles;
        m.frag[c] = dev_alloc<uint4>(std::max<uint64_t>(ntiles, 1) * score_tile_words(KO));
        launch_mfma_patterns(rows, m.S[c], (uint32_t)m.np[c], KO, spare, tern, m.frag[c], s);
    }
    m.score_factored = sv.KF > 0;
    m.score_ternary = tern;
    m.score_spare = spare;
}

static void finish_weights(DevModel &m, hipStream_t s, PatternRows *pr = nullptr, const ClassRows *cls = nullptr) {
    Scratch<unsigned long long> ms(4, s);
    for (int c = 0; c < 2; ++c) launch_reduce_maxsum(m.S[c], m.np[c], ms.get() + 2 * c, s);
    unsigned long long h[4];
    IG_HIP(hipMemcpyWithStream(h, ms.get(), sizeof(h), hipMemcpyDeviceToHost, s));
    for (int c = 0; c < 2; ++c) {
        m.maxS[c] = (int64_t)h[2 * c];
        // A(x) and N(x) are sums of a subset of one class's weights (Eq. 4)
        IG_REQUIRE(h[2 * c + 1] <= (unsigned long long)INT64_MAX, IG_E_OVERFLOW,
                   "sum of pattern weights exceeds int64");
    }
    build_score_operands(m, s, pr, cls);
}

// Ends of the coherence phases over the other class's records.  One phase (the
// whole class) measured fastest: splitting the scan lets covered candidates stop
// earlier, but each extra phase reloads the survivors and appends them through a
// shared counter, which cost more than the idle lanes it saved.
static std::vector<uint32_t> coherence_phases(uint32_t max_other) {
    return std::vector<uint32_t>{std::max<uint32_t>(max_other, 1)};
}

// Bytes of the (class, hash) keys that the de-duplication sorts on: 1 class bit and
// 39 hash bits.  Distinct intersections that share a key are told apart by the
// full comparison; at 2^24 distinct per class about 2^8 pairs of them do.  Fewer
// bits save a radix pass but cost more: the occurrences of two intersections that
// share a key interleave, and each one scans back over the other's to find its own.
constexpr int kPairKeyBytes = 5;
constexpr int kSortHashBits = 8 * kPairKeyBytes - 1;

constexpr uint32_t kMfmaWords = 16;   // widest operands of the subset-test contraction

// Matrix-core operands of one fit: the token view (factored, or the one-hot words
// in mode 3) and, per class c, the records of class 1 - c as A tiles (class c's
// coherence operand, and class 1 - c's support operand).
// Decide the subset-test path of a fit from the coherence_mfma option (0 auto:
// matrix cores when the operands fit 16 words; 1 matrix cores; 2 VALU; 3 matrix
// cores on the one-hot words; 4 matrix cores on the factored tokens with presence
// tokens; 5 matrix cores on the ternary bit tokens) and build the record tiles
// when it is the matrix cores.  Modes 0 and 1 take the ternary view (bit tokens
// only) of a fit from codes when it needs fewer words than the presence tokens.
static void mfma_setup(const DevModel &m, const ClassRows cls[2], uint32_t mode, uint32_t dense, MfmaFit &mf,
                       hipStream_t s) {
    IG_REQUIRE(mode <= 5, IG_E_INVAL, "coherence_mfma must be 0 to 5");
    IG_REQUIRE(dense <= 1, IG_E_INVAL, "fit_dense must be 0 or 1");
    const uint32_t KS = m.KS;
    const bool tern = m.tv.KF && (mode == 5 || ((mode == 0 || mode == 1) && (!m.fv.KF || m.tv.KF < m.fv.KF)));
    mf.view = mode == 3 ? FactorView{} : tern ? m.tv : m.fv;
    mf.KO = mf.view.KF ? mf.view.KF : KS;
    mf.RW = mf.view.ternary ? 2 * mf.KO : mf.KO;
    IG_REQUIRE(mode == 0 || mode == 2 || mf.KO <= kMfmaWords, IG_E_UNSUPPORTED,
               "the matrix-core subset tests handle up to 16 operand words");
    mf.on = mode != 2 && (mode != 0 || mf.KO <= kMfmaWords);
    if (!mf.on) return;
    if (mf.view.KF) {
        // each class's records, factored: its candidates' rows are built from them,
        // and the other class's record tiles hold them on the signed (or ternary) side
        for (int c = 0; c < 2; ++c) {
            mf.fr[c].reset(std::max<size_t>(cls[c].n, 1) * mf.RW, s);
            launch_operand_rows(nullptr, 0, nullptr, cls[c].X.get(), KS, cls[c].n, mf.view, false, mf.fr[c].get(),
                                s);
        }
    }
    for (int c = 0; c < 2; ++c) {
        const ClassRows &o = cls[1 - c];
        mf.frag[c].reset(std::max<size_t>((size_t)mfma_record_tiles(o.n) * mf.KO * 64, 1), s);
        if (mf.view.ternary)
            launch_mfma_records_ternary(mf.fr[1 - c].get(), o.n, mf.KO, m.tern_tokens, mf.frag[c].get(), s);
        else if (mf.view.KF) launch_mfma_records_signed(mf.fr[1 - c].get(), o.n, mf.view, mf.frag[c].get(), s);
        else launch_mfma_records(o.NX.get(), o.n, KS, mf.frag[c].get(), s);
    }
    // token buckets (ternary view): each candidate meets the records holding its
    // rarest token only
    mf.pruned = !dense && mf.view.ternary && m.L >= 1 && m.L <= 4096 && m.d >= 1;
    if (mf.pruned) {
        mf.L = m.L;
        mf.KSr = (m.L + 63) / 64;
        mf.dtests.reset(4, s);
        launch_fill_u64(reinterpret_cast<uint64_t *>(mf.dtests.get()), 0ull, 4, s);
        build_fit_buckets(m, cls, mf, s);
        for (int c = 0; c < 2; ++c) {
            const size_t rows = std::max<size_t>(cls[c].n, 1) * mf.KSr;
            mf.xr_coh[c].reset(rows, s);
            mf.xr_sup[c].reset(rows, s);
            launch_rank_rows(cls[c].X.get(), cls[c].n, KS, m.L, mf.bk[1 - c].rank.get(), mf.KSr, mf.xr_coh[c].get(), s);
            launch_rank_rows(cls[c].X.get(), cls[c].n, KS, m.L, mf.bk[c].rank.get(), mf.KSr, mf.xr_sup[c].get(), s);
        }
    }
}

// Coherence of class c's ncand candidate pair ids `cand` on the matrix cores
// (Eq. 3): appends the coherent ids to `out` and returns how many (synchronises
// the stream); adds the contraction's device time to *kernel_ms.  With rows_out,
// the coherent candidates' operand rows are kept for support and scoring: on token
// buckets every candidate's rows, with idx_out [kept] their positions in order;
// otherwise only the coherent ones' rows, in order (idx_out left empty).
static uint32_t mfma_coherence(MfmaFit &mf, const ClassRows cls[2], int c, uint32_t KS, const uint32_t *cand,
                               uint32_t ncand, uint32_t *out, float *kernel_ms, hipStream_t s,
                               Scratch<uint64_t> *rows_out = nullptr, Scratch<uint32_t> *idx_out = nullptr,
                               int sets = 0, uint64_t *tests = nullptr) {
    if (!ncand) return 0;
    Scratch<uint32_t> keep(ncand, s), kpos(ncand, s), ktot(1, s);
    Scratch<uint64_t> B((size_t)ncand * mf.RW, s);
    if (mf.pruned) {
        // the candidates against the other class's records that hold their bucket
        // token: grouped by bucket first, so that their operand rows are built in
        // bucket order (the contraction then reads them in order), flags in bucket
        // order too (coalesced stores); the coherent ids come out in that order
        CandGroups g;
        Scratch<uint32_t> sids(ncand, s);
        group_candidates(mf, mf.bk[1 - c], mf.xr_coh[c].get(), cls[c].n, KS, cand, nullptr, ncand, g, s,
                         sids.get(), false);
        if (mf.view.KF)
            launch_pair_rows_factored(mf.fr[c].get(), cls[c].n, sids.get(), ncand, mf.view, B.get(), s);
        else
            launch_operand_rows(cls[c].X.get(), cls[c].n, sids.get(), nullptr, KS, ncand, mf.view, false, B.get(),
                                s);
        pruned_contain(mf, mf.bk[1 - c], nullptr, g.first.get(), ncand, B.get(), false, keep.get(), sets,
                       mf.dtests.get() + c, kernel_ms, s, true);
        scan_exclusive_u32(keep.get(), kpos.get(), ncand, ktot.get(), s);
        if (rows_out) idx_out->reset(ncand, s);
        launch_compact(keep.get(), kpos.get(), sids.get(), ncand, out, s, rows_out ? idx_out->get() : nullptr);
        const uint32_t kept = host_read_u32(ktot.get(), 1, s)[0];
        if (rows_out) *rows_out = std::move(B);
        return kept;
    }
    if (mf.view.KF)
        launch_pair_rows_factored(mf.fr[c].get(), cls[c].n, cand, ncand, mf.view, B.get(), s);
    else
        launch_operand_rows(cls[c].X.get(), cls[c].n, cand, nullptr, KS, ncand, mf.view, false, B.get(), s);
    if (tests) *tests += (uint64_t)ncand * cls[1 - c].n;
    hipEvent_t ke[2];
    IG_HIP(hipEventCreate(&ke[0]));
    IG_HIP(hipEventCreate(&ke[1]));
    struct Ev {
        hipEvent_t *e;
        ~Ev() {
            (void)hipEventDestroy(e[0]);
            (void)hipEventDestroy(e[1]);
        }
    } evg{ke};
    IG_HIP(hipEventRecord(ke[0], s));
    launch_contain_mfma((int)mf.KO, false, B.get(), ncand, mf.frag[c].get(), cls[1 - c].n, keep.get(), s, sets,
                        mf.view.ternary != 0);
    IG_HIP(hipEventRecord(ke[1], s));
    scan_exclusive_u32(keep.get(), kpos.get(), ncand, ktot.get(), s);
    launch_compact(keep.get(), kpos.get(), cand, ncand, out, s);
    // the coherent candidates' operand rows, in the same order (support and scoring use them)
    if (rows_out) {
        rows_out->reset((size_t)ncand * mf.RW, s);
        launch_compact_rows(B.get(), keep.get(), kpos.get(), ncand, mf.RW, rows_out->get(), s);
    }
    const uint32_t kept = host_read_u32(ktot.get(), 1, s)[0];
    float tk = 0;
    IG_HIP(hipEventElapsedTime(&tk, ke[0], ke[1]));
    if (kernel_ms) *kernel_ms += tk;
    return kept;
}

// The operand rows of the fit's contractions, for ig_model_info.
static void note_fit_operands(DevModel &m, const MfmaFit &mf) {
    m.fit_words = mf.KO;
    m.fit_tokens = mf.view.ternary ? m.tern_tokens : mf.view.KF ? m.fac_tokens : m.L;
}

static void fit_from_rows(DevModel &m, ClassRows cls[2], const ig_fit_opts *opts, hipStream_t s, Timer &tm) {
    const uint32_t KS = m.KS, K = m.K;
    const uint64_t fit_pairs = (uint64_t)cls[0].n * (cls[0].n ? cls[0].n - 1 : 0) / 2 +
                               (uint64_t)cls[1].n * (cls[1].n ? cls[1].n - 1 : 0) / 2;
    Tuning tu = tuning_for(opts, KS, fit_pairs);
    uint64_t M[2];
    for (int c = 0; c < 2; ++c) {
        uint64_t n = cls[c].n;
        IG_REQUIRE(n <= 92000, IG_E_UNSUPPORTED, "more than 92,000 training records in one class");
        M[c] = n + n * (n ? n - 1 : 0) / 2;
        m.stats.n_class[c] = n;
        m.stats.pairs[c] = n * (n ? n - 1 : 0) / 2;
        m.stats.support_tests[c] = 0;
    }
    // items per pair-space chunk: ~80 bytes of scratch per item (sort pairs, flags,
    // candidates and their matrix-core operand rows)
    uint64_t chunk_items = 1ull << 31;
    if (opts && opts->mem_budget_bytes) chunk_items = std::max<uint64_t>(opts->mem_budget_bytes / 80, 4096);
    struct Piece {
        int c;
        uint64_t q0, cnt;
    };
    std::vector<std::vector<Piece>> chunks;
    {
        std::vector<Piece> cur;
        uint64_t used = 0;
        for (int c = 0; c < 2; ++c) {
            uint64_t q = 0;
            while (q < M[c]) {
                uint64_t take = std::min(M[c] - q, chunk_items - used);
                cur.push_back({c, q, take});
                used += take;
                q += take;
                if (used == chunk_items) {
                    chunks.push_back(cur);
                    cur.clear();
                    used = 0;
                }
            }
        }
        if (!cur.empty()) chunks.push_back(cur);
    }
    m.stats.chunks[0] = m.stats.chunks[1] = 0;
    for (auto &ch : chunks)
        for (int c = 0; c < 2; ++c)
            if (std::any_of(ch.begin(), ch.end(), [&](const Piece &p) { return p.c == c; })) m.stats.chunks[c]++;

    // survivors (coherent pair ids) per class, grown as chunks add candidates
    Scratch<uint32_t> surv[2];
    size_t surv_cap[2] = {0, 0};
    Scratch<uint32_t> counters(4, s);   // nsurv[0], nsurv[1], queue, spare
    Scratch<unsigned long long> tests(2, s);
    launch_fill_u32(counters.get(), 0u, 4, s);
    launch_fill_u64(reinterpret_cast<uint64_t *>(tests.get()), 0ull, 2, s);
    uint64_t distinct[2] = {0, 0};

    // row descriptors for the de-duplication kernel (segment = class)
    Scratch<unsigned char> rowsegs(2 * rows_of_seg_size(), s);
    {
        std::vector<unsigned char> h(2 * rows_of_seg_size());
        for (int c = 0; c < 2; ++c) fill_rows_of_seg(h.data() + c * rows_of_seg_size(), cls[c].X.get(), cls[c].n, KS, K);
        upload(rowsegs.get(), h.data(), h.size(), s);
    }
    const uint32_t grid = coherence_grid(tu.grid_per_cu);
    MfmaFit mf;
    mfma_setup(m, cls, opts ? opts->coherence_mfma : 0u, opts ? opts->fit_dense : 0u, mf, s);
    const bool use_mfma = mf.on;
    if (use_mfma) {
        mfma_tuning(opts, mf.KO, fit_pairs, tu);
        note_fit_operands(m, mf);
        // scoring follows the fit's factored view
        if (mf.view.KF) m.score_pref = mf.view.ternary ? 1 : 0;
        m.fit_buckets = mf.pruned;
    }
    Scratch<uint64_t> surv_rows[2];   // operand rows of the coherent candidates (one-chunk fits)
    Scratch<uint32_t> surv_idx[2];    // on token buckets: their positions among surv_rows
    uint64_t mfma_surv[2] = {0, 0}, mfma_tests[2] = {0, 0};
    float ms_pairs = 0, ms_sort = 0, ms_dedup = 0, ms_coh = 0;
    hipEvent_t e[5];
    for (auto &x : e) IG_HIP(hipEventCreate(&x));
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard() {
            for (int i = 0; i < 5; ++i) (void)hipEventDestroy(e[i]);
        }
    } evg{e};
    tm.mark(1);
    for (auto &ch : chunks) {
        uint64_t items = 0;
        for (auto &p : ch) items += p.cnt;
        Scratch<uint32_t> segc(2, s), cand(items, s), tot(1, s);
        // one chunk holding both classes' whole pair spaces: de-duplication with a
        // partial sort, candidates in pair order; the full sort below when it cannot
        // separate two candidates
        bool done = false;
        if (chunks.size() == 1 && dedup_partitioned_fits(items)) {
            uint64_t q0[2] = {0, 0}, cnt[2] = {0, 0};
            for (auto &p : ch) {
                q0[p.c] = p.q0;
                cnt[p.c] = p.cnt;
            }
            Scratch<uint32_t> err(1, s);
            IG_HIP(hipEventRecord(e[0], s));   // pairs and sort stages: none (all in the de-duplication)
            IG_HIP(hipEventRecord(e[1], s));
            IG_HIP(hipEventRecord(e[2], s));
            launch_dedup_partitioned(cls[0].X.get(), cls[0].n, q0[0], cnt[0], cls[1].X.get(), cls[1].n, q0[1], cnt[1],
                                     KS, K, cand.get(), tot.get(), segc.get(), err.get(), s);
            done = host_read_u32(err.get(), 1, s)[0] == 0;
        }
        if (!done) {
            Scratch<uint64_t> k0(items, s), k1(items, s);
            Scratch<uint32_t> v0(items, s), v1(items, s), flags(items, s), pos(items, s);
            IG_HIP(hipEventRecord(e[0], s));
            uint64_t at = 0;
            for (auto &p : ch) {
                launch_pair_hash(cls[p.c].X.get(), cls[p.c].n, KS, K, p.q0, p.cnt, (uint32_t)p.c, 1, k0.get() + at,
                                 v0.get() + at, s, kPairKeyBytes);
                at += p.cnt;
            }
            IG_HIP(hipEventRecord(e[1], s));
            int where = radix_sort_pairs(k0.get(), v0.get(), k1.get(), v1.get(), items,
                                         0xffu & ~((1u << (8 - kPairKeyBytes)) - 1), s);
            uint64_t *ks = where ? k1.get() : k0.get();
            uint32_t *vs = where ? v1.get() : v0.get();
            IG_HIP(hipEventRecord(e[2], s));
            launch_dedup_flags(ks, vs, items, rowsegs.get(), 1, flags.get(), segc.get(), s);
            scan_exclusive_u32(flags.get(), pos.get(), items, tot.get(), s);
            launch_seg_counts(ks, items, pos.get(), tot.get(), 1, 2, segc.get(), s);
            launch_compact(flags.get(), pos.get(), vs, items, cand.get(), s);
        }
        IG_HIP(hipEventRecord(e[3], s));
        std::vector<uint32_t> hc = host_read_u32(segc.get(), 2, s);
        std::vector<uint32_t> hn = host_read_u32(counters.get(), 2, s);
        float t01, t12, t23;
        IG_HIP(hipEventElapsedTime(&t01, e[0], e[1]));
        IG_HIP(hipEventElapsedTime(&t12, e[1], e[2]));
        IG_HIP(hipEventElapsedTime(&t23, e[2], e[3]));
        ms_pairs += t01;
        ms_sort += t12;
        ms_dedup += t23;
        // grow the survivor buffers to hold every candidate of this chunk
        for (int c = 0; c < 2; ++c) {
            distinct[c] += hc[c];
            const size_t have = use_mfma ? (size_t)mfma_surv[c] : (size_t)hn[c];
            size_t need = have + hc[c];
            if (need > surv_cap[c]) {
                size_t cap = std::max<size_t>(need, surv_cap[c] * 3 / 2);
                Scratch<uint32_t> nb(cap, s);
                if (have) IG_HIP(hipMemcpyAsync(nb.get(), surv[c].get(), have * 4, hipMemcpyDeviceToDevice, s));
                surv[c] = std::move(nb);
                surv_cap[c] = cap;
            }
        }
        if (use_mfma) {
            // stage time read when the fit ends (no synchronisation here)
            KernelClock::Item &coh_it = mf.clock.open(s, &ms_coh);
            for (int c = 0; c < 2; ++c) {
                const uint32_t *cc = cand.get() + (c == 0 ? 0 : hc[0]);
                // one chunk: keep the survivors' operand rows for support and scoring
                // (on token buckets support builds them again in its own order)
                const bool keep_rows = chunks.size() == 1 && !mf.pruned;
                mfma_surv[c] += mfma_coherence(mf, cls, c, KS, cc, hc[c], surv[c].get() + mfma_surv[c],
                                               &m.stats.kernel_ms[0], s, keep_rows ? &surv_rows[c] : nullptr,
                                               keep_rows ? &surv_idx[c] : nullptr, tu.coh_sets, &mfma_tests[c]);
            }
            mf.clock.close(coh_it, s);
            continue;
        }
        // coherence in phases over the other class's records (input order); the
        // uncovered ids ping-pong between the de-duplication output and `alt`
        const std::vector<uint32_t> bounds = coherence_phases(std::max(cls[0].n, cls[1].n));
        Scratch<uint32_t> alt(std::max<size_t>((size_t)hc[0] + hc[1], 1), s);
        Scratch<uint32_t> pcount(2 * 2 * bounds.size(), s);   // per phase, per class: output counter
        launch_fill_u32(pcount.get(), 0u, 2 * 2 * bounds.size(), s);
        std::vector<CohSeg> hs;
        std::vector<uint32_t> seg_first, seg_count;   // slice of hs used by each phase
        {
            uint32_t *cur[2] = {cand.get(), cand.get() + hc[0]};
            uint32_t *nxt[2] = {alt.get(), alt.get() + hc[0]};
            const uint32_t *curcnt[2] = {segc.get(), segc.get() + 1};
            uint32_t r_begin = 0;
            for (size_t p = 0; p < bounds.size(); ++p) {
                const uint32_t r_end = bounds[p];
                seg_first.push_back((uint32_t)hs.size());
                for (int c = 0; c < 2; ++c) {
                    const uint32_t n_o = cls[1 - c].n;
                    if (r_begin >= n_o && !(r_begin == 0 && n_o == 0)) continue;   // finished earlier
                    const bool last = r_end >= n_o;
                    CohSeg g{};
                    g.X = cls[c].X.get();
                    g.NXo = cls[1 - c].NX.get();
                    g.cand = cur[c];
                    g.cand_off = nullptr;
                    g.ncand = curcnt[c];
                    g.out = last ? surv[c].get() : nxt[c];
                    g.nout = last ? counters.get() + c : pcount.get() + 4 * p + c;
                    g.tests = tests.get() + c;
                    g.n = cls[c].n;
                    g.n_o = n_o;
                    hs.push_back(g);
                    if (!last) {
                        curcnt[c] = pcount.get() + 4 * p + c;
                        std::swap(cur[c], nxt[c]);
                    }
                }
                seg_count.push_back((uint32_t)hs.size() - seg_first.back());
                r_begin = r_end;
            }
        }
        Scratch<CohSeg> dsegs(std::max<size_t>(hs.size(), 1), s);
        if (!hs.empty())
            upload(dsegs.get(), hs.data(), hs.size() * sizeof(CohSeg), s);
        IG_HIP(hipEventRecord(e[3], s));   // brackets the coherence phases
        {
            uint32_t r_begin = 0;
            for (size_t p = 0; p < bounds.size(); ++p) {
                if (seg_count[p])
                    launch_coherence((int)KS, tu.cpl, dsegs.get() + seg_first[p], seg_count[p], r_begin, bounds[p],
                                     counters.get() + 2, grid, s);
                r_begin = bounds[p];
            }
        }
        IG_HIP(hipEventRecord(e[4], s));
        IG_HIP(hipStreamSynchronize(s));   // host copies above must outlive their transfers
        float t34;
        IG_HIP(hipEventElapsedTime(&t34, e[3], e[4]));
        ms_coh += t34;
    }
    tm.mark(4);
    std::vector<uint32_t> hn = host_read_u32(counters.get(), 2, s);
    unsigned long long ht[2];
    IG_HIP(hipMemcpyWithStream(ht, tests.get(), sizeof(ht), hipMemcpyDeviceToHost, s));
    if (use_mfma)
        for (int c = 0; c < 2; ++c) {
            hn[c] = (uint32_t)mfma_surv[c];
            ht[c] = mfma_tests[c];
        }
    for (int c = 0; c < 2; ++c) {
        m.stats.distinct[c] = distinct[c];
        m.stats.tests[c] = ht[c];
    }
    const bool chunked = chunks.size() > 1;
    PatternRows prow;
    for (int c = 0; c < 2; ++c) {
        // frag[1 - c] holds class c's own records (it is class 1-c's coherence operand)
        order_and_weigh(m, c, cls[c], surv[c].get(), hn[c], chunked, tu, s, &tm, c == 0 ? 5 : 8,
                        use_mfma ? mf.frag[1 - c].get() : nullptr, mf.view, &prow,
                        surv_rows[c].get() ? &surv_rows[c] : nullptr, use_mfma ? &mf : nullptr,
                        surv_idx[c].get());
        m.stats.coherent[c] = m.np[c];
        if (c == 0) tm.mark(3);   // end of class 0's support
    }
    tm.mark(6);
    finish_weights(m, s, &prow, cls);
    tm.mark(7);
    mf.finish(s);
    mf.clock.collect();
    mf.put_tests(m);
    m.stats.ms[1] = ms_pairs;
    m.stats.ms[2] = ms_sort;
    m.stats.ms[3] = ms_dedup;
    m.stats.ms[4] = ms_coh;
}

static void alloc_class_rows(ClassRows cls[2], const uint32_t *counts, uint32_t KS, hipStream_t s) {
    for (int c = 0; c < 2; ++c) {
        const size_t rows = std::max<uint32_t>(counts[c], 1);
        cls[c].n = counts[c];
        cls[c].X.reset(rows * KS, s);
        cls[c].NX.reset(rows * KS, s);
    }
}

static DevModel *new_model() {
    DevModel *m = new DevModel();
    IG_HIP(hipGetDevice(&m->device));
    if (const ig_allocator *u = current_user_allocator()) {
        m->user = *u;
        m->has_user = true;
    }
    return m;
}

// Stage times from the fit's events: 0 start, 1 packed, 4 coherence done,
// 5 class-0 support start, 3 class-0 support end, 8 class-1 support start,
// 6 class-1 support end, 7 done.
static void record_times(DevModel &m, Timer &tm) {
    float a, b, c0, c1;
    if (tm.elapsed(0, 1, a)) m.stats.ms[0] = a;
    if (tm.elapsed(5, 3, c0) && tm.elapsed(8, 6, c1)) {
        m.stats.ms[6] = c0 + c1;
        if (tm.elapsed(4, 6, b)) m.stats.ms[5] = b - c0 - c1;
    }
    if (tm.elapsed(0, 7, a)) m.stats.ms[7] = a;
}

DevModel *fit_codes(const uint16_t *d_codes, const uint8_t *d_labels, uint32_t n, uint32_t d,
                    const uint16_t *h_nbins, const ig_fit_opts *opts, hipStream_t s) {
    uint32_t L, K;
    check_nbins(h_nbins, d, L, K);
    IG_REQUIRE(n == 0 || (d_codes && d_labels), IG_E_INVAL, "codes or labels is NULL");
    const int KS = storage_words((int)K);
    IG_REQUIRE(KS > 0, IG_E_UNSUPPORTED, "unsupported word count");
    std::unique_ptr<DevModel> m(new_model());
    m->K = K;
    m->KS = (uint32_t)KS;
    m->L = L;
    m->d = d;
    Timer tm(s);
    tm.mark(0);
    std::vector<uint32_t> tab = token_tables(h_nbins, d, (uint32_t)KS);
    m->meta = dev_alloc<uint32_t>(tab.size());
    m->nbins = dev_alloc<uint16_t>(d);
    upload(m->meta, tab.data(), tab.size() * 4, s);
    upload(m->nbins, h_nbins, d * 2, s);
    set_key_pieces(*m, h_nbins, d, s);
    set_factor_table(*m, h_nbins, d, s);
    set_factor_table(*m, h_nbins, d, s, true);
    Scratch<uint32_t> err(1, s), pos(n ? n : 1, s), counts(2, s);
    launch_fill_u32(err.get(), 0u, 1, s);
    launch_fill_u32(counts.get(), 0u, 2, s);
    launch_validate_codes(d_codes, (size_t)n * d, d, m->nbins, err.get(), s);
    if (n) launch_split_labels(d_labels, n, pos.get(), counts.get(), err.get(), s);
    std::vector<uint32_t> h = host_read_u32(err.get(), 1, s);   // also completes the table uploads
    IG_REQUIRE(!(h[0] & 1u), IG_E_INVAL, "a code is not below its feature's bin count");
    IG_REQUIRE(!(h[0] & 2u), IG_E_INVAL, "a label is not 0 or 1");
    std::vector<uint32_t> hc = host_read_u32(counts.get(), 2, s);
    ClassRows cls[2];
    alloc_class_rows(cls, hc.data(), (uint32_t)KS, s);
    launch_pack_split(d_codes, d_labels, n, d, (uint32_t)KS, m->meta, pos.get(), cls[0].X.get(), cls[1].X.get(),
                      cls[0].NX.get(), cls[1].NX.get(), s);
    fit_from_rows(*m, cls, opts, s, tm);
    record_times(*m, tm);
    return m.release();
}

DevModel *fit_packed(const uint64_t *d_words, const uint8_t *d_labels, uint32_t n, uint32_t K,
                     const ig_fit_opts *opts, hipStream_t s) {
    IG_REQUIRE(K >= 1 && K <= 64, IG_E_UNSUPPORTED, "K must be in 1..64");
    IG_REQUIRE(n == 0 || (d_words && d_labels), IG_E_INVAL, "words or labels is NULL");
    const int KS = storage_words((int)K);
    std::unique_ptr<DevModel> m(new_model());
    m->K = K;
    m->KS = (uint32_t)KS;
    m->L = 64 * K;
    m->d = 0;
    Timer tm(s);
    tm.mark(0);
    Scratch<uint32_t> err(1, s), pos(n ? n : 1, s), counts(2, s);
    launch_fill_u32(err.get(), 0u, 1, s);
    launch_fill_u32(counts.get(), 0u, 2, s);
    if (n) launch_split_labels(d_labels, n, pos.get(), counts.get(), err.get(), s);
    std::vector<uint32_t> h = host_read_u32(err.get(), 1, s);
    IG_REQUIRE(!(h[0] & 2u), IG_E_INVAL, "a label is not 0 or 1");
    std::vector<uint32_t> hc = host_read_u32(counts.get(), 2, s);
    ClassRows cls[2];
    alloc_class_rows(cls, hc.data(), (uint32_t)KS, s);
    launch_split_packed(d_words, d_labels, n, K, (uint32_t)KS, pos.get(), cls[0].X.get(), cls[1].X.get(),
                        cls[0].NX.get(), cls[1].NX.get(), s);
    fit_from_rows(*m, cls, opts, s, tm);
    record_times(*m, tm);
    return m.release();
}

DevModel *import_patterns(const uint16_t *const h_codes[2], const uint32_t *const h_f[2], const uint64_t count[2],
                          uint32_t d, const uint16_t *h_nbins, hipStream_t s) {
    uint32_t L, K;
    check_nbins(h_nbins, d, L, K);
    const int KS = storage_words((int)K);
    std::unique_ptr<DevModel> m(new_model());
    m->K = K;
    m->KS = (uint32_t)KS;
    m->L = L;
    m->d = d;
    std::vector<uint32_t> tab = token_tables(h_nbins, d, (uint32_t)KS);
    m->meta = dev_alloc<uint32_t>(tab.size());
    m->nbins = dev_alloc<uint16_t>(d);
    upload(m->meta, tab.data(), tab.size() * 4, s);
    upload(m->nbins, h_nbins, d * 2, s);
    set_factor_table(*m, h_nbins, d, s);
    set_factor_table(*m, h_nbins, d, s, true);
    for (int c = 0; c < 2; ++c) {
        const uint64_t cnt = count[c];
        IG_REQUIRE(cnt < (1ull << 31), IG_E_UNSUPPORTED, "more than 2^31 patterns in one class");
        IG_REQUIRE(cnt == 0 || (h_codes[c] && h_f[c]), IG_E_INVAL, "pattern codes or supports is NULL");
        m->np[c] = cnt;
        m->W[c] = dev_alloc<uint64_t>(cnt * KS);
        m->f[c] = dev_alloc<uint32_t>(cnt);
        m->S[c] = dev_alloc<int64_t>(cnt);
        if (!cnt) continue;
        Scratch<uint16_t> dc(cnt * d, s);
        Scratch<uint32_t> df(cnt, s), err(1, s), ids(cnt, s), v1(cnt, s), tot(1, s);
        Scratch<uint64_t> Wraw(cnt * KS, s), k0(cnt, s), k1(cnt, s);
        upload(dc.get(), h_codes[c], cnt * d * 2, s);
        upload(df.get(), h_f[c], cnt * 4, s);
        launch_fill_u32(err.get(), 0u, 1, s);
        launch_pack_patterns(dc.get(), (uint32_t)cnt, d, (uint32_t)KS, m->meta, m->nbins, Wraw.get(), err.get(), s);
        std::vector<uint32_t> he = host_read_u32(err.get(), 1, s);
        IG_REQUIRE(!(he[0] & 1u), IG_E_INVAL, "a pattern code is neither absent nor below its bin count");
        IG_REQUIRE(!(he[0] & 2u), IG_E_INVAL, "a pattern has no token");
        launch_iota(ids.get(), cnt, s);
        uint32_t *vcur = ids.get(), *valt = v1.get();
        for (int k = (int)K - 1; k >= 0; --k) {
            launch_row_word(Wraw.get(), vcur, cnt, (uint32_t)KS, (uint32_t)k, k0.get(), s);
            int where = radix_sort_pairs(k0.get(), vcur, k1.get(), valt, cnt, 0xffu, s);
            if (where) std::swap(vcur, valt);
        }
        launch_gather_rows(Wraw.get(), vcur, cnt, (uint32_t)KS, (uint32_t)KS, m->W[c], df.get(), m->f[c], s);
        // distinctness: ordered rows must all differ from their predecessor
        launch_fill_u32(tot.get(), 0u, 1, s);
        launch_adjacent_equal(m->W[c], cnt, (uint32_t)KS, tot.get(), s);
        launch_weights(m->W[c], m->f[c], cnt, (uint32_t)KS, m->S[c], s);
        std::vector<uint32_t> dup = host_read_u32(tot.get(), 1, s);
        IG_REQUIRE(dup[0] == 0, IG_E_INVAL, "pattern set of class " + std::to_string(c) + " has repeated patterns");
    }
    finish_weights(*m, s);
    IG_HIP(hipStreamSynchronize(s));   // the model is complete when it is returned
    return m.release();
}


// ------------------------------------------------------------ batched fit ----
// A library-owned stream per device for captured sequences (a caller's stream
// may be the legacy default stream, which cannot be captured).
static std::mutex g_batch_mu;

static hipStream_t internal_stream() {
    static hipStream_t st[64] = {};
    int dev = 0;
    IG_HIP(hipGetDevice(&dev));
    IG_REQUIRE(dev >= 0 && dev < 64, IG_E_UNSUPPORTED, "device index beyond 63");
    if (!st[dev]) IG_HIP(hipStreamCreateWithFlags(&st[dev], hipStreamNonBlocking));
    return st[dev];
}

struct BProb {
    uint32_t n = 0, d = 0, K = 0, KS = 0, L = 0;
    const uint16_t *codes = nullptr;
    const uint8_t *labels = nullptr;
    const uint16_t *nbins = nullptr;
    std::unique_ptr<DevModel> m;
    ClassRows cls[2];
    uint64_t M[2] = {0, 0};
    Scratch<uint32_t> err, pos, counts;
    uint64_t pairs() const {
        return (uint64_t)cls[0].n * (cls[0].n ? cls[0].n - 1 : 0) / 2 +
               (uint64_t)cls[1].n * (cls[1].n ? cls[1].n - 1 : 0) / 2;
    }
};

struct GraphGuard {
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    ~GraphGuard() {
        if (x) (void)hipGraphExecDestroy(x);
        if (g) (void)hipGraphDestroy(g);
    }
};

// Enumeration, one radix sort, one de-duplication and one coherence launch for
// every (problem, class) of the group, captured and launched as one graph; then
// ordering and support per problem.  All problems have the same KS.
static void run_group(std::vector<BProb *> &G, const ig_fit_opts *opts, hipStream_t s) {
    const uint32_t KS = G[0]->KS;
    const uint32_t nseg = 2 * (uint32_t)G.size();
    int segbits = 1;
    while ((1u << segbits) < nseg) ++segbits;
    std::vector<uint64_t> off(nseg + 1, 0);
    uint32_t max_other = 1;
    uint64_t group_pairs = 0;
    for (uint32_t g = 0; g < G.size(); ++g) {
        for (int c = 0; c < 2; ++c) {
            const uint32_t sg = 2 * g + c;
            off[sg + 1] = off[sg] + G[g]->M[c];
            max_other = std::max(max_other, G[g]->cls[1 - c].n);
        }
        group_pairs += G[g]->pairs();
    }
    const size_t items = off[nseg];
    IG_REQUIRE(items < (1ull << 32), IG_E_UNSUPPORTED, "group of more than 2^32 candidates");
    const Tuning tu = tuning_for(opts, KS, group_pairs / std::max<size_t>(G.size(), 1));
    const size_t cap = std::max<size_t>(items, 1);
    Scratch<uint64_t> k0(cap, s), k1(cap, s);
    Scratch<uint32_t> v0(cap, s), v1(cap, s), flags(cap, s), pos(cap, s), cand(cap, s), surv(cap, s);
    Scratch<uint32_t> tot(1, s), segc(nseg, s), segoff(nseg, s), cnt(nseg + 1, s);
    Scratch<unsigned long long> tests(nseg, s);
    Scratch<uint32_t> rws(radix_ws_size(cap), s), sws(scan_ws_size(cap), s);
    Scratch<unsigned char> rowsegs(nseg * rows_of_seg_size(), s);
    Scratch<CohSeg> cohsegs(nseg, s);
    // per problem: matrix-core operands when its subset tests run there; their
    // segments then give the captured VALU coherence no candidates (a zero count)
    const uint32_t mode = opts ? opts->coherence_mfma : 0u;
    std::vector<MfmaFit> mf(G.size());
    for (uint32_t g = 0; g < G.size(); ++g) {
        mfma_setup(*G[g]->m, G[g]->cls, mode, opts ? opts->fit_dense : 0u, mf[g], s);
        if (mf[g].on) {
            note_fit_operands(*G[g]->m, mf[g]);
            G[g]->m->fit_buckets = mf[g].pruned;
        }
    }
    Scratch<uint32_t> zero(1, s);
    {
        std::vector<unsigned char> hr(nseg * rows_of_seg_size());
        std::vector<CohSeg> hc(nseg);
        for (uint32_t g = 0; g < G.size(); ++g)
            for (int c = 0; c < 2; ++c) {
                const uint32_t sg = 2 * g + c;
                fill_rows_of_seg(hr.data() + sg * rows_of_seg_size(), G[g]->cls[c].X.get(), G[g]->cls[c].n, KS,
                                 G[g]->K);
                CohSeg &h = hc[sg];
                h = CohSeg{};
                h.X = G[g]->cls[c].X.get();
                h.NXo = G[g]->cls[1 - c].NX.get();
                h.cand = cand.get();
                h.cand_off = segoff.get() + sg;
                h.ncand = mf[g].on ? zero.get() : segc.get() + sg;
                h.out = surv.get() + off[sg];
                h.nout = cnt.get() + sg;
                h.tests = tests.get() + sg;
                h.n = G[g]->cls[c].n;
                h.n_o = G[g]->cls[1 - c].n;
            }
        upload(rowsegs.get(), hr.data(), hr.size(), s);
        upload(cohsegs.get(), hc.data(), hc.size() * sizeof(CohSeg), s);
        IG_HIP(hipStreamSynchronize(s));   // nothing may be in flight on s when capture begins
    }
    const uint32_t grid = coherence_grid(tu.grid_per_cu);
    // the segment bits and as many hash bits as a single fit's keys, whole bytes
    const int batch_key_bytes = std::min(8, (segbits + kSortHashBits + 7) / 8);
    GraphGuard gg;
    IG_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    try {
        launch_fill_u32(cnt.get(), 0u, nseg + 1, s);
        launch_fill_u32(zero.get(), 0u, 1, s);
        launch_fill_u64(reinterpret_cast<uint64_t *>(tests.get()), 0ull, nseg, s);
        for (uint32_t g = 0; g < G.size(); ++g)
            for (int c = 0; c < 2; ++c) {
                const uint32_t sg = 2 * g + c;
                launch_pair_hash(G[g]->cls[c].X.get(), G[g]->cls[c].n, KS, G[g]->K, 0, G[g]->M[c], sg, segbits,
                                 k0.get() + off[sg], v0.get() + off[sg], s, batch_key_bytes);
            }
        const int where = radix_sort_pairs(k0.get(), v0.get(), k1.get(), v1.get(), items,
                                           0xffu & ~((1u << (8 - batch_key_bytes)) - 1), s, rws.get());
        uint64_t *ks = where ? k1.get() : k0.get();
        uint32_t *vs = where ? v1.get() : v0.get();
        launch_dedup_flags(ks, vs, items, rowsegs.get(), segbits, flags.get(), nullptr, s);
        scan_exclusive_u32(flags.get(), pos.get(), items, tot.get(), s, sws.get());
        launch_seg_counts(ks, items, pos.get(), tot.get(), segbits, nseg, segc.get(), s, segoff.get());
        launch_compact(flags.get(), pos.get(), vs, items, cand.get(), s);
        launch_coherence((int)KS, tu.cpl, cohsegs.get(), nseg, 0, max_other, cnt.get() + nseg, grid, s);
    } catch (...) {
        hipGraph_t dead = nullptr;
        (void)hipStreamEndCapture(s, &dead);
        if (dead) (void)hipGraphDestroy(dead);
        throw;
    }
    IG_HIP(hipStreamEndCapture(s, &gg.g));
    IG_HIP(hipGraphInstantiate(&gg.x, gg.g, nullptr, nullptr, 0));
    hipEvent_t e0, e1;
    IG_HIP(hipEventCreate(&e0));
    IG_HIP(hipEventCreate(&e1));
    IG_HIP(hipEventRecord(e0, s));
    IG_HIP(hipGraphLaunch(gg.x, s));
    IG_HIP(hipEventRecord(e1, s));
    IG_HIP(hipStreamSynchronize(s));
    float graph_ms = 0;
    (void)hipEventElapsedTime(&graph_ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    std::vector<uint32_t> hdist = host_read_u32(segc.get(), nseg, s);
    std::vector<uint32_t> hsurv = host_read_u32(cnt.get(), nseg, s);
    std::vector<uint32_t> hoff = host_read_u32(segoff.get(), nseg, s);
    std::vector<unsigned long long> htests(nseg);
    IG_HIP(hipMemcpyAsync(htests.data(), tests.get(), nseg * 8, hipMemcpyDeviceToHost, s));
    IG_HIP(hipStreamSynchronize(s));
    // coherence on the matrix cores for the problems that use them (dense counts)
    std::vector<float> mfma_ms(G.size(), 0.0f), mfma_kernel(G.size(), 0.0f);
    for (uint32_t g = 0; g < G.size(); ++g) {
        if (!mf[g].on) continue;
        const auto t0 = std::chrono::steady_clock::now();
        Tuning tg = tuning_for(opts, KS, G[g]->pairs());
        mfma_tuning(opts, mf[g].KO, G[g]->pairs(), tg);
        for (int c = 0; c < 2; ++c) {
            const uint32_t sg = 2 * g + c;
            uint64_t t = 0;
            hsurv[sg] = mfma_coherence(mf[g], G[g]->cls, c, KS, cand.get() + hoff[sg], hdist[sg],
                                       surv.get() + off[sg], &mfma_kernel[g], s, nullptr, nullptr, tg.coh_sets,
                                       &t);
            htests[sg] = (unsigned long long)t;
        }
        mfma_ms[g] = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    for (uint32_t g = 0; g < G.size(); ++g) {
        DevModel &m = *G[g]->m;
        Tuning tp = tuning_for(opts, KS, G[g]->pairs());
        if (mf[g].on) mfma_tuning(opts, mf[g].KO, G[g]->pairs(), tp);
        Timer tm(s);
        tm.mark(4);
        PatternRows prow;
        for (int c = 0; c < 2; ++c) {
            const uint32_t sg = 2 * g + c;
            m.stats.n_class[c] = G[g]->cls[c].n;
            m.stats.pairs[c] = G[g]->M[c] - G[g]->cls[c].n;
            m.stats.distinct[c] = hdist[sg];
            m.stats.tests[c] = htests[sg];
            m.stats.chunks[c] = G[g]->M[c] ? 1 : 0;
            order_and_weigh(m, c, G[g]->cls[c], surv.get() + off[sg], hsurv[sg], false, tp, s, &tm,
                            c == 0 ? 5 : 8, mf[g].on ? mf[g].frag[1 - c].get() : nullptr, mf[g].view, &prow,
                            nullptr, mf[g].on ? &mf[g] : nullptr);
            m.stats.coherent[c] = m.np[c];
            if (c == 0) tm.mark(3);
        }
        tm.mark(6);
        finish_weights(m, s, &prow, G[g]->cls);
        tm.mark(7);
        mf[g].finish(s);
        mf[g].put_tests(m);
        record_times(m, tm);
        // the group's captured stages, split by this problem's share of the pairs
        const double share = group_pairs ? (double)G[g]->pairs() / (double)group_pairs : 0.0;
        m.stats.ms[4] = (float)(graph_ms * share) + mfma_ms[g];
        m.stats.ms[1] = m.stats.ms[2] = m.stats.ms[3] = 0.0f;
        mf[g].clock.collect();
        m.stats.kernel_ms[0] = mfma_kernel[g];
    }
}

void fit_batch(const ig_problem *probs, uint32_t np, const ig_fit_opts *opts, hipStream_t user,
               std::vector<DevModel *> &out) {
    std::vector<BProb> P(np);
    for (uint32_t p = 0; p < np; ++p) {
        BProb &b = P[p];
        uint32_t L, K;
        check_nbins(probs[p].h_nbins, probs[p].d, L, K);
        IG_REQUIRE(probs[p].n == 0 || (probs[p].d_codes && probs[p].d_labels), IG_E_INVAL,
                   "problem " + std::to_string(p) + ": codes or labels is NULL");
        b.n = probs[p].n;
        b.d = probs[p].d;
        b.L = L;
        b.K = K;
        b.KS = (uint32_t)storage_words((int)K);
        b.codes = probs[p].d_codes;
        b.labels = probs[p].d_labels;
        b.nbins = probs[p].h_nbins;
    }
    IG_HIP(hipStreamSynchronize(user));   // inputs produced on the caller's stream are complete
    std::lock_guard<std::mutex> lock(g_batch_mu);
    hipStream_t s = internal_stream();
    // validate, split and pack every problem (one synchronisation for all checks)
    for (auto &b : P) {
        b.m.reset(new_model());
        b.m->K = b.K;
        b.m->KS = b.KS;
        b.m->L = b.L;
        b.m->d = b.d;
        std::vector<uint32_t> tab = token_tables(b.nbins, b.d, b.KS);
        b.m->meta = dev_alloc<uint32_t>(tab.size());
        b.m->nbins = dev_alloc<uint16_t>(b.d);
        upload(b.m->meta, tab.data(), tab.size() * 4, s);
        upload(b.m->nbins, b.nbins, b.d * 2, s);
        set_key_pieces(*b.m, b.nbins, b.d, s);
        set_factor_table(*b.m, b.nbins, b.d, s);
        set_factor_table(*b.m, b.nbins, b.d, s, true);
        b.err.reset(1, s);
        b.pos.reset(b.n ? b.n : 1, s);
        b.counts.reset(2, s);
        launch_fill_u32(b.err.get(), 0u, 1, s);
        launch_fill_u32(b.counts.get(), 0u, 2, s);
        launch_validate_codes(b.codes, (size_t)b.n * b.d, b.d, b.m->nbins, b.err.get(), s);
        if (b.n) launch_split_labels(b.labels, b.n, b.pos.get(), b.counts.get(), b.err.get(), s);
    }
    std::vector<uint32_t> herr(np), hcnt(2 * (size_t)np);
    for (uint32_t p = 0; p < np; ++p) {
        IG_HIP(hipMemcpyAsync(&herr[p], P[p].err.get(), 4, hipMemcpyDeviceToHost, s));
        IG_HIP(hipMemcpyAsync(&hcnt[2 * p], P[p].counts.get(), 8, hipMemcpyDeviceToHost, s));
    }
    IG_HIP(hipStreamSynchronize(s));
    for (uint32_t p = 0; p < np; ++p) {
        IG_REQUIRE(!(herr[p] & 1u), IG_E_INVAL, "problem " + std::to_string(p) + ": a code is not below its bin count");
        IG_REQUIRE(!(herr[p] & 2u), IG_E_INVAL, "problem " + std::to_string(p) + ": a label is not 0 or 1");
        IG_REQUIRE(hcnt[2 * p] <= 92000 && hcnt[2 * p + 1] <= 92000, IG_E_UNSUPPORTED,
                   "problem " + std::to_string(p) + ": more than 92,000 training records in one class");
    }
    for (uint32_t p = 0; p < np; ++p) {
        BProb &b = P[p];
        alloc_class_rows(b.cls, &hcnt[2 * p], b.KS, s);
        launch_pack_split(b.codes, b.labels, b.n, b.d, b.KS, b.m->meta, b.pos.get(), b.cls[0].X.get(),
                          b.cls[1].X.get(), b.cls[0].NX.get(), b.cls[1].NX.get(), s);
        for (int c = 0; c < 2; ++c) {
            const uint64_t n = b.cls[c].n;
            b.M[c] = n + n * (n ? n - 1 : 0) / 2;
        }
    }
    // groups: same storage width, at most 64 problems, bounded scratch
    uint64_t group_items = 1ull << 30;
    if (opts && opts->mem_budget_bytes) group_items = std::max<uint64_t>(opts->mem_budget_bytes / 40, 4096);
    std::vector<uint32_t> order(np);
    for (uint32_t p = 0; p < np; ++p) order[p] = p;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return P[a].KS < P[b].KS; });
    std::vector<BProb *> G;
    uint64_t G_items = 0;
    auto flush = [&]() {
        if (!G.empty()) run_group(G, opts, s);
        G.clear();
        G_items = 0;
    };
    for (uint32_t idx : order) {
        BProb &b = P[idx];
        const uint64_t it = b.M[0] + b.M[1];
        if (it > group_items) {   // on its own, with the plain (chunking) path
            Timer tm(s);
            tm.mark(0);
            fit_from_rows(*b.m, b.cls, opts, s, tm);
            record_times(*b.m, tm);
            continue;
        }
        if (!G.empty() && (G[0]->KS != b.KS || G.size() == 64 || G_items + it > group_items)) flush();
        G.push_back(&b);
        G_items += it;
    }
    flush();
    IG_HIP(hipStreamSynchronize(s));
    for (auto &b : P) out.push_back(b.m.release());
}
}  // namespace ig

// ===================================================================== C ABI ====
using ig::DevModel;

struct ig_model {
    DevModel *m;
};

template <class F>
static ig_status guarded(F &&fn) {
    try {
        fn();
        ig::g_last_error.clear();
        return IG_OK;
    } catch (const ig::Error &e) {
        ig::set_error(e.what());
        return e.code;
    } catch (const std::bad_alloc &) {
        ig::set_error("host allocation failed");
        return IG_E_NOMEM;
    } catch (const std::exception &e) {
        ig::set_error(e.what());
        return IG_E_DEVICE;
    }
}

static ig_model *wrap(DevModel *m) {
    ig_model *w = new (std::nothrow) ig_model{m};
    if (!w) {
        delete m;
        throw ig::Error(IG_E_NOMEM, "host allocation failed");
    }
    return w;
}

static void check_model(const ig_model *m) {
    IG_REQUIRE(m && m->m, IG_E_INVAL, "model is NULL");
    int dev = 0;
    IG_HIP(hipGetDevice(&dev));
    IG_REQUIRE(dev == m->m->device, IG_E_INVAL, "model lives on another device than the current one");
}

extern "C" {

ig_status ig_fit(const uint16_t *d_codes, const uint8_t *d_labels, uint32_t n, uint32_t d, const uint16_t *h_nbins,
                 const ig_fit_opts *opts, void *stream, ig_model **out) {
    return guarded([&] {
        IG_REQUIRE(out != nullptr, IG_E_INVAL, "out is NULL");
        ig::UserAllocScope scope(opts ? opts->alloc : nullptr);
        DevModel *m = ig::fit_codes(d_codes, d_labels, n, d, h_nbins, opts, (hipStream_t)stream);
        *out = wrap(m);
    });
}

ig_status ig_fit_packed(const uint64_t *d_words, const uint8_t *d_labels, uint32_t n, uint32_t K,
                        const ig_fit_opts *opts, void *stream, ig_model **out) {
    return guarded([&] {
        IG_REQUIRE(out != nullptr, IG_E_INVAL, "out is NULL");
        ig::UserAllocScope scope(opts ? opts->alloc : nullptr);
        DevModel *m = ig::fit_packed(d_words, d_labels, n, K, opts, (hipStream_t)stream);
        *out = wrap(m);
    });
}

ig_status ig_fit_batch(const ig_problem *probs, uint32_t n_probs, const ig_fit_opts *opts, void *stream,
                       ig_model **outs) {
    return guarded([&] {
        IG_REQUIRE(outs != nullptr && (n_probs == 0 || probs != nullptr), IG_E_INVAL, "NULL argument");
        ig::UserAllocScope scope(opts ? opts->alloc : nullptr);
        std::vector<DevModel *> made;
        try {
            ig::fit_batch(probs, n_probs, opts, (hipStream_t)stream, made);
        } catch (...) {
            for (auto *m : made) delete m;
            throw;
        }
        std::vector<ig_model *> w(n_probs, nullptr);
        for (uint32_t p = 0; p < n_probs; ++p) w[p] = new (std::nothrow) ig_model{made[p]};
        bool ok = std::all_of(w.begin(), w.end(), [](ig_model *x) { return x != nullptr; });
        if (!ok) {
            for (uint32_t p = 0; p < n_probs; ++p) {
                delete made[p];
                delete w[p];
            }
            throw ig::Error(IG_E_NOMEM, "host allocation failed");
        }
        for (uint32_t p = 0; p < n_probs; ++p) outs[p] = w[p];
    });
}

ig_status ig_model_digest(const ig_model *m, uint32_t cls, uint64_t *out) {
    return guarded([&] {
        check_model(m);
        IG_REQUIRE(cls <= 1 && out, IG_E_INVAL, "class must be 0 or 1 and out non-NULL");
        const DevModel &M = *m->m;
        hipStream_t s = nullptr;
        ig::Scratch<unsigned long long> d(1, s);
        ig::launch_digest(M.W[cls], M.f[cls], M.S[cls], M.np[cls], M.KS, M.K, d.get(), s);
        unsigned long long h = 0;
        IG_HIP(hipMemcpyAsync(&h, d.get(), 8, hipMemcpyDeviceToHost, s));
        IG_HIP(hipStreamSynchronize(s));
        *out = h;
    });
}

static ig::ScoreModel score_model(const ig::DevModel &M) {
    ig::ScoreModel sm{};
    for (int c = 0; c < 2; ++c) {
        sm.P[c] = M.W[c];
        sm.S[c] = M.S[c];
        sm.np[c] = M.np[c];
        sm.maxS[c] = M.maxS[c];
        sm.frag[c] = M.frag[c];
        sm.ftiles[c] = M.ftiles[c];
        sm.btile[c] = M.btile[c];
    }
    sm.nbucket = (M.btile[0] && M.btile[1]) ? M.L : 0u;
    sm.KS = M.KS;
    const ig::FactorView &sv = M.score_ternary ? M.tv : M.fv;
    sm.KO = M.score_factored ? sv.KF : M.KS;
    if (M.score_factored) sm.fv = sv;
    sm.spare = M.score_spare;
    sm.tslots = M.score_ternary ? ig::tern_bias_slots(M.tern_tokens) : 0u;
    return sm;
}

ig_status ig_score_ex(const ig_model *m, const uint16_t *d_codes, uint32_t n_flows, int64_t *d_out, uint32_t mode,
                      void *stream) {
    return guarded([&] {
        check_model(m);
        const DevModel &M = *m->m;
        IG_REQUIRE(M.d > 0, IG_E_INVAL, "model was fitted from packed words: use ig_score_packed");
        IG_REQUIRE(n_flows < (1u << 31), IG_E_UNSUPPORTED, "n_flows must be below 2^31");
        IG_REQUIRE(n_flows == 0 || (d_codes && d_out), IG_E_INVAL, "codes or out is NULL");
        IG_REQUIRE(mode <= IG_SCORE_PRUNED, IG_E_INVAL, "unknown scoring mode");
        const ig::ScoreModel sm = score_model(M);
        hipStream_t s = (hipStream_t)stream;
        const bool mfma = M.frag[0] && M.frag[1];
        IG_REQUIRE(mode != IG_SCORE_PRUNED || (mfma && sm.nbucket), IG_E_UNSUPPORTED,
                   "the model's scoring tiles are not grouped by token");
        if (mfma && sm.nbucket && mode != IG_SCORE_DENSE) {
            ig::Scratch<uint32_t> ws(ig::prune_scratch_words(sm.nbucket, n_flows, M.d, sm.KO), s);
            if (ig::launch_score_mfma_pruned(sm, d_codes, n_flows, M.d, M.meta, M.nbins, d_out, ws.get(), s)) return;
            IG_REQUIRE(mode != IG_SCORE_PRUNED, IG_E_UNSUPPORTED, "too many flows for one pruned scoring launch");
        }
        if (mfma)
            ig::launch_score_mfma(sm, d_codes, nullptr, M.K, n_flows, M.d, M.meta, M.nbins, d_out, s);
        else
            ig::launch_score(sm, d_codes, nullptr, M.K, n_flows, M.d, M.meta, M.nbins, d_out, 2, s);
    });
}

ig_status ig_score(const ig_model *m, const uint16_t *d_codes, uint32_t n_flows, int64_t *d_out, void *stream) {
    return ig_score_ex(m, d_codes, n_flows, d_out, IG_SCORE_AUTO, stream);
}

ig_status ig_score_noalloc(const ig_model *m, const uint16_t *d_codes, uint32_t n_flows, int64_t *d_out,
                           void *stream) {
    return guarded([&] {
        check_model(m);
        const DevModel &M = *m->m;
        IG_REQUIRE(M.d > 0, IG_E_INVAL, "model was fitted from packed words: use ig_score_packed");
        IG_REQUIRE(n_flows < (1u << 31), IG_E_UNSUPPORTED, "n_flows must be below 2^31");
        IG_REQUIRE(n_flows == 0 || (d_codes && d_out), IG_E_INVAL, "codes or out is NULL");
        const ig::ScoreModel sm = score_model(M);
        hipStream_t s = (hipStream_t)stream;
        const bool mfma = M.frag[0] && M.frag[1];
        if (mfma && sm.nbucket) {
            const size_t need = ig::prune_scratch_words(sm.nbucket, n_flows, M.d, sm.KO);
            const size_t have = ig::noalloc_scratch_words();
            IG_REQUIRE(need <= have, IG_E_UNSUPPORTED,
                       "the call's " + std::to_string(need) + " words of scratch exceed the fixed array of " +
                           std::to_string(have) + " words (IG_NOALLOC_SCRATCH_BYTES)");
            if (ig::launch_score_mfma_pruned(sm, d_codes, n_flows, M.d, M.meta, M.nbins, d_out,
                                             ig::noalloc_scratch(), s))
                return;
        }
        if (mfma)
            ig::launch_score_mfma(sm, d_codes, nullptr, M.K, n_flows, M.d, M.meta, M.nbins, d_out, s);
        else
            ig::launch_score(sm, d_codes, nullptr, M.K, n_flows, M.d, M.meta, M.nbins, d_out, 2, s);
    });
}

ig_status ig_score_packed(const ig_model *m, const uint64_t *d_words, uint32_t n_flows, int64_t *d_out,
                          void *stream) {
    return guarded([&] {
        check_model(m);
        const DevModel &M = *m->m;
        IG_REQUIRE(n_flows < (1u << 31), IG_E_UNSUPPORTED, "n_flows must be below 2^31");
        IG_REQUIRE(n_flows == 0 || (d_words && d_out), IG_E_INVAL, "words or out is NULL");
        const ig::ScoreModel sm = score_model(M);
        // words may hold several bins of a feature: factored operands cannot test them
        if (M.frag[0] && M.frag[1] && !M.score_factored)
            ig::launch_score_mfma(sm, nullptr, d_words, M.K, n_flows, M.d, M.meta, M.nbins, d_out, (hipStream_t)stream);
        else
            ig::launch_score(sm, nullptr, d_words, M.K, n_flows, M.d, M.meta, M.nbins, d_out, 2, (hipStream_t)stream);
    });
}

ig_status ig_evidence(const ig_model *m, const uint16_t *d_codes, uint32_t n_flows, uint32_t k, uint32_t *d_count,
                      uint64_t *d_words, uint32_t *d_f, int64_t *d_S, void *stream) {
    return guarded([&] {
        check_model(m);
        const DevModel &M = *m->m;
        IG_REQUIRE(M.d > 0, IG_E_INVAL, "model was fitted from packed words: flows are given as codes");
        IG_REQUIRE(k >= 1 && k <= ig::evidence_max_k(), IG_E_INVAL, "k must be in 1..256");
        IG_REQUIRE(n_flows < (1u << 31), IG_E_UNSUPPORTED, "n_flows must be below 2^31");
        IG_REQUIRE(n_flows == 0 || (d_codes && d_count && d_words && d_f && d_S), IG_E_INVAL, "NULL argument");
        IG_REQUIRE(M.np[0] < (1ull << 32) && M.np[1] < (1ull << 32), IG_E_UNSUPPORTED,
                   "more than 2^32 patterns in one class");
        ig::EvidenceModel em{};
        for (int c = 0; c < 2; ++c) {
            em.W[c] = M.W[c];
            em.f[c] = M.f[c];
            em.S[c] = M.S[c];
            em.np[c] = M.np[c];
            em.bperm[c] = (M.bperm[0] && M.bperm[1]) ? M.bperm[c] : nullptr;
            em.brow[c] = (M.bperm[0] && M.bperm[1]) ? M.brow[c] : nullptr;
        }
        em.KS = M.KS;
        em.K = M.K;
        em.d = M.d;
        em.off = M.meta;
        em.nbins = M.nbins;
        ig::launch_evidence(em, d_codes, n_flows, k, d_count, d_words, d_f, d_S, (hipStream_t)stream);
    });
}

ig_status ig_normal_moments(const int64_t *d_scores, const uint8_t *d_labels, uint32_t n, ig_moments *out,
                            void *stream) {
    return guarded([&] {
        IG_REQUIRE(out && (n == 0 || (d_scores && d_labels)), IG_E_INVAL, "NULL argument");
        ig_moments mo{};
        if (n) ig::normal_moments(d_scores, d_labels, n, &mo, (hipStream_t)stream);
        *out = mo;
    });
}

ig_status ig_r3_threshold(const ig_moments *m, double r, int64_t *out) {
    return guarded([&] {
        IG_REQUIRE(m && out, IG_E_INVAL, "NULL argument");
        *out = ig::r3_threshold(*m, r);
    });
}

ig_status ig_classify(const int64_t *d_scores, uint32_t n, int64_t r3_threshold, uint32_t flags, uint8_t *d_label,
                      uint8_t *d_rule, void *stream) {
    return guarded([&] {
        IG_REQUIRE(n == 0 || (d_scores && d_label), IG_E_INVAL, "scores or labels is NULL");
        IG_REQUIRE(!(flags & ~(IG_CLASSIFY_R3 | IG_CLASSIFY_NO_R2)), IG_E_INVAL, "unknown classify flags");
        ig::classify(d_scores, n, r3_threshold, flags, d_label, d_rule, (hipStream_t)stream);
    });
}

ig_status ig_detection_metrics(const int64_t *d_scores, const uint8_t *d_pred, const uint8_t *d_truth, uint32_t n,
                               ig_metrics *out, void *stream) {
    return guarded([&] {
        IG_REQUIRE(out && (n == 0 || (d_scores && d_pred && d_truth)), IG_E_INVAL, "NULL argument");
        IG_REQUIRE(n < (1u << 31), IG_E_UNSUPPORTED, "n must be below 2^31");
        ig_metrics mt{};
        ig::detection_metrics(d_scores, d_pred, d_truth, n, &mt, (hipStream_t)stream);
        *out = mt;
    });
}

ig_status ig_model_bucket_sizes(const ig_model *m, uint32_t cls, uint32_t *h_counts) {
    return guarded([&] {
        check_model(m);
        IG_REQUIRE(cls <= 1 && h_counts, IG_E_INVAL, "class must be 0 or 1 and h_counts non-NULL");
        const DevModel &M = *m->m;
        IG_REQUIRE(M.brow[0] && M.brow[1], IG_E_UNSUPPORTED, "the model has no token buckets");
        std::vector<uint32_t> br(M.L + 1);
        IG_HIP(hipMemcpy(br.data(), M.brow[cls], (M.L + 1) * 4, hipMemcpyDeviceToHost));
        for (uint32_t u = 0; u < M.L; ++u) h_counts[u] = br[u + 1] - br[u];
    });
}

ig_status ig_model_get_info(const ig_model *m, ig_model_info *info) {
    return guarded([&] {
        IG_REQUIRE(m && m->m && info, IG_E_INVAL, "model or info is NULL");
        const DevModel &M = *m->m;
        std::memset(info, 0, sizeof(*info));
        info->K = M.K;
        info->L = M.L;
        info->d = M.d;
        info->flags = ((M.frag[0] && M.frag[1]) ? IG_MODEL_SCORE_MFMA : 0u) |
                      (M.score_factored ? IG_MODEL_FACTORED : 0u) |
                      ((M.frag[0] && M.frag[1] && M.btile[0] && M.btile[1]) ? IG_MODEL_BUCKETED : 0u) |
                      (M.fit_buckets ? IG_MODEL_FIT_BUCKETS : 0u);
        info->mfma_tokens = M.score_ternary ? M.tern_tokens : M.score_factored ? M.fac_tokens : M.L;
        info->mfma_words = M.score_ternary ? M.tv.KF : M.score_factored ? M.fv.KF : M.K;
        info->fit_tokens = M.fit_tokens;
        info->fit_words = M.fit_words;
        for (int c = 0; c < 2; ++c) {
            info->n_patterns[c] = M.np[c];
            info->max_weight[c] = M.maxS[c];
        }
    });
}

ig_status ig_model_export(const ig_model *m, uint32_t cls, uint64_t *h_words, uint32_t *h_f, int64_t *h_S) {
    return guarded([&] {
        check_model(m);
        IG_REQUIRE(cls <= 1, IG_E_INVAL, "class must be 0 or 1");
        const DevModel &M = *m->m;
        const uint64_t n = M.np[cls];
        if (!n || !(h_words || h_f || h_S)) return;
        IG_REQUIRE(n < (1ull << 32), IG_E_UNSUPPORTED, "more than 2^32 patterns in one class");
        // rows in canonical order, sorted on the device
        hipStream_t s = nullptr;
        ig::Scratch<uint32_t> perm(n, s), fo(n, s);
        // rows gathered in order and cut to K words on the device: one contiguous copy
        ig::Scratch<uint64_t> rows(n * M.K, s), So(n, s);
        ig::canonical_permutation(M, M.W[cls], 0, nullptr, n, perm.get(), s);
        ig::launch_gather_rows(M.W[cls], perm.get(), n, M.KS, M.K, rows.get(), M.f[cls], fo.get(), s);
        ig::launch_permute_u64(reinterpret_cast<const uint64_t *>(M.S[cls]), perm.get(), n, So.get(), s);
        IG_HIP(hipStreamSynchronize(s));
        if (h_words) IG_HIP(hipMemcpy(h_words, rows.get(), n * M.K * 8, hipMemcpyDeviceToHost));
        if (h_f) IG_HIP(hipMemcpy(h_f, fo.get(), n * 4, hipMemcpyDeviceToHost));
        if (h_S) IG_HIP(hipMemcpy(h_S, So.get(), n * 8, hipMemcpyDeviceToHost));
    });
}

ig_status ig_model_import(const uint16_t *const h_codes[2], const uint32_t *const h_f[2], const uint64_t count[2],
                          uint32_t d, const uint16_t *h_nbins, void *stream, ig_model **out) {
    return guarded([&] {
        IG_REQUIRE(out && h_codes && h_f && count, IG_E_INVAL, "NULL argument");
        DevModel *m = ig::import_patterns(h_codes, h_f, count, d, h_nbins, (hipStream_t)stream);
        *out = wrap(m);
    });
}

ig_status ig_fit_stats(const ig_model *m, ig_stats *out) {
    return guarded([&] {
        IG_REQUIRE(m && m->m && out, IG_E_INVAL, "model or out is NULL");
        *out = m->m->stats;
    });
}

void ig_model_free(ig_model *m) {
    if (!m) return;
    delete m->m;
    delete m;
}

ig_status ig_release_memory(void) {
    return guarded([&] { ig::release_memory(); });
}

ig_status ig_memory_stats(uint64_t *reserved, uint64_t *in_use, uint64_t *cached) {
    return guarded([&] {
        IG_REQUIRE(reserved && in_use && cached, IG_E_INVAL, "NULL argument");
        ig::memory_stats(reserved, in_use, cached);
    });
}

const char *ig_last_error(void) { return ig::g_last_error.c_str(); }

const char *ig_version(void) { return "libig 0.2 (gfx950)"; }

ig_status ig_probe_mfma_fp4(uint32_t iters, void *stream, double *ops_per_s, float *ms) {
    return guarded([&] {
        IG_REQUIRE(ops_per_s != nullptr, IG_E_INVAL, "ops_per_s is NULL");
        *ops_per_s = ig::probe_mfma_fp4(iters, (hipStream_t)stream, ms);
    });
}

ig_status ig_probe_hbm_copy(const void *d_src, void *d_dst, size_t bytes, void *stream, double *bytes_per_s,
                            float *ms) {
    return guarded([&] {
        IG_REQUIRE(bytes_per_s != nullptr, IG_E_INVAL, "bytes_per_s is NULL");
        const uintptr_t a = (uintptr_t)d_src, b = (uintptr_t)d_dst;
        IG_REQUIRE(a + bytes <= b || b + bytes <= a, IG_E_INVAL, "source and destination overlap");
        *bytes_per_s = ig::probe_copy(d_src, d_dst, bytes, (hipStream_t)stream, ms);
    });
}

}  // extern "C"
