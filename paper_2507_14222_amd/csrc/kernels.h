// Launchers of libig's kernels (host-side declarations).
#pragma once
#include "common.h"

namespace ig {

// pack.hip
void launch_validate_codes(const uint16_t *codes, size_t total, uint32_t d, const uint16_t *nbins, uint32_t *err,
                           hipStream_t s);
void launch_split_labels(const uint8_t *labels, uint32_t n, uint32_t *pos, uint32_t *counts, uint32_t *err,
                         hipStream_t s);
void launch_pack_split(const uint16_t *codes, const uint8_t *labels, uint32_t n, uint32_t d, uint32_t KS,
                       const uint32_t *meta, const uint32_t *pos, uint64_t *X0, uint64_t *X1, uint64_t *NX0,
                       uint64_t *NX1, hipStream_t s);
void launch_split_packed(const uint64_t *words, const uint8_t *labels, uint32_t n, uint32_t K, uint32_t KS,
                         const uint32_t *pos, uint64_t *X0, uint64_t *X1, uint64_t *NX0, uint64_t *NX1,
                         hipStream_t s);
void launch_pack_patterns(const uint16_t *codes, uint32_t m, uint32_t d, uint32_t KS, const uint32_t *meta,
                          const uint16_t *nbins, uint64_t *W, uint32_t *err, hipStream_t s);

// pairs.hip
// key_bytes: only the top key_bytes bytes of each key are kept (the rest zero), so a
// radix sort needs only that many passes; equal keys are compared in full anyway.
void launch_pair_hash(const uint64_t *X, uint32_t n, uint32_t KS, uint32_t K, uint64_t q0, uint64_t count,
                      uint32_t seg, int segbits, uint64_t *keys, uint32_t *vals, hipStream_t s, int key_bytes = 8);
// De-duplication with a partial sort (see pairs.hip) over the pair ids [q0c, q0c +
// cntc) of both classes' records Xc: cand [cnt0 + cnt1] = the distinct candidates'
// pair ids (the first occurrence of each), class 0's then class 1's; total and
// seg_counts [2] their numbers; *err set when the hashes could not tell two
// candidates apart or a partition had too many distinct keys (then use the full
// sort).
bool dedup_partitioned_fits(uint64_t items);
void launch_dedup_partitioned(const uint64_t *X0, uint32_t n0, uint64_t q00, uint64_t cnt0, const uint64_t *X1,
                              uint32_t n1, uint64_t q01, uint64_t cnt1, uint32_t KS, uint32_t K, uint32_t *cand,
                              uint32_t *total, uint32_t *seg_counts, uint32_t *err, hipStream_t s);
size_t rows_of_seg_size();
void fill_rows_of_seg(void *dst, const uint64_t *X, uint32_t n, uint32_t KS, uint32_t K);
void launch_dedup_flags(const uint64_t *keys, const uint32_t *vals, size_t m, const void *segs_dev, int segbits,
                        uint32_t *flags, uint32_t *seg_counts, hipStream_t s);
// distinct candidates per segment from the exclusive scan `pos` (and its total)
void launch_seg_counts(const uint64_t *keys, size_t m, const uint32_t *pos, const uint32_t *total, int segbits,
                       uint32_t nseg, uint32_t *seg_counts, hipStream_t s, uint32_t *seg_offsets = nullptr);
// out[pos[e]] = vals[e] for the flagged e (and idx[pos[e]] = e when idx is given);
// with perm, element e stands for perm[e]: out[pos[e]] = vals[perm[e]], idx = perm[e]
void launch_compact(const uint32_t *flags, const uint32_t *pos, const uint32_t *vals, size_t m, uint32_t *out,
                    hipStream_t s, uint32_t *idx = nullptr, const uint32_t *perm = nullptr);
void launch_gather_word(const uint64_t *X, uint32_t n, uint32_t KS, uint32_t k, const uint32_t *ids, size_t m,
                        uint64_t *keys, hipStream_t s);
void launch_word_range(const uint64_t *X, uint32_t n, uint32_t KS, uint32_t K, const uint32_t *ids, size_t m,
                       unsigned long long *orv, unsigned long long *andv, hipStream_t s);
// With len (no newflag): also the token count of each row when the row width allows
// (returns whether len was written).
bool launch_materialize(const uint64_t *X, uint32_t n, uint32_t KS, const uint32_t *ids, size_t m, uint64_t *W,
                        uint32_t *newflag, hipStream_t s, uint32_t *len = nullptr);
void launch_compact_rows(const uint64_t *W, const uint32_t *flags, const uint32_t *pos, size_t m, uint32_t KS,
                         uint64_t *out, hipStream_t s);
// out row e = the first KD words of row r of W [.][KS], r = ids[e] (or ids2[ids[e]]);
// fout[e] = fin[r] when fin is given
void launch_gather_rows(const uint64_t *W, const uint32_t *ids, size_t m, uint32_t KS, uint32_t KD, uint64_t *out,
                        const uint32_t *fin, uint32_t *fout, hipStream_t s, const uint32_t *ids2 = nullptr);
void launch_row_word(const uint64_t *W, const uint32_t *ids, size_t m, uint32_t KS, uint32_t k, uint64_t *keys,
                     hipStream_t s);
void launch_iota(uint32_t *v, size_t m, hipStream_t s);

// Compressed sort keys of patterns of a fit from codes.  Inside one 64-bit word
// the tokens of one feature form a piece with at most one set bit in any pattern
// (a record has one bin per feature and an intersection keeps at most that one).
// A piece's code is 0 when empty, else 1 + the index of its set bit; the codes,
// most significant piece first (words ascending, higher bits first within a
// word), are packed into key words kw = 0, 1, ...  Comparing key words as
// unsigned (kw0, kw1, ...) orders patterns exactly as comparing (w0, w1, ...).
struct KeyPiece {
    uint8_t word, lo, width, kw, shift, pad[3];   // bits [lo, lo+width) of word -> kw << shift
};
// keys[k * m + e] = key word k of pattern ids[e] (rows X [n][KS]), or of row X[e]
// when ids is null
void launch_compress_keys(const uint64_t *X, uint32_t n, uint32_t KS, const uint32_t *ids, size_t m,
                          const KeyPiece *pieces, uint32_t npieces, uint64_t *keys, hipStream_t s);
// OR and AND of each of nk key arrays of length m (orv/andv preset to 0 / ~0)
void launch_key_range(const uint64_t *keys, uint32_t nk, size_t m, unsigned long long *orv,
                      unsigned long long *andv, hipStream_t s);
// out[e] = src[perm[e]]
void launch_permute_u64(const uint64_t *src, const uint32_t *perm, size_t m, uint64_t *out, hipStream_t s);
void launch_permute_u32(const uint32_t *src, const uint32_t *perm, size_t m, uint32_t *out, hipStream_t s);
// count of ordered rows equal to their predecessor (0 = all distinct)
void launch_adjacent_equal(const uint64_t *W, size_t m, uint32_t KS, uint32_t *d_count, hipStream_t s);
// S = f * popcount^2 (Eq. 2) for given rows and supports
void launch_weights(const uint64_t *W, const uint32_t *f, size_t m, uint32_t KS, int64_t *S, hipStream_t s);
// S = f |b|^2 from token counts len [m]
void launch_weights_len(const uint32_t *f, const uint32_t *len, size_t m, int64_t *S, hipStream_t s);

// factor.hip -- factored tokens for the matrix-core operands.
// A feature with nb bins takes m = ceil(log2 nb) bit tokens and one or two presence
// tokens instead of nb one-hot tokens.  A pattern's (candidate's) factored row, a
// bitset, sets for every feature it holds the bits of the bin index and the
// presence tokens; the side that holds every feature (records; flows in scoring)
// is written with signed values instead (see FactorView::tok), so that the
// contraction counts the bits in which the bin indices differ over the features the
// pattern holds: zero exactly when "b inside r" (Eq. 6 on the one-hot packing of
// Eq. 5).  Records and flows hold one bin per feature and candidates and patterns
// at most one, so every row of a fit from codes has a factored form; a bin of a
// feature is read back from the one-hot row as the index of its one set bit.
struct FacFeature {
    uint16_t off, nb;            // one-hot token range [off, off + nb) of the feature
    uint8_t w0, nw, pad[2];      // its tokens lie in output words w0 .. w0 + nw - 1 (nw <= 2)
    uint32_t mask;               // masks of bin c: mask + c * nw + (word - w0)
};
struct FacPiece {                // the part of a feature inside one one-hot word
    uint8_t lo, width;           // bits [lo, lo + width) of that word
    uint8_t w0, nw;              // output words of the feature (FacFeature)
    uint16_t base, pad;          // bin of bit lo
    uint32_t mask;               // FacFeature::mask of the feature
    uint32_t pad2;               // 16 bytes: one scalar load per piece
};
struct FactorView {
    const FacFeature *feat = nullptr;   // [d]
    const uint64_t *mask = nullptr;     // the pattern-side tokens of every (feature, bin)
    const uint32_t *fbeg = nullptr;     // [KF + 1]: features touching word w are
    const uint32_t *fend = nullptr;     //   [fbeg[w], fend[w]) (features in token order)
    const FacPiece *piece = nullptr;    // pieces grouped by one-hot word
    const uint32_t *pbeg = nullptr;     // [nwords + 1]: pieces of one-hot word k are [pbeg[k], pbeg[k + 1])
    // Digit ranges for rows of record pairs: entries of output word o are
    // [wbeg[o], wbeg[o + 1]) of wfe, each {x: bit in the spanning mask, y: 1 when the
    // feature's tokens span two words, z | w << 32: its tokens in word o}
    const uint4 *wfe = nullptr;
    const uint32_t *wbeg = nullptr;     // [KF + 1]
    // Signed operands of the side that holds every feature (records; flows in
    // scoring): tok[t], t < KF * 64, = kind | bit << 8 | feature << 16, kind 0 no
    // token, 1 bit `bit` of the bin index (+1.0 when 0, -1.0 when 1), 2 and 3 the
    // two parts of the popcount of the bin index (presence_parts); fbit[2 f + i] =
    // the bit tokens of feature f in word feat[f].w0 + i
    const uint32_t *tok = nullptr;
    const uint64_t *fbit = nullptr;
    const uint64_t *bitw = nullptr;     // [KF]: the bit tokens of every feature, per word
    const uint32_t *ptok = nullptr;     // [d]: first presence token | count << 24 (~0: none)
    uint32_t d = 0, KF = 0;             // KF = 0: no factoring (operands are the one-hot words)
    // ternary = 1: bit tokens only, no presence tokens.  A row is two bitsets of KF
    // words, P (every bit token of each feature the row holds) then V (the bits of
    // its bin indices, V inside P); both sides of a contraction read P AND NOT V as
    // +1, P AND V as -1, the rest as 0, so a (candidate, record) product sums to
    // |P_b| - 2 (bits in which their bin indices differ): |P_b| exactly when b lies
    // inside r.  mask holds only the bin bits; fbit the feature's tokens (P), and
    // a piece's pad2 its feature.
    uint32_t ternary = 0;
    uint32_t nmask = 0;                 // entries of mask
    uint32_t npiece = 0;                // entries of piece
    uint32_t nwords = 0;                // one-hot storage words pbeg covers (the fit's KS)
};
// Operand rows out[m][KO], KO = fv.KF when factoring, else KS (out[m][2 KO], P then
// V, for a ternary view): row e is the pattern X[i] AND X[j] of pair id ids[e] (ids
// non-null, rows X [n][KS]) or the row W[e] [m][KS]; complement writes NOT of every
// word (not for a ternary view).
void launch_operand_rows(const uint64_t *X, uint32_t n, const uint32_t *ids, const uint64_t *W, uint32_t KS, size_t m,
                         const FactorView &fv, bool complement, uint64_t *out, hipStream_t s);
// Factored operand rows of record pairs from the records' own factored rows FR
// [n][fv.KF]: row e (pair id ids[e]) is FR[i] AND FR[j] with the tokens of every
// feature on which the two records differ cleared (a one-bin-per-feature fit).
void launch_pair_rows_factored(const uint64_t *FR, uint32_t n, const uint32_t *ids, size_t m, const FactorView &fv,
                               uint64_t *out, hipStream_t s);

// subset.hip -- the subset-test kernels (Eq. 6 inside Eq. 3, Eq. 2 and Eq. 4)
struct CohSeg {                 // one (problem, class) for one coherence phase
    const uint64_t *X;          // class rows [n][KS]
    const uint64_t *NXo;        // complemented other-class rows [n_o][KS]
    const uint32_t *cand;       // input: candidate pair ids still uncovered
    const uint32_t *cand_off;   // if non-null, the ids start at cand + *cand_off
    const uint32_t *ncand;      // device count of cand
    uint32_t *out;              // output: ids uncovered by this phase (appended)
    uint32_t *nout;             // device counter of out
    unsigned long long *tests;  // sum of t(b)
    uint32_t n, n_o;
};
// One phase of the coherence filter (Eq. 3) over all segments (same KS): other-
// class records [r_begin, r_end) in input order.  Tasks of 64*cpl candidates are
// pulled from `queue` (zeroed by the launcher).
void launch_coherence(int KS, int cpl, const CohSeg *segs_dev, uint32_t nseg, uint32_t r_begin, uint32_t r_end,
                      uint32_t *queue, uint32_t grid, hipStream_t s);
// persistent grid of the coherence kernel: grid_per_cu workgroups per compute unit
// Compute units of the current device (256 when it cannot be read)
uint32_t device_cus();
uint32_t coherence_grid(uint32_t grid_per_cu);
// digest of the set of (row [first K words], f, S) over rows [m][KS], order-free
void launch_digest(const uint64_t *W, const uint32_t *f, const int64_t *S, size_t m, uint32_t KS, uint32_t K,
                   unsigned long long *out, hipStream_t s);

// Subset tests on the matrix cores (fp4 0/1 contraction, dense, KO <= 8 operand
// words): columns are m operand rows B [m][KO], the A side is n_rec records in
// the tile layout of launch_mfma_records (mfma_record_tiles(n_rec) * KO * 64 uint4
// built from complemented operand rows).  count = false: out[e] = 1 when no
// record contains row e (coherence, Eq. 3); count = true: out[e] = the number of
// records containing it (support f, Eq. 2).
uint32_t mfma_record_tiles(uint32_t n);
void launch_mfma_records(const uint64_t *NX, uint32_t n, uint32_t KS, uint4 *frag, hipStream_t s);
// The same tiles for factored tokens: records on the signed side (FactorView::tok)
// from their factored rows FR [n][fv.KF]; KO = fv.KF.
void launch_mfma_records_signed(const uint64_t *FR, uint32_t n, const FactorView &fv, uint4 *frag, hipStream_t s);
// Bias slots of a ternary view with T bit tokens: the top tern_bias_slots(T) tokens
// of its last word hold no bit token.  In the record tiles the top slot is +1.0 and
// the others +6.0; each candidate row carries there the nibbles (weights 0, +-0.5
// .. +-6) that add 1 - |P| to its product with every record, so that a product is
// 1 when the record contains the candidate and at most -1 otherwise.  1 - |P| is
// reached with one +1.0 slot (the remainder modulo 3), floor((|P| - 1) / 36) slots
// of 36 and two of at most 24: 3 + floor((T - 1) / 36) slots.
__host__ __device__ constexpr uint32_t tern_bias_slots(uint32_t T) { return 3u + (T ? (T - 1u) / 36u : 0u); }
// The same tiles for a ternary view, from the records' ternary rows FR [n][2 KO]
// with T bit tokens: the same nibbles as the candidate side (P AND NOT V +1.0, P
// AND V -1.0, else 0) and the bias slots; rows past n are 0 on every token.
void launch_mfma_records_ternary(const uint64_t *FR, uint32_t n, uint32_t KO, uint32_t T, uint4 *frag,
                                 hipStream_t s);
// The same tiles of records listed per bucket (bucket u < nb: the brec[u] records
// list[ro[u] ..] in tiles [bt[u], bt[u + 1]), the last one padded with empty rows).
void launch_mfma_records_ternary_lists(const uint64_t *FR, uint32_t KO, uint32_t T, const uint32_t *list,
                                       const uint32_t *ro, const uint32_t *bt, const uint32_t *brec, uint32_t nb,
                                       uint32_t ntiles, uint4 *frag, hipStream_t s);
// sets: 32-column sets per wave (1..3, capped by what fits the registers at KO
// words; 0 = the default for KO).  ternary: B rows are [m][2 KO] ternary rows and
// the tiles come from launch_mfma_records_ternary.
void launch_contain_mfma(int KO, bool count, const uint64_t *B, size_t m, const uint4 *frag, uint32_t n_rec,
                         uint32_t *out, hipStream_t s, int sets = 0, bool ternary = false);

// The contraction pruned by token buckets (ternary rows only, see
// k_contain_mfma_pruned): candidates of bucket u are positions [cs[u], cs[u + 1])
// of perm (position -> row of B and of out; null: the identity); workgroups [uoff[u], uoff[u + 1])
// take them contain_pruned_cols(KO, sets) at a time against the record tiles
// [bt[u], bt[u + 1]) of bucket u (brec[u] real records), u < nb.  units =
// uoff[nb].  out as launch_contain_mfma's.
struct ContainBuckets {
    const uint32_t *perm;       // position -> candidate (null: the identity)
    const uint4 *desc;          // [2 units]: each work unit's ranges (launch_contain_plan)
    bool by_position;           // out[position] instead of out[candidate] (coalesced stores)
};
uint32_t contain_pruned_cols(int KO, int sets);
// units: the grid, at least uoff[nb] (workgroups past it end at once)
void launch_contain_mfma_pruned(int KO, bool count, const uint64_t *B, const uint4 *frag, const ContainBuckets &k,
                                uint32_t units, uint32_t *out, hipStream_t s, int sets = 0);
// uoff [nb + 1] of the pruned contraction's work units from the bucket starts first
// [nb + 1] and cols candidates per unit; *tests += the pairs it examines (nrec [nb]:
// records per bucket); with desc, the ranges of each of `bound` units (candidates,
// record tiles bt [nb + 1], records), 2 uint4 per unit, empty past the last unit.
void launch_contain_plan(const uint32_t *first, const uint32_t *nrec, uint32_t nb, uint32_t cols, uint32_t *uoff,
                         unsigned long long *tests, hipStream_t s, const uint32_t *bt = nullptr, uint32_t bound = 0,
                         uint4 *desc = nullptr);

// Support f and weight S of m ordered patterns W [m][KS] against the complemented
// rows NX [n][KS] of their class.
void launch_support(int KS, int cpl, const uint64_t *W, size_t m, const uint64_t *NX, uint32_t n, uint32_t *f,
                    int64_t *S, hipStream_t s);

struct ScoreModel {
    const uint64_t *P[2];       // patterns of class 0 / 1 [np][KS]
    const int64_t *S[2];
    uint64_t np[2];
    uint32_t KS;
    int64_t maxS[2];            // largest weight of each class
    const uint4 *frag[2];       // matrix-core operands of the patterns and weights (or null)
    uint32_t ftiles[2];         // 32-row tiles of frag
    uint32_t KO;                // operand words of frag (factored or one-hot)
    FactorView fv;              // the factoring of frag (fv.KF = 0: one-hot)
    bool spare;                 // frag holds +1.0 at the unused last token (see k_mfma_patterns)
    uint32_t tslots;            // fv.ternary: bias slots of the view (tern_bias_slots)
    const uint32_t *btile[2];   // [nbucket + 1]: first tile of each token bucket (null: not bucketed)
    uint32_t nbucket;           // buckets = tokens L
};

// prune.hip -- token buckets (see prune.hip).
// cnt[u] += records of X [n][KS] holding token u < L (cnt preset by the caller)
void launch_token_counts(const uint64_t *X, uint32_t n, uint32_t KS, uint32_t L, uint32_t *cnt, hipStream_t s);
// key[e] = the token of row e with the smallest cost[token] (lowest token on ties)
void launch_bucket_keys(const uint64_t *W, size_t m, uint32_t KS, uint32_t L, const uint32_t *cost, uint64_t *key,
                        uint32_t *err, hipStream_t s);
// first[key[e]] = e where ascending keys change (first preset by the caller)
void launch_bucket_first(const uint64_t *key, size_t m, uint32_t *first, hipStream_t s);
// Per-call work of pruned scoring, carved from prune_scratch_words(L, n, d, KO) u32
// (16-byte aligned): flow lists, work units, and the flows' B operands.
struct PruneWork {
    uint32_t *cnt, *cursor, *foff, *uoff, *queue, *list;
    uint4 *ops;
};
size_t prune_scratch_words(uint32_t L, uint32_t n_flows, uint32_t d, uint32_t KO);
// Token buckets of the fit's contractions (see prune.hip).  Elements are grouped
// by a key <= L: out (perm or list) holds them key after key, first [L + 2] the
// first position of each key (first[L + 1] = m); ws: bucket_ws_words(m, L) u32.
size_t bucket_ws_words(size_t m, uint32_t L);
// Xr [n][KSr]: the tokens of each record of X [n][KS] renumbered by rank [L] (a
// permutation of 0 .. L - 1; KSr * 64 >= L).
void launch_rank_rows(const uint64_t *X, uint32_t n, uint32_t KS, uint32_t L, const uint16_t *rank, uint32_t KSr,
                      uint64_t *Xr, hipStream_t s);
// Candidates grouped by bucket, the token inv[q] of the lowest renumbered token q
// they hold: candidate e is the pair id ids[e] of the renumbered records Xr
// [n][KSr] (their intersection), or row e of W [m][KS] (one-hot words, renumbered
// through rank); L for a candidate without a token.  perm [m]: candidate indices
// (may be null when ids_out is given); ids_out [m] (optional, with ids): the ids in
// the same order.
void launch_group_candidates(const uint64_t *Xr, uint32_t n, uint32_t KSr, const uint32_t *ids, const uint64_t *W,
                             uint32_t KS, size_t m, uint32_t L, const uint16_t *rank, const uint16_t *inv,
                             uint32_t *key, uint32_t *perm, uint32_t *first, uint32_t *ws, hipStream_t s,
                             uint32_t *ids_out = nullptr);
// The records of X [n][KS] (d tokens each) under each token they hold: list
// [n d] of record indices, key [n d] scratch; ws: bucket_ws_words(n d, L) u32.
void launch_group_records(const uint64_t *X, uint32_t n, uint32_t KS, uint32_t L, uint32_t d, uint32_t *key,
                          uint32_t *list, uint32_t *first, uint32_t *ws, hipStream_t s);
PruneWork prune_work(uint32_t *ws, uint32_t L, uint32_t n_flows, uint32_t d);
// Lists of the valid flows holding each token, work units of SC_COLS-flow blocks
// and rt-tile ranges per (class, bucket), and out initialised ((0,0) valid,
// (-1,-1) invalid flows).
void launch_prune_lists(const uint16_t *codes, uint32_t n, uint32_t d, const uint32_t *off, const uint16_t *nbins,
                        uint32_t L, const uint32_t *bt0, const uint32_t *bt1, uint32_t rt, uint32_t cols,
                        int64_t *out, PruneWork &w, hipStream_t s);
// uint4 per 32-pattern tile of the scoring operands at KO operand words
constexpr uint32_t score_tile_words(uint32_t KO) { return KO * 64 + 8; }
// Scoring on the matrix cores (KO <= 8, every weight < 2^28): each 32-pattern tile
// of frag holds the patterns' operand rows (KO * 64 uint4, tokens as -1.0) and the
// non-zero lanes of the int8 operand of their 7-bit weight chunks (8 uint4):
// ceil(m/32) * score_tile_words(KO) uint4 from launch_mfma_patterns.  Flows given as codes are factored like the
// patterns; flows given as words need one-hot operands (fv.KF = 0).
// spare: the last token of the last word is used by no row; it then carries the
// +1 that starts each containment count (flows hold 1 there), so the accumulators
// can start at 0.  tern: W holds ternary rows [m][2 KS] (P then V) of a ternary
// view with bias slots (tern_bias_slots); the tiles take the candidate side of the
// ternary contraction and the flows the record side (ScoreModel::tslots).
// With buckets (bt, brow: [L + 1] each, ntiles = bt[L]), the tiles [bt[u], bt[u + 1])
// hold positions [brow[u], brow[u + 1]) of the order perm, row perm[e] at position
// e (perm may be null: the identity); without, ntiles is ceil(m / 32) and tile t
// holds rows 32 t ...
void launch_mfma_patterns(const uint64_t *W, const int64_t *S, uint32_t m, uint32_t KS, bool spare, bool tern,
                          uint4 *frag, hipStream_t s, const uint32_t *perm = nullptr, const uint32_t *bt = nullptr,
                          const uint32_t *brow = nullptr, uint32_t L = 0, uint32_t ntiles = 0);
void launch_score_mfma(const ScoreModel &m, const uint16_t *codes, const uint64_t *words, uint32_t K,
                       uint32_t n_flows, uint32_t d, const uint32_t *meta, const uint16_t *nbins, int64_t *out,
                       hipStream_t s);
// Eq. 4 on the matrix cores for flows given as codes, each flow tested only against
// the token buckets of its own tokens (m.btile non-null).  ws: prune_scratch_words(
// m.nbucket, n_flows, d, m.KO) u32 of device scratch (16-byte aligned), used until the stream reaches the
// end of the call.  false (nothing launched) when the work units of the call could
// overflow 32-bit counts; the caller then scores densely.
bool launch_score_mfma_pruned(const ScoreModel &m, const uint16_t *codes, uint32_t n_flows, uint32_t d,
                              const uint32_t *meta, const uint16_t *nbins, int64_t *out, uint32_t *ws, hipStream_t s);
// Eq. 4 for n_flows flows: codes [n][d] (meta = off|flo|fhi, nbins) or packed
// words [n][K].  out [n][2] = (A, N) is initialised by the launcher.
void launch_score(const ScoreModel &m, const uint16_t *codes, const uint64_t *words, uint32_t K, uint32_t n_flows,
                  uint32_t d, const uint32_t *meta, const uint16_t *nbins, int64_t *out, int fpl, hipStream_t s);

void launch_reduce_maxsum(const int64_t *S, size_t m, unsigned long long *d_max_sum /*[2]*/, hipStream_t s);

// evidence.hip -- the heaviest patterns inside each flow (see ig_evidence)
struct EvidenceModel {
    const uint64_t *W[2];
    const uint32_t *f[2];
    const int64_t *S[2];
    uint64_t np[2];
    const uint32_t *bperm[2];   // rows grouped by token bucket, or null (scan every row)
    const uint32_t *brow[2];    // [L + 1] bucket starts in bperm
    uint32_t KS, K, d;
    const uint32_t *off;        // token offset of each feature
    const uint16_t *nbins;
};
uint32_t evidence_max_k();
void launch_evidence(const EvidenceModel &m, const uint16_t *codes, uint32_t n, uint32_t k, uint32_t *count,
                     uint64_t *words, uint32_t *f, int64_t *S, hipStream_t s);

// noalloc.hip -- the fixed scratch array of ig_score_noalloc: its size in u32, and
// the current device's copy (looked up once per device)
size_t noalloc_scratch_words();
uint32_t *noalloc_scratch();

// regulate.hip -- Regulations 1-3 and the detection metrics (Section 3.1, Table 2)
void normal_moments(const int64_t *scores, const uint8_t *labels, uint32_t n, ig_moments *h, hipStream_t s);
int64_t r3_threshold(const ig_moments &mo, double r);
void classify(const int64_t *scores, uint32_t n, int64_t r3_cut, uint32_t flags, uint8_t *label, uint8_t *rule,
              hipStream_t s);
void detection_metrics(const int64_t *scores, const uint8_t *pred, const uint8_t *truth, uint32_t n, ig_metrics *h,
                       hipStream_t s);

// probe.hip -- attainable peaks (include/ig_probe.h); both wait for the stream
double probe_mfma_fp4(uint32_t iters, hipStream_t s, float *ms);                          // operations/s
double probe_copy(const void *src, void *dst, size_t bytes, hipStream_t s, float *ms);   // bytes/s

}  // namespace ig
