/*
 * ig.h -- C ABI of libig, the MI355X (gfx950) implementation of the hot path of
 * Interpretable Generalization (IG) intrusion detection:
 *
 *   Section 3.1, Eq. 1   candidates: every record and every pairwise intersection
 *                        of records of one class
 *   Section 3.1, Eq. 3   coherence: keep a candidate only when no record of the
 *                        other class contains it (subset test of Eq. 6)
 *   Section 3.1, Eq. 2   weight S_c(b) = f_c(b) * |b|^2
 *   Section 3.1, Eq. 4   scores A(x), N(x) of a flow x
 *   Section 3.2, Eq. 5   records are bitsets packed into K = ceil(L/64) words
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Classes.  Label 0 is "normal" (class "-"), label 1 is "attack" (class "+").
 *   Class-1 patterns are summed into A, class-0 patterns into N (Eq. 4).
 * Tokens.  Record i, feature f, bin c (c < nbins[f]) is token off[f] + c with
 *   off[f] = nbins[0] + ... + nbins[f-1]; L = sum of nbins; token j is bit j%64
 *   of word j/64 (least significant bit first).  Unused high bits are zero.
 * Readings.  f_c(b) counts the class-c training records (repeats included)
 *   that contain b; |b| is the number of tokens of b; the empty intersection is
 *   never a pattern.  A pattern set is a set: a model holds its rows in an
 *   unspecified order (whatever the fit produced them in); ig_model_export
 *   reports them in ascending order of (w_0, ..., w_{K-1}) compared as unsigned
 *   64-bit words, w_0 most significant.
 * Memory.  Pointers named d_* are device (HBM) pointers on the current HIP
 *   device; h_* are host pointers.  Inputs are borrowed for the duration of the
 *   call (until the stream reaches the call's last kernel for the asynchronous
 *   entry points) and never modified.  Outputs are written only on IG_OK.
 * Streams.  `stream` is a hipStream_t (NULL = the legacy default stream).  All
 *   device work of a call is ordered on it.
 * Errors.  Every call returns an ig_status; nothing throws across the ABI.
 *   ig_last_error() returns a thread-local message for the last failing call.
 *   Argument checks that need no device data run before any device work.
 * Threads.  A model is immutable after it is built: scoring the same model on
 *   several streams or host threads at once is safe.  Fitting calls may run
 *   concurrently on different streams (each uses stream-ordered scratch).
 * Limits.  L <= 4096 (K <= 64); d <= 4096; at most 92,000 training records per
 *   class (pair ids are 32-bit); n_flows < 2^31.
 */
#ifndef IG_H
#define IG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    IG_OK = 0,
    IG_E_INVAL = -1,        /* bad argument or out-of-range input value            */
    IG_E_NOMEM = -2,        /* device or host allocation failed                     */
    IG_E_DEVICE = -3,       /* a HIP runtime call failed                            */
    IG_E_OVERFLOW = -4,     /* a score could exceed int64                           */
    IG_E_UNSUPPORTED = -5   /* size beyond the limits above                         */
} ig_status;

#define IG_ABSENT 0xFFFFu   /* pattern code rows only: feature not in the pattern  */

typedef struct ig_model ig_model;   /* opaque; owns the device-resident pattern sets */

/* One row of a tuning table (written by the project's autotuner).  A row with
 * mfma_words = 0 gives the VALU kernels' launch shape for problems stored with
 * `ks` words (0 = any width); a row with mfma_words = W gives the matrix-core
 * contractions' shape for problems whose operands take W words.  Of the rows that
 * match, the one with the largest min_pairs not above the problem's pairs wins
 * (an exact ks beats ks = 0).  Tuning never changes results. */
typedef struct {
    uint32_t ks;             /* storage words (0 = any; VALU rows)                   */
    uint32_t min_pairs;      /* smallest problem (pairs of both classes) it covers   */
    uint32_t filter_cpl;     /* coherence kernel: candidates per lane, 1 or 2        */
    uint32_t grid_per_cu;    /* coherence kernel: workgroups per compute unit, 1..32 */
    uint32_t support_cpl;    /* support kernel: patterns per lane, 1 or 2            */
    uint32_t mfma_words;     /* 0: a VALU row; else the operand words it is for      */
    uint32_t coherence_sets; /* matrix-core coherence: 32-column sets per wave, 1..3
                                (capped by the registers at that width; 0 default)  */
    uint32_t support_sets;   /* matrix-core support: the same                        */
} ig_tune_entry;

/* A caller's device allocator (e.g. a framework's caching allocator).  alloc
 * returns `bytes` of device memory on the current device, usable by work queued on
 * `stream` (NULL for a model buffer, which every stream may use), or NULL when it
 * cannot; free takes back a block alloc returned, with the stream the library last
 * used it on (NULL for model buffers: by then no queued work uses them).  Both may
 * be called from any host thread that calls the library.  A model built with an
 * allocator returns its buffers to it in ig_model_free: the allocator (and ctx)
 * must stay valid until every such model is freed. */
typedef struct {
    void *(*alloc)(size_t bytes, void *stream, void *ctx);
    void (*free)(void *ptr, void *stream, void *ctx);
    void *ctx;
} ig_allocator;

/* Optional knobs of a fit.  Zero-initialise and set what is needed. */
typedef struct {
    uint64_t mem_budget_bytes;  /* 0: no limit.  Otherwise the pair space of a class
                                   is processed in chunks so that the fit's scratch
                                   stays near this many bytes (results unchanged).   */
    uint32_t filter_cpl;        /* candidates per lane of the coherence kernel
                                   (0 = tuned default; 1 or 2); overrides the table   */
    uint32_t score_fpl;         /* reserved                                           */
    uint32_t block;             /* reserved (workgroups are 256 threads)              */
    uint32_t n_tune;            /* rows in `tune`                                     */
    const ig_tune_entry *tune;  /* host tuning table (may be NULL)                    */
    uint32_t coherence_mfma;    /* coherence (Eq. 3) and support (Eq. 2) kernels:
                                   0 = automatic: matrix cores when the operands fit
                                       16 words, else the VALU path;
                                   1 = matrix cores: a dense contraction with fp4
                                       operands and fp32 accumulation, exact; no early
                                       exit, so ig_stats.tests counts every (candidate,
                                       other-class record) pair.  Fits from codes use
                                       factored tokens: those of mode 5 when they
                                       take fewer words than those of mode 4, else
                                       those of mode 4; other fits the K one-hot
                                       words; at most 16 words;
                                   2 = VALU path: AND-NOT chains with early exit in
                                       input order (ig_stats.tests = sum of t(b));
                                   3 = matrix cores on the one-hot words (K <= 16);
                                   4 = matrix cores on factored tokens with presence
                                       tokens (bits of the bin index plus one or two
                                       presence tokens per feature: 207 tokens, 4
                                       words, for 41 features of ~11 bins);
                                   5 = matrix cores on ternary bit tokens whenever
                                       the fit has them (else as 1): the bits of each
                                       feature's bin index alone, +1 / -1 on both
                                       sides for a bit of a feature the row holds, 0
                                       for one it lacks, plus a few bias tokens: 165
                                       + 7 tokens, 3 words, for 41 features of ~11
                                       bins.
                                   All give the same patterns, f and S.             */
    uint32_t fit_dense;         /* matrix-core coherence and support on the ternary
                                   bit tokens (mode 5, or 0 / 1 when they apply):
                                   0 = token buckets: the records of the tested class
                                       are listed under each token they hold, and a
                                       candidate meets only the records holding its
                                       token held by the fewest (a record without it
                                       cannot contain the candidate, Eq. 6), so
                                       ig_stats.tests and support_tests count the
                                       (candidate, record) pairs of its bucket;
                                   1 = every record (dense).
                                   Both give the same patterns, f and S.             */
    const ig_allocator *alloc;  /* NULL: the library's device arena (chunks taken from
                                   the runtime once and sub-allocated, see
                                   ig_release_memory); else every model buffer and
                                   every scratch block of the call comes from it.
                                   When it fails, the call returns IG_E_NOMEM, frees
                                   what it took and builds no model.                 */
} ig_fit_opts;

/* Counters and timings of a fit (Section 3.3 stages). */
typedef struct {
    uint64_t n_class[2];     /* training records per class                           */
    uint64_t pairs[2];       /* n_c (n_c - 1) / 2                                    */
    uint64_t distinct[2];    /* distinct non-empty members of B^c (Eq. 1)            */
    uint64_t coherent[2];    /* |P^c| (Eq. 3)                                        */
    uint64_t tests[2];       /* subset tests made by the coherence kernel: on the VALU
                                path the sum over distinct candidates of t(b), the
                                other-class records examined in input order up to and
                                including the first that contains b (all of them when
                                none does); on the matrix cores every pair, or with
                                token buckets (fit_dense = 0) the pairs of each
                                candidate and the records of its bucket             */
    uint64_t support_tests[2]; /* subset tests of Eq. 2 made by the support kernel:
                                |P^c| * n_c, or with token buckets the pairs of
                                each pattern and the records of its bucket          */
    uint32_t chunks[2];      /* pair-space chunks used for the class                 */
    float ms[8];             /* device time per stage: 0 pack, 1 pairs+hash, 2 sort,
                                3 dedup, 4 coherence, 5 order, 6 support, 7 total
                                (batched fits: a group's shared stages are split
                                over its problems by their share of the pairs)       */
    float kernel_ms[2];      /* device time of the subset-test kernels alone:
                                0 coherence, 1 support (0 when not measured)         */
} ig_stats;

typedef struct {
    uint32_t K;              /* words per bitset                                     */
    uint32_t L;              /* token universe size                                  */
    uint32_t d;              /* features (0 for a model fitted from packed words)    */
    uint32_t flags;          /* IG_MODEL_* bits                                      */
    uint32_t mfma_tokens;    /* tokens per row of the matrix-core operands: the
                                factored count, or L when they are one-hot           */
    uint32_t mfma_words;     /* 64-token words per row of those operands             */
    uint64_t n_patterns[2];  /* |P^0|, |P^1|                                         */
    int64_t max_weight[2];   /* largest S of each class                              */
    uint32_t fit_tokens;     /* tokens per operand row of the fit's matrix-core
                                contractions (coherence, support): the ternary bit
                                tokens, the factored count or L; 0 when the fit ran
                                on the vector ALUs or the model was imported         */
    uint32_t fit_words;      /* 64-token words per operand row of those              */
} ig_model_info;

/* ig_model_info.flags.  IG_MODEL_SCORE_MFMA: ig_score evaluates Eq. 4 on the
 * matrix cores (operands of at most 8 words, every weight below 2^28), otherwise
 * on the vector ALUs; both give identical scores.  IG_MODEL_FACTORED: those
 * operands use factored tokens; ig_score_packed (whose words may hold several
 * bins of a feature) then runs on the vector ALUs. */
#define IG_MODEL_SCORE_MFMA 1u
#define IG_MODEL_FACTORED 2u
/* IG_MODEL_BUCKETED: the matrix-core scoring tiles are grouped by token bucket
 * (fits from codes and imported models), so ig_score can prune (ig_score_ex). */
#define IG_MODEL_BUCKETED 4u
/* IG_MODEL_FIT_BUCKETS: the fit's coherence and support contractions tested each
 * candidate only against the records holding its token held by the fewest of them
 * (ig_fit_opts.fit_dense = 0). */
#define IG_MODEL_FIT_BUCKETS 8u

/* One problem of a batched fit. */
typedef struct {
    const uint16_t *d_codes;  /* [n][d] row-major bin codes                           */
    const uint8_t *d_labels;  /* [n] 0/1                                              */
    uint32_t n, d;
    const uint16_t *h_nbins;  /* [d]                                                  */
} ig_problem;

/* ---------------------------------------------------------------------------
 * ig_fit -- Eq. 1, Eq. 3 and Eq. 2 for both classes (Section 3.1; data layout of
 * Section 3.2; the three stages of Section 3.3).
 *   d_codes  device [n][d] uint16, row-major; d_codes[i*d+f] < h_nbins[f]
 *   d_labels device [n] uint8 in {0,1}
 *   h_nbins  host [d], each >= 1; L = sum <= 4096
 * Builds *out, a device-resident model holding P^0 and P^1 with f and S.  Synchronises `stream` before returning (pattern counts are
 * data-dependent).  IG_E_INVAL if any code or label is out of range (checked on
 * the device before anything is fitted).  On error *out is left untouched.
 * ------------------------------------------------------------------------- */
ig_status ig_fit(const uint16_t *d_codes, const uint8_t *d_labels, uint32_t n, uint32_t d,
                 const uint16_t *h_nbins, const ig_fit_opts *opts, void *stream, ig_model **out);

/* ig_fit for general token sets given already packed (Eq. 5): d_words device
 * [n][K] uint64.  The model has d = 0 and can only score packed flows. */
ig_status ig_fit_packed(const uint64_t *d_words, const uint8_t *d_labels, uint32_t n, uint32_t K,
                        const ig_fit_opts *opts, void *stream, ig_model **out);

/* ---------------------------------------------------------------------------
 * ig_fit_batch -- n_probs independent fits (problems of any size and width).
 * Problems are grouped by word width and by memory; for each group, pair
 * enumeration, one radix sort, one de-duplication and one coherence launch
 * over every (problem, class) of the group run as a single captured HIP graph,
 * followed by ordering and support per problem.  A problem too large for a group
 * is fitted on its own as by ig_fit.  outs[p] receives exactly the model ig_fit
 * would build for probs[p] (same patterns, f, S, counters).  All problems are
 * validated first; on any error no model is returned and outs is untouched.
 * Synchronises `stream` before returning.
 * ------------------------------------------------------------------------- */
ig_status ig_fit_batch(const ig_problem *probs, uint32_t n_probs, const ig_fit_opts *opts,
                       void *stream, ig_model **outs);

/* ---------------------------------------------------------------------------
 * ig_score -- Eq. 4 for n_flows flows given as bin codes (same d and nbins as
 * the model), fused packing + coverage + weighting + reduction (Section 3.3,
 * inference).  Asynchronous on `stream`.
 *   d_codes device [n_flows][d] uint16
 *   d_out   device [n_flows][2] int64, written as (A, N) per flow.
 *           A flow with a code >= its feature's bin count gets (-1, -1).
 * Pruned by token buckets when the model has them (see ig_score_ex), with
 * stream-ordered scratch from the library; safe to call concurrently on several
 * streams.
 * ------------------------------------------------------------------------- */
ig_status ig_score(const ig_model *m, const uint16_t *d_codes, uint32_t n_flows, int64_t *d_out,
                   void *stream);

/* ---------------------------------------------------------------------------
 * ig_score_ex -- ig_score with a choice of kernels; all give identical scores.
 *   IG_SCORE_DENSE   every flow is tested against every pattern.
 *   IG_SCORE_PRUNED  exact pruning of Eq. 4: a pattern lies inside a flow only if
 *                    the flow holds every token of the pattern (Eq. 6).  The model
 *                    files each pattern under one of its tokens (its bucket: the
 *                    token the fewest training records of its class hold, or for
 *                    an imported model the token of the feature with the most
 *                    bins), and each
 *                    flow is tested only against the buckets of the d tokens it
 *                    holds.  Needs IG_MODEL_BUCKETED (IG_E_UNSUPPORTED otherwise)
 *                    and device scratch of about 4 * (n_flows * d + 5 L) bytes,
 *                    which the library takes from its stream-ordered cache.
 *   IG_SCORE_AUTO    pruned when the model is bucketed, else dense (= ig_score).
 * ------------------------------------------------------------------------- */
#define IG_SCORE_AUTO 0u
#define IG_SCORE_DENSE 1u
#define IG_SCORE_PRUNED 2u
ig_status ig_score_ex(const ig_model *m, const uint16_t *d_codes, uint32_t n_flows, int64_t *d_out, uint32_t mode,
                      void *stream);

/* ---------------------------------------------------------------------------
 * ig_score_noalloc -- ig_score for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  Same results as ig_score; calls no allocating routine.  Pruned
 * scoring's per-call work goes to a fixed array of IG_NOALLOC_SCRATCH_BYTES in
 * the library's device memory (each GPU the library runs on holds its own copy
 * until the process ends) instead of library-allocated scratch, so a call needs
 *   4 * (ceil4(n_flows * d + 5 L + 3) + 8 W n_flows) <= IG_NOALLOC_SCRATCH_BYTES
 * with W the model's scoring operand words (ig_model_info.mfma_words) and
 * ceil4 rounding up to a multiple of 4 (IG_E_UNSUPPORTED beyond; e.g. about
 * 32,000 flows of 41 features, 464 tokens and 3 words).  Models without token buckets score with the dense kernels, which
 * need no scratch.  Every call on one GPU shares that GPU's array: calls that
 * overlap on a GPU (on different streams, or from different host threads) race
 * and can return wrong scores; order them (one stream, or events).  Each call
 * clears what it uses before using it.  Asynchronous on `stream`.
 * ------------------------------------------------------------------------- */
#define IG_NOALLOC_SCRATCH_BYTES (8u << 20)
ig_status ig_score_noalloc(const ig_model *m, const uint16_t *d_codes, uint32_t n_flows, int64_t *d_out,
                           void *stream);

/* ig_score for flows already packed: d_words device [n_flows][K] uint64 (always
 * dense: such words may hold several bins of a feature). */
ig_status ig_score_packed(const ig_model *m, const uint64_t *d_words, uint32_t n_flows,
                          int64_t *d_out, void *stream);

/* ---------------------------------------------------------------------------
 * ig_evidence -- the evidence of each flow's scores: the coherent patterns of
 * each class inside the flow, the terms Eq. 4 sums into A (class 1) and N
 * (class 0); Sections 2 and 5 present the matched patterns as the readable
 * account of a detection.  The k reported per (flow, class) are the heaviest:
 * weight S descending, then the words ascending in the canonical order (w_0 most
 * significant, unsigned) -- a unique list.  Asynchronous on `stream`.
 *   d_codes  device [n_flows][d] uint16 (same d and nbins as the model)
 *   k        1..256 (IG_E_INVAL otherwise)
 *   d_count  device [n_flows][2] uint32: how many patterns of class 0 / 1 lie
 *            inside the flow (all of them, not only the k); 0xFFFFFFFF for a flow
 *            with a code out of range (its slots are zero)
 *   d_words  device [n_flows][2][k][K] uint64: the patterns, best first
 *   d_f, d_S device [n_flows][2][k] uint32 / int64: their supports and weights
 *   Slots past min(k, count) are zero.  Models with token buckets
 *   (IG_MODEL_BUCKETED) test each flow only against the buckets of its tokens;
 *   others against every pattern.  One workgroup per (flow, class): meant for
 *   the flows a caller wants explained, not for whole test sets.
 * ------------------------------------------------------------------------- */
ig_status ig_evidence(const ig_model *m, const uint16_t *d_codes, uint32_t n_flows, uint32_t k, uint32_t *d_count,
                      uint64_t *d_words, uint32_t *d_f, int64_t *d_S, void *stream);

/* ===========================================================================
 * The classifier of Section 3.1 and the detection metrics of Table 2, on the
 * scores (A, N) that ig_score wrote (device [n][2] int64; (-1, -1) marks a flow
 * with a code out of range).
 *   Regulation 1  attack when A >= N
 *   Regulation 2  attack when A = N = 0 (covered by Regulation 1; reported as the
 *                 deciding rule)
 *   Regulation 3  attack when N < mu_N - r sigma_N
 * Readings: mu_N and sigma_N are the mean and the population standard deviation
 * of N over the normal (label 0) training records, scored by the model like any
 * flow; r is a given constant (Table 2 names 0.568).  Regulation 3 is decided
 * exactly: the real values mu_N - r sigma_N, with r the exact value of the double,
 * are never rounded.
 * ======================================================================== */

/* Exact moments of N over the normal records: mu_N = sum / count,
 * sigma_N^2 = (count * sumsq - sum^2) / count^2. */
typedef struct {
    uint64_t count;      /* records labelled 0 with valid scores                  */
    uint64_t sum[2];     /* sum of N, 128-bit unsigned, least significant word first */
    uint64_t sumsq[3];   /* sum of N^2, 192-bit unsigned                          */
} ig_moments;

/* Confusion counts of predicted labels against the truth (attack = positive) and
 * the AUC of the margin A - N as an exact fraction: over every (attack, normal)
 * pair of flows, auc_num counts 2 when the attack flow's margin is larger and 1
 * when they are equal; auc_den = 2 * attacks * normals. */
typedef struct {
    uint64_t tp, fp, tn, fn;
    uint64_t auc_num, auc_den;
    uint64_t invalid;    /* flows skipped: predicted label 255 (no valid scores)   */
} ig_metrics;

/* ig_classify flags */
#define IG_CLASSIFY_R3 1u      /* apply Regulation 3 with the given threshold      */
#define IG_CLASSIFY_NO_R2 2u   /* report A = N = 0 as decided by Regulation 1      */

/* Moments of N over the records with d_labels[i] == 0 (device [n] uint8, each 0
 * or 1, IG_E_INVAL otherwise), skipping flows without valid scores.  d_scores
 * device [n][2].  Synchronous. */
ig_status ig_normal_moments(const int64_t *d_scores, const uint8_t *d_labels, uint32_t n, ig_moments *out,
                            void *stream);

/* Regulation 3 as an integer cut: *out = T such that, for every integer N >= 0,
 * N < mu_N - r sigma_N exactly when N < T.  Host only (exact big-integer
 * arithmetic).  IG_E_INVAL when r is negative or not finite, or m->count = 0. */
ig_status ig_r3_threshold(const ig_moments *m, double r, int64_t *out);

/* Labels of n flows: d_label device [n] uint8 (1 attack, 0 normal, 255 for a flow
 * without valid scores); d_rule device [n] uint8 (may be NULL): the regulation
 * that decided (1, 2 or 3; 0 when invalid).  Regulation 3 fires when flags has
 * IG_CLASSIFY_R3 and N < r3_threshold (ig_r3_threshold).  Asynchronous. */
ig_status ig_classify(const int64_t *d_scores, uint32_t n, int64_t r3_threshold, uint32_t flags, uint8_t *d_label,
                      uint8_t *d_rule, void *stream);

/* Detection metrics of predicted labels d_pred (device [n], from ig_classify)
 * against d_truth (device [n] uint8, each 0 or 1, IG_E_INVAL otherwise), with
 * the AUC ranked by A - N of d_scores.  Synchronous; uses library scratch of
 * about 40 bytes per flow. */
ig_status ig_detection_metrics(const int64_t *d_scores, const uint8_t *d_pred, const uint8_t *d_truth, uint32_t n,
                               ig_metrics *out, void *stream);

/* Patterns of class `cls` filed under each token bucket (diagnostics of pruned
 * scoring): h_counts host [L] uint32.  IG_E_UNSUPPORTED when the model has no
 * buckets (IG_MODEL_BUCKETED clear).  Synchronous. */
ig_status ig_model_bucket_sizes(const ig_model *m, uint32_t cls, uint32_t *h_counts);

/* Sizes of a model. */
ig_status ig_model_get_info(const ig_model *m, ig_model_info *info);

/* Copy class `cls` of a model to the host: h_words [n][K] (may be NULL),
 * h_f [n] (may be NULL), h_S [n] (may be NULL), with n = info.n_patterns[cls],
 * rows in ascending order of (w_0, ..., w_{K-1}) (sorted on the device, with
 * scratch of about 24 bytes per pattern).  Synchronous. */
ig_status ig_model_export(const ig_model *m, uint32_t cls, uint64_t *h_words, uint32_t *h_f,
                          int64_t *h_S);

/* Build a model from given pattern sets (e.g. loaded from storage).
 *   h_codes[c]  host [count[c]][d] uint16 pattern code rows; IG_ABSENT marks a
 *               feature the pattern does not contain; at least one feature set
 *   h_f[c]      host [count[c]] supports f
 * Each pattern is packed and weighted with S = f * |b|^2 (Eq. 2) on the device.  Patterns of a class must be distinct
 * (IG_E_INVAL otherwise).  Synchronous. */
ig_status ig_model_import(const uint16_t *const h_codes[2], const uint32_t *const h_f[2],
                          const uint64_t count[2], uint32_t d, const uint16_t *h_nbins,
                          void *stream, ig_model **out);

/* 64-bit digest of the set of (row, f, S) of class `cls`, independent of the order
 * the rows are held in, computed on the device: compares models that are too
 * large to copy out.  Equal pattern sets give equal digests.  Synchronous. */
ig_status ig_model_digest(const ig_model *m, uint32_t cls, uint64_t *out);

/* Counters and stage timings of the fit that built the model (zeros for an
 * imported model). */
ig_status ig_fit_stats(const ig_model *m, ig_stats *out);

/* Release a model (NULL-safe).  The caller must not free a model while a
 * scoring call that uses it is still queued on a stream. */
void ig_model_free(ig_model *m);

/* The library's own device memory on the current device (used when no caller
 * allocator is given): hands cached scratch blocks and wholly free arena chunks
 * back to the runtime.  Models stay valid.  Waits for the scratch's last users. */
ig_status ig_release_memory(void);

/* Bytes of the current device's arena: reserved from the runtime, held by models
 * and live scratch, and cached (freed scratch kept for reuse). */
ig_status ig_memory_stats(uint64_t *reserved, uint64_t *in_use, uint64_t *cached);

/* Thread-local text of the last error ("" when none). */
const char *ig_last_error(void);

/* Library version string. */
const char *ig_version(void);

#ifdef __cplusplus
}
#endif
#endif /* IG_H */
