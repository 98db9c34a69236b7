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

/* One row of a tuning table (written by the project's autotuner): the launch
 * shape to use for problems stored with `ks` words and at least `min_pairs`
 * same-class pairs.  The matching row with the largest min_pairs wins; a row with
 * ks = 0 matches any width.  Tuning never changes results. */
typedef struct {
    uint32_t ks;             /* storage words (0 = any)                               */
    uint32_t min_pairs;      /* smallest problem (pairs of both classes) it covers   */
    uint32_t filter_cpl;     /* coherence kernel: candidates per lane, 1 or 2        */
    uint32_t grid_per_cu;    /* coherence kernel: workgroups per compute unit, 1..32 */
    uint32_t support_cpl;    /* support kernel: patterns per lane, 1 or 2            */
    uint32_t reserved[3];
} ig_tune_entry;

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
                                       factored tokens (per feature the bits of its
                                       bin index plus presence tokens: 207 instead of
                                       464 tokens for 41 features of ~11 bins), else
                                       the K one-hot words; at most 16 words;
                                   2 = VALU path: AND-NOT chains with early exit in
                                       input order (ig_stats.tests = sum of t(b));
                                   3 = matrix cores on the one-hot words (K <= 16).
                                   All give the same patterns, f and S.             */
    uint32_t reserved;
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
                                none does); on the matrix cores every pair           */
    uint64_t support_tests[2]; /* |P^c| * n_c subset tests of Eq. 2                  */
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
} ig_model_info;

/* ig_model_info.flags.  IG_MODEL_SCORE_MFMA: ig_score evaluates Eq. 4 on the
 * matrix cores (operands of at most 8 words, every weight below 2^28), otherwise
 * on the vector ALUs; both give identical scores.  IG_MODEL_FACTORED: those
 * operands use factored tokens; ig_score_packed (whose words may hold several
 * bins of a feature) then runs on the vector ALUs. */
#define IG_MODEL_SCORE_MFMA 1u
#define IG_MODEL_FACTORED 2u

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
 * Needs no scratch memory; safe to call concurrently on several streams.
 * ------------------------------------------------------------------------- */
ig_status ig_score(const ig_model *m, const uint16_t *d_codes, uint32_t n_flows, int64_t *d_out,
                   void *stream);

/* ig_score for flows already packed: d_words device [n_flows][K] uint64. */
ig_status ig_score_packed(const ig_model *m, const uint64_t *d_words, uint32_t n_flows,
                          int64_t *d_out, void *stream);

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

/* Thread-local text of the last error ("" when none). */
const char *ig_last_error(void);

/* Library version string. */
const char *ig_version(void);

#ifdef __cplusplus
}
#endif
#endif /* IG_H */
