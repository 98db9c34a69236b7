/*
 * ig_oracle.c -- plain CPU oracle of the Interpretable Generalization (IG) hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this file's library.  It shares no code,
 * header, table or helper with the HIP library; the two meet only at the seeded
 * inputs that the synthetic generators produce.
 *
 * Every step is the plain definition from the paper, written out in the
 * paper's order, with no blocking, fusion or reordering:
 *
 *   Eq. 5  pack each record's tokens into K = ceil(L/64) 64-bit words
 *   Eq. 1  B^c = { x AND x' : x, x' in X^c, pair taken once } union X^c
 *   Eq. 3  P^c = { b in B^c : b is a subset of no record of the other class }
 *          (the subset test is Eq. 6: b AND r == b on every word)
 *   Eq. 2  S_c(b) = f_c(b) * |b|^2
 *   Eq. 4  A(x) = sum over P^+ of S_+(b) [b subset of x],
 *          N(x) = sum over P^- of S_-(b) [b subset of x]
 *
 * Readings taken where the paper is silent (each is listed with the design
 * notes of the repository):
 *   - f_c(b) is the support: the number of class-c training records (repeats
 *     counted) that contain b.
 *   - |b| is the number of set bits (tokens) of b.
 *   - the empty intersection is never a pattern.
 *   - label 1 = attack = class "+" (scored into A); label 0 = normal = "-" (N).
 *   - patterns are reported in ascending order of (w_0, ..., w_{K-1}) compared
 *     as unsigned 64-bit integers, w_0 first.
 *   - bit j of the token universe lives in word j/64 at bit position j%64.
 *   - t(b), the number of opposite-class records examined before the first one
 *     that contains b (that record included), or all of them when none does,
 *     scanning the opposite class in input order.  Its sum is the count of
 *     subset tests the coherence step has to make.
 *
 * Parallelism: OpenMP loops over independent candidates or flows only; each
 * iteration is the plain definition.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define IGO_ABSENT 0xFFFFu

enum { IGO_OK = 0, IGO_E_INVAL = -1, IGO_E_NOMEM = -2 };

typedef struct {
    uint32_t K, L, d;
    uint64_t n_class[2];   /* training records of each class                  */
    uint64_t pairs[2];     /* n_c (n_c - 1) / 2 pair intersections            */
    uint64_t distinct[2];  /* distinct non-empty members of B^c                */
    uint64_t tests[2];     /* sum of t(b) over the distinct candidates         */
    uint64_t count[2];     /* |P^c|                                            */
    uint64_t *words[2];    /* count[c] * K words, ascending                    */
    uint32_t *f[2];        /* support of each pattern                          */
    int64_t *S[2];         /* weight of each pattern                           */
} igo_model;

/* ---------------------------------------------------------------- Eq. 5 ---- */
/* Token universe size L = sum of bins, words per record K = ceil(L / 64). */
static int universe(const uint16_t *nbins, uint32_t d, uint32_t *L, uint32_t *K)
{
    uint64_t s = 0;
    for (uint32_t f = 0; f < d; ++f) s += nbins[f];
    if (s == 0 || s > 65536) return IGO_E_INVAL;
    *L = (uint32_t)s;
    *K = (uint32_t)((s + 63) / 64);
    return IGO_OK;
}

/* Pack n code rows: feature f with bin c is token off[f] + c, where off[f] is
 * the number of bins of the features before f (Section 3.1 tokenisation: every
 * value is tied to its column).  A code equal to IGO_ABSENT sets no token (used
 * only for pattern sets given as codes).  Returns IGO_E_INVAL for a code that is
 * neither IGO_ABSENT nor below the feature's bin count. */
int igo_pack(const uint16_t *codes, uint64_t n, uint32_t d, const uint16_t *nbins,
             uint32_t K, uint64_t *out)
{
    uint32_t *off = (uint32_t *)malloc(sizeof(uint32_t) * (d ? d : 1));
    if (!off) return IGO_E_NOMEM;
    uint32_t acc = 0;
    for (uint32_t f = 0; f < d; ++f) { off[f] = acc; acc += nbins[f]; }
    memset(out, 0, sizeof(uint64_t) * n * K);
    int rc = IGO_OK;
    for (uint64_t i = 0; i < n; ++i) {
        for (uint32_t f = 0; f < d; ++f) {
            uint32_t c = codes[i * d + f];
            if (c == IGO_ABSENT) continue;
            if (c >= nbins[f]) { rc = IGO_E_INVAL; continue; }
            uint32_t bit = off[f] + c;
            out[i * K + bit / 64] |= (uint64_t)1 << (bit % 64);
        }
    }
    free(off);
    return rc;
}

/* ------------------------------------------------------- set primitives ---- */
/* Eq. 6: b is a subset of r when (b AND r) == b on every word. */
static int subset(const uint64_t *b, const uint64_t *r, uint32_t K)
{
    for (uint32_t k = 0; k < K; ++k)
        if ((b[k] & r[k]) != b[k]) return 0;
    return 1;
}

static int is_empty(const uint64_t *b, uint32_t K)
{
    for (uint32_t k = 0; k < K; ++k)
        if (b[k]) return 0;
    return 1;
}

static uint32_t popcount_row(const uint64_t *b, uint32_t K)
{
    uint32_t p = 0;
    for (uint32_t k = 0; k < K; ++k) p += (uint32_t)__builtin_popcountll(b[k]);
    return p;
}

/* Canonical order: (w_0, ..., w_{K-1}) as unsigned integers, w_0 first. */
static uint32_t g_sort_K;
static int cmp_rows(const void *a, const void *b)
{
    const uint64_t *x = (const uint64_t *)a, *y = (const uint64_t *)b;
    for (uint32_t k = 0; k < g_sort_K; ++k) {
        if (x[k] < y[k]) return -1;
        if (x[k] > y[k]) return 1;
    }
    return 0;
}

static uint64_t sort_unique(uint64_t *rows, uint64_t m, uint32_t K)
{
    if (m == 0) return 0;
    g_sort_K = K;
    qsort(rows, m, sizeof(uint64_t) * K, cmp_rows);
    uint64_t w = 1;
    for (uint64_t r = 1; r < m; ++r) {
        if (memcmp(rows + r * K, rows + (w - 1) * K, sizeof(uint64_t) * K) != 0) {
            if (w != r) memcpy(rows + w * K, rows + r * K, sizeof(uint64_t) * K);
            ++w;
        }
    }
    return w;
}

/* ---------------------------------------------------------------- Eq. 1 ---- */
/* B^c: every record of the class, and the intersection of every pair of
 * records taken once (i < j), without the empty set, sorted and unique.
 * Returns the number of distinct candidates; *out owns count*K words. */
static int candidates(const uint64_t *X, uint64_t n, uint32_t K, uint64_t **out,
                      uint64_t *count)
{
    uint64_t m_max = n + n * (n - (n ? 1 : 0)) / 2;
    uint64_t *rows = (uint64_t *)malloc(sizeof(uint64_t) * K * (m_max ? m_max : 1));
    if (!rows) return IGO_E_NOMEM;
    uint64_t m = 0;
    for (uint64_t i = 0; i < n; ++i) {            /* the records themselves */
        if (is_empty(X + i * K, K)) continue;
        memcpy(rows + m * K, X + i * K, sizeof(uint64_t) * K);
        ++m;
    }
    for (uint64_t i = 0; i < n; ++i) {            /* pairwise intersections */
        for (uint64_t j = i + 1; j < n; ++j) {
            uint64_t *b = rows + m * K;
            int nz = 0;
            for (uint32_t k = 0; k < K; ++k) {
                b[k] = X[i * K + k] & X[j * K + k];
                nz |= b[k] != 0;
            }
            if (nz) ++m;
        }
    }
    *count = sort_unique(rows, m, K);
    *out = rows;
    return IGO_OK;
}

/* ---------------------------------------------------------------- Eq. 3 ---- */
/* Position (1-based) of the first record of Xo that contains b, scanning Xo in
 * input order, or 0 when none does (b is then coherent). */
static uint64_t first_cover(const uint64_t *b, const uint64_t *Xo, uint64_t no, uint32_t K)
{
    for (uint64_t t = 0; t < no; ++t)
        if (subset(b, Xo + t * K, K)) return t + 1;
    return 0;
}

/* ---------------------------------------------------------------- Eq. 2 ---- */
/* f_c(b): number of class-c records that contain b (repeats counted). */
static uint32_t support(const uint64_t *b, const uint64_t *X, uint64_t n, uint32_t K)
{
    uint32_t f = 0;
    for (uint64_t i = 0; i < n; ++i) f += (uint32_t)subset(b, X + i * K, K);
    return f;
}

/* One class: candidates, coherence against the other class, weights. */
static int fit_class(const uint64_t *Xc, uint64_t nc, const uint64_t *Xo, uint64_t no,
                     uint32_t K, igo_model *m, int c)
{
    uint64_t *cand = NULL, ncand = 0;
    int rc = candidates(Xc, nc, K, &cand, &ncand);
    if (rc) return rc;
    m->pairs[c] = nc * (nc - (nc ? 1 : 0)) / 2;
    m->distinct[c] = ncand;
    uint64_t *tpos = (uint64_t *)malloc(sizeof(uint64_t) * (ncand ? ncand : 1));
    if (!tpos) { free(cand); return IGO_E_NOMEM; }
    uint64_t tests = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : tests)
    for (int64_t q = 0; q < (int64_t)ncand; ++q) {
        uint64_t t = first_cover(cand + (uint64_t)q * K, Xo, no, K);
        tpos[q] = t;
        tests += t ? t : no;
    }
    m->tests[c] = tests;
    uint64_t keep = 0;
    for (uint64_t q = 0; q < ncand; ++q) keep += tpos[q] == 0;
    m->count[c] = keep;
    m->words[c] = (uint64_t *)malloc(sizeof(uint64_t) * K * (keep ? keep : 1));
    m->f[c] = (uint32_t *)malloc(sizeof(uint32_t) * (keep ? keep : 1));
    m->S[c] = (int64_t *)malloc(sizeof(int64_t) * (keep ? keep : 1));
    if (!m->words[c] || !m->f[c] || !m->S[c]) { free(cand); free(tpos); return IGO_E_NOMEM; }
    uint64_t w = 0;
    for (uint64_t q = 0; q < ncand; ++q)
        if (tpos[q] == 0) memcpy(m->words[c] + (w++) * K, cand + q * K, sizeof(uint64_t) * K);
    free(cand);
    free(tpos);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t p = 0; p < (int64_t)keep; ++p) {
        const uint64_t *b = m->words[c] + (uint64_t)p * K;
        uint32_t f = support(b, Xc, nc, K);
        uint32_t len = popcount_row(b, K);
        m->f[c][p] = f;
        m->S[c][p] = (int64_t)f * (int64_t)len * (int64_t)len;
    }
    return IGO_OK;
}

void igo_free(igo_model *m)
{
    if (!m) return;
    for (int c = 0; c < 2; ++c) {
        free(m->words[c]); free(m->f[c]); free(m->S[c]);
        m->words[c] = NULL; m->f[c] = NULL; m->S[c] = NULL;
    }
}

/* Split the packed records by label, keeping input order within a class. */
static int split_classes(const uint64_t *R, uint64_t n, uint32_t K, const uint8_t *labels,
                         uint64_t *Xs[2], uint64_t ns[2])
{
    ns[0] = ns[1] = 0;
    for (uint64_t i = 0; i < n; ++i) {
        if (labels[i] > 1) return IGO_E_INVAL;
        ns[labels[i]]++;
    }
    for (int c = 0; c < 2; ++c) {
        Xs[c] = (uint64_t *)malloc(sizeof(uint64_t) * K * (ns[c] ? ns[c] : 1));
        if (!Xs[c]) return IGO_E_NOMEM;
    }
    uint64_t at[2] = {0, 0};
    for (uint64_t i = 0; i < n; ++i) {
        int c = labels[i];
        memcpy(Xs[c] + (at[c]++) * K, R + i * K, sizeof(uint64_t) * K);
    }
    return IGO_OK;
}

/* Fit both classes from code rows (labels: 0 normal, 1 attack). */
int igo_fit(const uint16_t *codes, uint64_t n, uint32_t d, const uint8_t *labels,
            const uint16_t *nbins, igo_model *m)
{
    memset(m, 0, sizeof(*m));
    uint32_t L, K;
    if (universe(nbins, d, &L, &K)) return IGO_E_INVAL;
    m->K = K; m->L = L; m->d = d;
    uint64_t *R = (uint64_t *)malloc(sizeof(uint64_t) * K * (n ? n : 1));
    if (!R) return IGO_E_NOMEM;
    int rc = igo_pack(codes, n, d, nbins, K, R);
    for (uint64_t i = 0; rc == IGO_OK && i < n * d; ++i)
        if (codes[i] == IGO_ABSENT) rc = IGO_E_INVAL;   /* records carry every feature */
    uint64_t *Xs[2] = {NULL, NULL}, ns[2];
    if (rc == IGO_OK) rc = split_classes(R, n, K, labels, Xs, ns);
    free(R);
    if (rc == IGO_OK) {
        m->n_class[0] = ns[0]; m->n_class[1] = ns[1];
        for (int c = 0; c < 2 && rc == IGO_OK; ++c)
            rc = fit_class(Xs[c], ns[c], Xs[1 - c], ns[1 - c], K, m, c);
    }
    free(Xs[0]); free(Xs[1]);
    if (rc) igo_free(m);
    return rc;
}

/* ---------------------------------------------------------------- Eq. 4 ---- */
/* A(x) and N(x) for n_flows packed flows against a fitted model. */
int igo_score_packed(const igo_model *m, const uint64_t *T, uint64_t n_flows, int64_t *A, int64_t *N)
{
    const uint32_t K = m->K;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < (int64_t)n_flows; ++t) {
        const uint64_t *x = T + (uint64_t)t * K;
        int64_t a = 0, nn = 0;
        for (uint64_t p = 0; p < m->count[1]; ++p)
            if (subset(m->words[1] + p * K, x, K)) a += m->S[1][p];
        for (uint64_t p = 0; p < m->count[0]; ++p)
            if (subset(m->words[0] + p * K, x, K)) nn += m->S[0][p];
        A[t] = a;
        N[t] = nn;
    }
    return IGO_OK;
}

int igo_score(const igo_model *m, const uint16_t *codes, uint64_t n_flows, uint32_t d,
              const uint16_t *nbins, int64_t *A, int64_t *N)
{
    uint32_t L, K;
    if (universe(nbins, d, &L, &K) || K != m->K || d != m->d) return IGO_E_INVAL;
    uint64_t *T = (uint64_t *)malloc(sizeof(uint64_t) * K * (n_flows ? n_flows : 1));
    if (!T) return IGO_E_NOMEM;
    int rc = igo_pack(codes, n_flows, d, nbins, K, T);
    if (rc == IGO_OK) rc = igo_score_packed(m, T, n_flows, A, N);
    free(T);
    return rc;
}

/* Model built from given pattern code rows and supports (for scoring a given
 * pattern set): pack each pattern (Eq. 5) and weight it by Eq. 2 with the given
 * f.  Rows stay in the order given (scores do not depend on it).  Patterns must
 * be distinct and non-empty. */
int igo_model_from_patterns(const uint16_t *codes0, const uint32_t *f0, uint64_t m0,
                            const uint16_t *codes1, const uint32_t *f1, uint64_t m1,
                            uint32_t d, const uint16_t *nbins, igo_model *m)
{
    memset(m, 0, sizeof(*m));
    uint32_t L, K;
    if (universe(nbins, d, &L, &K)) return IGO_E_INVAL;
    m->K = K; m->L = L; m->d = d;
    const uint16_t *cs[2] = {codes0, codes1};
    const uint32_t *fs[2] = {f0, f1};
    uint64_t ms[2] = {m0, m1};
    for (int c = 0; c < 2; ++c) {
        m->count[c] = ms[c];
        m->words[c] = (uint64_t *)malloc(sizeof(uint64_t) * K * (ms[c] ? ms[c] : 1));
        m->f[c] = (uint32_t *)malloc(sizeof(uint32_t) * (ms[c] ? ms[c] : 1));
        m->S[c] = (int64_t *)malloc(sizeof(int64_t) * (ms[c] ? ms[c] : 1));
        if (!m->words[c] || !m->f[c] || !m->S[c]) { igo_free(m); return IGO_E_NOMEM; }
        if (igo_pack(cs[c], ms[c], d, nbins, K, m->words[c])) { igo_free(m); return IGO_E_INVAL; }
        for (uint64_t p = 0; p < ms[c]; ++p) {
            uint32_t len = popcount_row(m->words[c] + p * K, K);
            m->f[c][p] = fs[c][p];
            m->S[c][p] = (int64_t)fs[c][p] * (int64_t)len * (int64_t)len;
        }
    }
    return IGO_OK;
}

/* ----------------------------------------------- one-at-a-time evaluation ---- */
/* The score of single flows straight from the definitions, without a fitted
 * pattern set: for each flow x, every member b of B^c with b subset of x is
 * enumerated (Eq. 1), kept if no other-class record contains it (Eq. 3),
 * weighted by Eq. 2 and summed (Eq. 4).  Used on samples of large workloads,
 * where fitting the whole oracle model would take too long. */
static int64_t direct_class_score(const uint64_t *x, const uint64_t *Xc, uint64_t nc,
                                  const uint64_t *Xo, uint64_t no, uint32_t K)
{
    /* members of B^c inside x: intersections of records, restricted to x */
    uint64_t cap = 1024, m = 0;
    uint64_t *rows = (uint64_t *)malloc(sizeof(uint64_t) * K * cap);
    uint64_t *b = (uint64_t *)malloc(sizeof(uint64_t) * K);
    if (!rows || !b) { free(rows); free(b); return -1; }
    for (uint64_t i = 0; i < nc; ++i) {
        for (uint64_t j = i; j < nc; ++j) {          /* j == i: the record itself */
            int nz = 0;
            for (uint32_t k = 0; k < K; ++k) { b[k] = Xc[i * K + k] & Xc[j * K + k]; nz |= b[k] != 0; }
            if (!nz || !subset(b, x, K)) continue;
            if (m == cap) {
                cap *= 2;
                uint64_t *nr = (uint64_t *)realloc(rows, sizeof(uint64_t) * K * cap);
                if (!nr) { free(rows); free(b); return -1; }
                rows = nr;
            }
            memcpy(rows + m * K, b, sizeof(uint64_t) * K);
            ++m;
        }
    }
    uint64_t u = sort_unique(rows, m, K);
    int64_t s = 0;
    for (uint64_t q = 0; q < u; ++q) {
        const uint64_t *bb = rows + q * K;
        if (first_cover(bb, Xo, no, K)) continue;
        uint32_t f = support(bb, Xc, nc, K);
        uint32_t len = popcount_row(bb, K);
        s += (int64_t)f * (int64_t)len * (int64_t)len;
    }
    free(rows);
    free(b);
    return s;
}

int igo_score_direct(const uint16_t *codes, uint64_t n, uint32_t d, const uint8_t *labels,
                     const uint16_t *nbins, const uint16_t *flows, uint64_t n_flows,
                     int64_t *A, int64_t *N)
{
    uint32_t L, K;
    if (universe(nbins, d, &L, &K)) return IGO_E_INVAL;
    uint64_t *R = (uint64_t *)malloc(sizeof(uint64_t) * K * (n ? n : 1));
    uint64_t *T = (uint64_t *)malloc(sizeof(uint64_t) * K * (n_flows ? n_flows : 1));
    if (!R || !T) { free(R); free(T); return IGO_E_NOMEM; }
    int rc = igo_pack(codes, n, d, nbins, K, R);
    if (rc == IGO_OK) rc = igo_pack(flows, n_flows, d, nbins, K, T);
    uint64_t *Xs[2] = {NULL, NULL}, ns[2];
    if (rc == IGO_OK) rc = split_classes(R, n, K, labels, Xs, ns);
    free(R);
    if (rc == IGO_OK) {
        // serial over classes, parallel over flows
        int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
        for (int64_t t = 0; t < (int64_t)n_flows; ++t) {
            const uint64_t *x = T + (uint64_t)t * K;
            int64_t a = direct_class_score(x, Xs[1], ns[1], Xs[0], ns[0], K);
            int64_t nn = direct_class_score(x, Xs[0], ns[0], Xs[1], ns[1], K);
            if (a < 0 || nn < 0) bad = 1;
            A[t] = a;
            N[t] = nn;
        }
        if (bad) rc = IGO_E_NOMEM;
    }
    free(Xs[0]); free(Xs[1]); free(T);
    return rc;
}

/* Facts about single pairs of class-c records, straight from the definitions:
 * b = x_i AND x_j (i == j gives the record itself), whether b is coherent
 * (Eq. 3), its support f (Eq. 2) and t(b).  i and j index class c's records in
 * input order. */
int igo_pair_facts(const uint16_t *codes, uint64_t n, uint32_t d, const uint8_t *labels,
                   const uint16_t *nbins, int cls, const uint64_t *pi, const uint64_t *pj,
                   uint64_t n_pairs, uint64_t *out_words, uint8_t *out_coherent,
                   uint32_t *out_f, uint64_t *out_t)
{
    uint32_t L, K;
    if (universe(nbins, d, &L, &K) || cls < 0 || cls > 1) return IGO_E_INVAL;
    uint64_t *R = (uint64_t *)malloc(sizeof(uint64_t) * K * (n ? n : 1));
    if (!R) return IGO_E_NOMEM;
    int rc = igo_pack(codes, n, d, nbins, K, R);
    uint64_t *Xs[2] = {NULL, NULL}, ns[2];
    if (rc == IGO_OK) rc = split_classes(R, n, K, labels, Xs, ns);
    free(R);
    if (rc == IGO_OK) {
        const uint64_t *Xc = Xs[cls], *Xo = Xs[1 - cls];
        for (uint64_t q = 0; q < n_pairs; ++q)
            if (pi[q] >= ns[cls] || pj[q] >= ns[cls]) rc = IGO_E_INVAL;
        if (rc == IGO_OK) {
#pragma omp parallel for schedule(dynamic, 4)
            for (int64_t q = 0; q < (int64_t)n_pairs; ++q) {
                uint64_t *b = out_words + (uint64_t)q * K;
                for (uint32_t k = 0; k < K; ++k) b[k] = Xc[pi[q] * K + k] & Xc[pj[q] * K + k];
                /* the empty set lies inside the first other-class record, if any */
                uint64_t t = is_empty(b, K) ? (ns[1 - cls] ? 1 : 0) : first_cover(b, Xo, ns[1 - cls], K);
                out_coherent[q] = (uint8_t)(t == 0 && !is_empty(b, K));
                out_t[q] = t ? t : ns[1 - cls];
                out_f[q] = support(b, Xc, ns[cls], K);
            }
        }
    }
    free(Xs[0]); free(Xs[1]);
    return rc;
}

int igo_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void igo_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
