/*
 * Smith-Waterman / Gotoh reference oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * This file is the plain, slow, obviously-correct CPU statement of what the
 * batched alignment path computes.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it; the product library never
 * links, includes or calls it, and shares no code, table or constant with it.
 *
 * What is computed (the paper, section "Load balancing techniques": the aligner
 * is a Smith-Waterman variant that fills the whole dynamic-programming matrix,
 * so the cost of a pair is proportional to m*n; section "Performance results",
 * table of program parameters: affine gaps with separate open and extension
 * penalties, integer scores):
 *
 *   For 0 <= i < m (query) and 0 <= j < n (reference), with H = 0 outside the
 *   matrix and E, F = minus infinity outside it,
 *     E[i][j] = max(E[i][j-1] - ge, H[i][j-1] - go)      gap consuming reference
 *     F[i][j] = max(F[i-1][j] - ge, H[i-1][j] - go)      gap consuming query
 *     H[i][j] = max(0, H[i-1][j-1] + B[q_i][r_j], E[i][j], F[i][j])
 *   A gap run of length k costs go + (k-1)*ge (Gotoh's affine model).
 *   score S = max(0, max H).
 *
 * Tie rule (the paper is silent; this is the reading the whole project uses):
 *   end   = the lexicographically smallest (i, then j) cell with H = S,
 *           i.e. the first hit of a row-major scan with a strict '>' update;
 *   start = run the same recurrence on the reversed prefixes q[0..i_e] and
 *           r[0..j_e]; the first (row-major) reversed cell (a, b) with H' = S
 *           gives q_start = i_e - a, r_start = j_e - b.  This selects, among the
 *           optimal alignments that end at the reported end, the one with the
 *           largest query start and then the largest reference start.
 *   S = 0 reports every coordinate as -1.  Coordinates are 0-based inclusive.
 *
 * Validity domain: 1 <= go, 0 <= ge <= go.  Under go >= 1 every optimal local
 * alignment starts and ends with an aligned residue pair, which is what makes
 * the reversed-prefix start rule exact.
 *
 * Everything is int32 with a "minus infinity" of -2^30; no value can overflow
 * for sequence lengths below 2^24 and penalties up to 2^20.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#define ORACLE_NEG (-(1 << 30))
#define ORACLE_NSYM 24

typedef struct {
    int32_t score, q_start, q_end, r_start, r_end;
} oracle_result;

/* ------------------------------------------------------------------------ */
/* Substitution matrix, read from the NCBI-format text table.               */
/* ------------------------------------------------------------------------ */

typedef struct {
    char letters[ORACLE_NSYM + 1];
    int8_t score[ORACLE_NSYM][ORACLE_NSYM]; /* [query symbol][reference symbol] */
    int8_t code_of[256];                    /* ASCII -> index, -1 if not a symbol */
} oracle_matrix;

/* Parse "# comment" lines, one header line of symbols, then one line per row
 * (row symbol followed by its scores).  Returns 0 on success. */
int oracle_matrix_parse(const char* text, oracle_matrix* mx)
{
    memset(mx, 0, sizeof(*mx));
    memset(mx->code_of, -1, sizeof(mx->code_of));
    const char* p = text;
    int have_header = 0, rows = 0;
    while (*p) {
        const char* eol = strchr(p, '\n');
        size_t len = eol ? (size_t)(eol - p) : strlen(p);
        char line[512];
        if (len >= sizeof(line)) return -1;
        memcpy(line, p, len);
        line[len] = 0;
        p = eol ? eol + 1 : p + len;
        char* s = line;
        while (*s == ' ' || *s == '\t' || *s == '\r') ++s;
        if (*s == 0 || *s == '#') continue;
        if (!have_header) {
            int k = 0;
            for (char* t = strtok(s, " \t\r"); t; t = strtok(NULL, " \t\r")) {
                if (k >= ORACLE_NSYM || strlen(t) != 1) return -2;
                mx->letters[k] = t[0];
                mx->code_of[(unsigned char)t[0]] = (int8_t)k;
                ++k;
            }
            if (k != ORACLE_NSYM) return -3;
            have_header = 1;
            continue;
        }
        char* t = strtok(s, " \t\r");
        if (!t || strlen(t) != 1 || mx->code_of[(unsigned char)t[0]] < 0) return -4;
        int row = mx->code_of[(unsigned char)t[0]];
        int k = 0;
        for (t = strtok(NULL, " \t\r"); t; t = strtok(NULL, " \t\r")) {
            if (k >= ORACLE_NSYM) return -5;
            mx->score[row][k++] = (int8_t)atoi(t);
        }
        if (k != ORACLE_NSYM) return -6;
        ++rows;
    }
    return (have_header && rows == ORACLE_NSYM) ? 0 : -7;
}

/* ASCII letters -> symbol indices.  Returns the number of residues that are not
 * symbols of the matrix (those are written as -1). */
int64_t oracle_encode(const oracle_matrix* mx, const char* ascii, int64_t n, int8_t* out)
{
    int64_t bad = 0;
    for (int64_t k = 0; k < n; ++k) {
        out[k] = mx->code_of[(unsigned char)ascii[k]];
        if (out[k] < 0) ++bad;
    }
    return bad;
}

/* ------------------------------------------------------------------------ */
/* The recurrence.                                                          */
/* ------------------------------------------------------------------------ */

static inline int32_t imax(int32_t a, int32_t b) { return a > b ? a : b; }

/* Fill the whole m x n matrix row by row (query rows i, reference columns j).
 * The residue of row i is q[qdir*i] and of column j is r[rdir*j], so a
 * negative direction walks a sequence backwards from the given pointer (that
 * is how the reversed prefixes of the start pass are read).  Returns the best
 * score and its first cell in row-major order.  Hrow/Frow hold n int32; when
 * Hall is not NULL every H[i][j] is also stored there (row-major, m x n). */
static int32_t fill_matrix(const int8_t* q, int64_t qdir, int32_t m,
                           const int8_t* r, int64_t rdir, int32_t n,
                           const oracle_matrix* mx, int32_t go, int32_t ge,
                           int32_t* Hrow, int32_t* Frow, int32_t* best_i, int32_t* best_j,
                           int32_t* Hall)
{
    int32_t best = 0;
    *best_i = -1;
    *best_j = -1;
    for (int32_t j = 0; j < n; ++j) {
        Hrow[j] = 0;          /* H[-1][j] */
        Frow[j] = ORACLE_NEG; /* F[-1][j] */
    }
    for (int32_t i = 0; i < m; ++i) {
        const int8_t* brow = mx->score[q[qdir * i]];
        int32_t diag = 0;         /* H[i-1][j-1], starts as H[i-1][-1] = 0 */
        int32_t left = 0;         /* H[i][j-1], starts as H[i][-1] = 0 */
        int32_t e = ORACLE_NEG;   /* E[i][j-1] */
        for (int32_t j = 0; j < n; ++j) {
            int32_t up = Hrow[j]; /* H[i-1][j] */
            e = imax(e - ge, left - go);
            int32_t f = imax(Frow[j] - ge, up - go);
            int32_t h = diag + brow[r[rdir * j]];
            h = imax(h, e);
            h = imax(h, f);
            h = imax(h, 0);
            Frow[j] = f;
            Hrow[j] = h;
            if (Hall) Hall[(int64_t)i * n + j] = h;
            diag = up;
            left = h;
            if (h > best) { /* strict: keeps the first cell in row-major order */
                best = h;
                *best_i = i;
                *best_j = j;
            }
        }
    }
    return best;
}

/* One pair.  q and r are symbol indices (0..23).  Returns 0, or a negative
 * value on invalid arguments or an internal inconsistency. */
int oracle_align(const int8_t* q, int32_t m, const int8_t* r, int32_t n,
                 const oracle_matrix* mx, int32_t go, int32_t ge, oracle_result* out)
{
    out->score = 0;
    out->q_start = out->q_end = out->r_start = out->r_end = -1;
    if (go < 1 || ge < 0 || ge > go || m < 0 || n < 0) return -1;
    for (int32_t i = 0; i < m; ++i)
        if (q[i] < 0 || q[i] >= ORACLE_NSYM) return -2;
    for (int32_t j = 0; j < n; ++j)
        if (r[j] < 0 || r[j] >= ORACLE_NSYM) return -2;
    if (m == 0 || n == 0) return 0;

    int32_t* Hrow = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* Frow = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!Hrow || !Frow) { free(Hrow); free(Frow); return -3; }

    int32_t ie, je;
    int32_t S = fill_matrix(q, 1, m, r, 1, n, mx, go, ge, Hrow, Frow, &ie, &je, NULL);
    int rc = 0;
    if (S > 0) {
        /* Start pass: the same recurrence over the reversed prefixes. */
        int32_t a, b;
        int32_t S2 = fill_matrix(q + ie, -1, ie + 1, r + je, -1, je + 1, mx, go, ge,
                                 Hrow, Frow, &a, &b, NULL);
        if (S2 != S) {
            rc = -4; /* cannot happen under the validity domain */
        } else {
            out->score = S;
            out->q_end = ie;
            out->r_end = je;
            out->q_start = ie - a;
            out->r_start = je - b;
        }
    }
    free(Hrow);
    free(Frow);
    return rc;
}

/* Whole-matrix dump for small cases (tests only): H as int32 [m][n]. */
int oracle_fill_H(const int8_t* q, int32_t m, const int8_t* r, int32_t n,
                  const oracle_matrix* mx, int32_t go, int32_t ge, int32_t* H)
{
    if (go < 1 || ge < 0 || ge > go || m < 0 || n < 0) return -1;
    if (m == 0 || n == 0) return 0;
    int32_t* Hrow = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* Frow = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!Hrow || !Frow) { free(Hrow); free(Frow); return -3; }
    int32_t bi, bj;
    fill_matrix(q, 1, m, r, 1, n, mx, go, ge, Hrow, Frow, &bi, &bj, H);
    free(Hrow);
    free(Frow);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Batch driver: pairs are independent, so a pool of threads takes pairs one */
/* at a time; each pair is still computed single-threaded by oracle_align.   */
/* ------------------------------------------------------------------------ */

typedef struct {
    const int8_t* codes;
    const int64_t* offsets;
    int64_t n_seqs;
    const int32_t* pairs;
    int64_t n_pairs;
    const oracle_matrix* mx;
    int32_t go, ge;
    oracle_result* out;
    int64_t next;
    int error;
    pthread_mutex_t lock;
} batch_job;

static void* batch_worker(void* arg)
{
    batch_job* job = (batch_job*)arg;
    for (;;) {
        pthread_mutex_lock(&job->lock);
        int64_t k = job->next++;
        pthread_mutex_unlock(&job->lock);
        if (k >= job->n_pairs) break;
        int64_t qi = job->pairs[2 * k], ri = job->pairs[2 * k + 1];
        oracle_result* o = &job->out[k];
        if (qi < 0 || qi >= job->n_seqs || ri < 0 || ri >= job->n_seqs) {
            o->score = -1;
            o->q_start = o->q_end = o->r_start = o->r_end = -1;
            continue;
        }
        int64_t q0 = job->offsets[qi], q1 = job->offsets[qi + 1];
        int64_t r0 = job->offsets[ri], r1 = job->offsets[ri + 1];
        int rc = oracle_align(job->codes + q0, (int32_t)(q1 - q0), job->codes + r0,
                              (int32_t)(r1 - r0), job->mx, job->go, job->ge, o);
        if (rc != 0) {
            pthread_mutex_lock(&job->lock);
            job->error = rc;
            pthread_mutex_unlock(&job->lock);
        }
    }
    return NULL;
}

int oracle_batch(const int8_t* codes, const int64_t* offsets, int64_t n_seqs,
                 const int32_t* pairs, int64_t n_pairs, const oracle_matrix* mx,
                 int32_t go, int32_t ge, oracle_result* out, int n_threads)
{
    batch_job job;
    memset(&job, 0, sizeof(job));
    job.codes = codes;
    job.offsets = offsets;
    job.n_seqs = n_seqs;
    job.pairs = pairs;
    job.n_pairs = n_pairs;
    job.mx = mx;
    job.go = go;
    job.ge = ge;
    job.out = out;
    pthread_mutex_init(&job.lock, NULL);
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 256) n_threads = 256;
    pthread_t tid[256];
    for (int t = 0; t < n_threads; ++t) pthread_create(&tid[t], NULL, batch_worker, &job);
    for (int t = 0; t < n_threads; ++t) pthread_join(tid[t], NULL);
    pthread_mutex_destroy(&job.lock);
    return job.error;
}

size_t oracle_matrix_size(void) { return sizeof(oracle_matrix); }
