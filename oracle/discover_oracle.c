/*
 * Candidate-discovery reference oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain CPU statement of the step that picks which pairs get aligned.  Only
 * the test suite and the benchmark's CPU-baseline leg load it; the product
 * library never links, includes or calls it.
 *
 * What is computed (the paper, section "Protein similarity search pipeline":
 * the k-mer content of the sequences is a sparse matrix A with one row per
 * sequence and one column per k-mer, whose nonzero (s, x) records that k-mer
 * x occurs in sequence s; candidate pairs come from an overloaded sparse
 * product C = A_q * A_r^T whose semiring multiply yields one and whose add
 * counts, so that C[q][r] is the number of DISTINCT k-mers the two sequences
 * have in common; section "Similarity search at scale", program-parameter
 * table: k = 6 and a common k-mer threshold of 2, i.e. (q, r) is a candidate
 * when C[q][r] >= 2):
 *
 *   1. rows of A: for each sequence, the sorted set of its k-mers (every
 *      window of k consecutive residues; a sequence shorter than k has none);
 *   2. columns of A_r: for each k-mer, the references that hold it;
 *   3. C row by row (Gustavson): for every k-mer x of query q, add one to the
 *      accumulator of every reference that holds x;
 *   4. keep C[q][r] >= min_shared, subject to the pair filter below.
 *
 * Pair filters for a search of a set against itself (section "Load balancing
 * techniques": C is symmetric, so each unordered pair needs one alignment and
 * the diagonal none):
 *   mode 0  every (q, r) pair (two different sets, or the full square);
 *   mode 1  q < r (the strictly upper triangle; the triangularity scheme);
 *   mode 2  index-based scheme: below the diagonal (q > r) keep a pair whose
 *           indices have equal parity, above it (q < r) one whose parities
 *           differ; the diagonal is dropped.
 *
 * Output order: by query, then by reference, ascending.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define KMER_ALPHABET 24

typedef struct {
    int64_t* ptr;   /* [n + 1] */
    int64_t* cols;  /* sorted distinct k-mer codes of each row */
} kmer_rows;

static int cmp_i64(const void* a, const void* b)
{
    int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
    return (x > y) - (x < y);
}

/* Step 1: A as sorted distinct rows.  Codes are symbol indices 0..23; a
 * k-mer's code is its base-24 number. */
static int build_rows(const int8_t* codes, const int64_t* offs, int64_t n, int k, kmer_rows* A)
{
    int64_t total = 0;
    for (int64_t s = 0; s < n; ++s) {
        int64_t L = offs[s + 1] - offs[s];
        if (L < 0) return -1;
        if (L >= k) total += L - k + 1;
    }
    A->ptr = (int64_t*)malloc((size_t)(n + 1) * sizeof(int64_t));
    A->cols = (int64_t*)malloc((size_t)(total > 0 ? total : 1) * sizeof(int64_t));
    if (!A->ptr || !A->cols) return -2;
    int64_t w = 0;
    A->ptr[0] = 0;
    for (int64_t s = 0; s < n; ++s) {
        int64_t L = offs[s + 1] - offs[s];
        int64_t first = w;
        for (int64_t p = 0; p + k <= L; ++p) {
            int64_t x = 0;
            for (int t = 0; t < k; ++t) {
                int c = codes[offs[s] + p + t];
                if (c < 0 || c >= KMER_ALPHABET) return -3;
                x = x * KMER_ALPHABET + c;
            }
            A->cols[w++] = x;
        }
        qsort(A->cols + first, (size_t)(w - first), sizeof(int64_t), cmp_i64);
        int64_t u = first;
        for (int64_t t = first; t < w; ++t)
            if (t == first || A->cols[t] != A->cols[u - 1]) A->cols[u++] = A->cols[t];
        w = u;
        A->ptr[s + 1] = w;
    }
    return 0;
}

typedef struct {
    int64_t kmer;
    int64_t seq;
} entry;

static int cmp_entry(const void* a, const void* b)
{
    const entry* x = (const entry*)a;
    const entry* y = (const entry*)b;
    if (x->kmer != y->kmer) return (x->kmer > y->kmer) - (x->kmer < y->kmer);
    return (x->seq > y->seq) - (x->seq < y->seq);
}

static int keep_pair(int64_t q, int64_t r, int mode)
{
    if (mode == 0) return 1;
    if (q == r) return 0;
    if (mode == 1) return q < r;
    /* mode 2 */
    if (q > r) return (q & 1) == (r & 1);
    return (q & 1) != (r & 1);
}

/*
 * Candidates of the query set against the reference set.  Writes at most
 * `cap` triples (query, reference, shared) in (query, reference) order and
 * returns their total count in *n_found.  Return value: 0 ok, -1 bad
 * offsets, -2 out of memory, -3 a code outside 0..23, -4 bad arguments.
 */
int oracle_discover(const int8_t* q_codes, const int64_t* q_offs, int64_t n_q,
                    const int8_t* r_codes, const int64_t* r_offs, int64_t n_r,
                    int32_t k, int32_t min_shared, int32_t mode, int64_t cap,
                    int32_t* out_q, int32_t* out_r, int32_t* out_shared, int64_t* n_found)
{
    if (k < 1 || k > 12 || n_q < 0 || n_r < 0 || mode < 0 || mode > 2 || !n_found) return -4;
    kmer_rows Aq = {0, 0}, Ar = {0, 0};
    entry* col = NULL;
    int32_t* acc = NULL;
    int64_t* touched = NULL;
    int rc = build_rows(q_codes, q_offs, n_q, k, &Aq);
    if (rc == 0) rc = build_rows(r_codes, r_offs, n_r, k, &Ar);
    int64_t nr_ent = (rc == 0) ? Ar.ptr[n_r] : 0;

    /* Step 2: the columns of A_r, as (k-mer, reference) sorted by k-mer. */
    if (rc == 0) {
        col = (entry*)malloc((size_t)(nr_ent > 0 ? nr_ent : 1) * sizeof(entry));
        acc = (int32_t*)calloc((size_t)(n_r > 0 ? n_r : 1), sizeof(int32_t));
        touched = (int64_t*)malloc((size_t)(n_r > 0 ? n_r : 1) * sizeof(int64_t));
        if (!col || !acc || !touched) rc = -2;
    }
    if (rc == 0) {
        for (int64_t s = 0; s < n_r; ++s)
            for (int64_t t = Ar.ptr[s]; t < Ar.ptr[s + 1]; ++t) {
                col[t].kmer = Ar.cols[t];
                col[t].seq = s;
            }
        qsort(col, (size_t)nr_ent, sizeof(entry), cmp_entry);
    }

    /* Steps 3 and 4: one row of C at a time. */
    int64_t found = 0;
    for (int64_t q = 0; rc == 0 && q < n_q; ++q) {
        int64_t nt = 0;
        for (int64_t t = Aq.ptr[q]; t < Aq.ptr[q + 1]; ++t) {
            int64_t x = Aq.cols[t];
            int64_t lo = 0, hi = nr_ent; /* first entry with kmer >= x */
            while (lo < hi) {
                int64_t mid = lo + (hi - lo) / 2;
                if (col[mid].kmer < x) lo = mid + 1; else hi = mid;
            }
            for (int64_t e = lo; e < nr_ent && col[e].kmer == x; ++e) {
                int64_t r = col[e].seq;
                if (acc[r]++ == 0) touched[nt++] = r;
            }
        }
        qsort(touched, (size_t)nt, sizeof(int64_t), cmp_i64);
        for (int64_t t = 0; t < nt; ++t) {
            int64_t r = touched[t];
            if (acc[r] >= min_shared && keep_pair(q, r, mode)) {
                if (found < cap) {
                    out_q[found] = (int32_t)q;
                    out_r[found] = (int32_t)r;
                    if (out_shared) out_shared[found] = acc[r];
                }
                ++found;
            }
            acc[r] = 0;
        }
    }
    *n_found = found;
    free(Aq.ptr); free(Aq.cols); free(Ar.ptr); free(Ar.cols);
    free(col); free(acc); free(touched);
    return rc;
}

/* Number of distinct k-mers of each sequence (the diagonal of A A^T). */
int oracle_distinct_kmers(const int8_t* codes, const int64_t* offs, int64_t n, int32_t k, int64_t* out)
{
    if (k < 1 || k > 12 || n < 0) return -4;
    kmer_rows A = {0, 0};
    int rc = build_rows(codes, offs, n, k, &A);
    if (rc == 0)
        for (int64_t s = 0; s < n; ++s) out[s] = A.ptr[s + 1] - A.ptr[s];
    free(A.ptr); free(A.cols);
    return rc;
}
