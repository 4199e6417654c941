/*
 * Identity / coverage reference oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain CPU statement of the quantities the similarity-graph filter uses
 * after alignment.  Only the test suite and the benchmark's CPU-baseline leg
 * load it; the product library never links, includes or calls it.
 *
 * The paper keeps an aligned pair as an edge of the similarity graph when its
 * identity and its coverage reach thresholds (section "Protein similarity
 * search pipeline": identity and coverage are the alignment metrics the graph
 * is formed from; section "Similarity search at scale", program-parameter
 * table: identity threshold 0.30, coverage threshold 0.70).  It does not say
 * which of several optimal alignments the identity is measured on; the
 * reading taken here makes the result unique:
 *
 *   Given a pair's reported local alignment box q[qs..qe] x r[rs..re] (the
 *   score S and coordinates of the aligner), consider every GLOBAL alignment
 *   of q[qs..qe] with r[rs..re] under the same affine gap model (a gap run of
 *   length k costs go + (k-1)*ge; a run in one sequence may directly follow a
 *   run in the other, each paying its own opening).  Among them take the one
 *   that is largest in the order: higher score first, then more identical
 *   aligned pairs ("matches"), then fewer columns (aligned pairs plus gap
 *   positions).  Its score is S (the box is the span of an optimal local
 *   alignment); report (matches, columns).
 *
 *   identity = matches / columns; coverage of each sequence = (qe-qs+1)/m and
 *   (re-rs+1)/n.  With thresholds in thousandths, a pair is kept when
 *   1000*matches >= ani*columns and both 1000*(qe-qs+1) >= cov*m and
 *   1000*(re-rs+1) >= cov*n (integer arithmetic, no rounding).
 *
 * The computation is the textbook three-state (Gotoh) global recurrence over
 * (score, matches, columns) triples compared in that order; triples add along
 * a path and the order is compatible with addition, so the recurrence yields
 * the maximum over all alignments exactly.
 */
#include <stdint.h>
#include <stdlib.h>

typedef struct {
    int64_t s;  /* score */
    int64_t m;  /* identical aligned pairs */
    int64_t c;  /* columns */
    int ok;     /* 0: no alignment reaches this state */
} triple;

static triple none(void)
{
    triple t = {0, 0, 0, 0};
    return t;
}

static triple add(triple a, int64_t s, int64_t m, int64_t c)
{
    if (!a.ok) return a;
    a.s += s;
    a.m += m;
    a.c += c;
    return a;
}

/* a is strictly better than b */
static int better(triple a, triple b)
{
    if (!a.ok) return 0;
    if (!b.ok) return 1;
    if (a.s != b.s) return a.s > b.s;
    if (a.m != b.m) return a.m > b.m;
    return a.c < b.c;
}

static triple best2(triple a, triple b) { return better(b, a) ? b : a; }

/*
 * Global alignment of q[0..m) with r[0..n) (m, n >= 1); scores[24*a + b] is
 * the substitution score of query symbol a against reference symbol b.
 * Writes score, matches and columns.  Returns 0, or -1 on bad arguments /
 * memory.
 */
int oracle_identity_box(const int8_t* q, int32_t m, const int8_t* r, int32_t n, const int8_t* scores,
                        int32_t go, int32_t ge, int64_t* score, int64_t* matches, int64_t* columns)
{
    if (m < 1 || n < 1 || go < 0 || ge < 0) return -1;
    /* rows i = -1..m-1 stored at i+1; H = best of the three states */
    triple* H = (triple*)malloc(sizeof(triple) * (size_t)(n + 1) * 2);
    triple* F = (triple*)malloc(sizeof(triple) * (size_t)(n + 1) * 2);
    if (!H || !F) {
        free(H);
        free(F);
        return -1;
    }
    triple* Hp = H;        /* previous row */
    triple* Hc = H + n + 1; /* current row */
    triple* Fp = F;
    triple* Fc = F + n + 1;
    /* row -1: the empty prefix at column -1, then leading gaps in r */
    Hp[0].s = 0;
    Hp[0].m = 0;
    Hp[0].c = 0;
    Hp[0].ok = 1;
    Fp[0] = none();
    for (int32_t j = 0; j < n; ++j) {
        triple e = add(Hp[0], -(int64_t)go - (int64_t)j * ge, 0, j + 1);
        Hp[j + 1] = e;  /* only an E run reaches (-1, j) */
        Fp[j + 1] = none();
    }
    for (int32_t i = 0; i < m; ++i) {
        /* column -1: only a leading gap run in q, of length i+1, reaches it */
        triple col;
        col.s = -(int64_t)go - (int64_t)i * ge;
        col.m = 0;
        col.c = i + 1;
        col.ok = 1;
        Fc[0] = col;
        Hc[0] = col;
        triple E = none();
        for (int32_t j = 0; j < n; ++j) {
            /* E: gap consuming r (horizontal), F: gap consuming q (vertical) */
            E = best2(add(E, -(int64_t)ge, 0, 1), add(Hc[j], -(int64_t)go, 0, 1));
            triple Fv = best2(add(Fp[j + 1], -(int64_t)ge, 0, 1), add(Hp[j + 1], -(int64_t)go, 0, 1));
            const int8_t a = q[i], b = r[j];
            triple d = add(Hp[j], scores[24 * a + b], a == b ? 1 : 0, 1);
            triple h = best2(best2(d, E), Fv);
            Fc[j + 1] = Fv;
            Hc[j + 1] = h;
        }
        triple* t = Hp;
        Hp = Hc;
        Hc = t;
        t = Fp;
        Fp = Fc;
        Fc = t;
    }
    *score = Hp[n].s;
    *matches = Hp[n].m;
    *columns = Hp[n].c;
    free(H);
    free(F);
    return 0;
}

/*
 * One filter record per aligned pair: aligned[5k..5k+4] = score, q_start,
 * q_end, r_start, r_end of pair k (the aligner's output), pairs[2k], [2k+1]
 * the query and reference indices into one code buffer with offsets.
 * out[4k..4k+3] = box score, matches, columns, keep (all 0 when the pair's
 * score is 0).  Returns 0, or -1 on bad input.
 */
int oracle_identity_batch(const int8_t* codes, const int64_t* offsets, int64_t n_seqs, const int32_t* pairs,
                          int64_t n_pairs, const int32_t* aligned, const int8_t* scores, int32_t go, int32_t ge,
                          int32_t ani_permille, int32_t cov_permille, int64_t* out)
{
    for (int64_t k = 0; k < n_pairs; ++k) {
        int64_t* o = out + 4 * k;
        o[0] = o[1] = o[2] = o[3] = 0;
        const int32_t* a = aligned + 5 * k;
        if (a[0] <= 0) continue;
        int64_t qi = pairs[2 * k], ri = pairs[2 * k + 1];
        if (qi < 0 || qi >= n_seqs || ri < 0 || ri >= n_seqs) return -1;
        int64_t m = offsets[qi + 1] - offsets[qi], n = offsets[ri + 1] - offsets[ri];
        if (a[1] < 0 || a[2] < a[1] || a[2] >= m || a[3] < 0 || a[4] < a[3] || a[4] >= n) return -1;
        int64_t s, mt, c;
        if (oracle_identity_box(codes + offsets[qi] + a[1], a[2] - a[1] + 1, codes + offsets[ri] + a[3],
                                a[4] - a[3] + 1, scores, go, ge, &s, &mt, &c) != 0)
            return -1;
        o[0] = s;
        o[1] = mt;
        o[2] = c;
        o[3] = (1000 * mt >= (int64_t)ani_permille * c) && (1000 * (int64_t)(a[2] - a[1] + 1) >= (int64_t)cov_permille * m) &&
               (1000 * (int64_t)(a[4] - a[3] + 1) >= (int64_t)cov_permille * n);
    }
    return 0;
}
