/*
 * Runs the oracle's entry points on small inputs, for builds under
 * AddressSanitizer and UndefinedBehaviorSanitizer (and OpenMP), and checks
 * what the mathematics fixes independently of the oracle's code:
 *   - K_n has C(n,3) triangles; with time 7 + 2^k on the edges at vertex 0
 *     and 7 elsewhere, hist[k] = C(n-1,2) and hist[0] = C(n-1,3);
 *   - a random multigraph with duplicates, reversed copies and self-loops:
 *     the triangle count equals a brute force over vertex triples of its
 *     adjacency matrix, every reduction sums to it, the record list holds it,
 *     and participation counts sum to three times it;
 *   - the directed census of the same graph sums to its triangle count;
 *   - empty inputs and self-loops only give nothing.
 * Prints "ok <name>" or "FAIL <name>" per check and PASSED at the end.
 */
#include <stdio.h>

#include "../../oracle/oracle.c"

static int failures = 0;

static void check(int cond, const char *name)
{
    printf("%s %s\n", cond ? "ok" : "FAIL", name);
    if (!cond) ++failures;
}

static uint64_t lcg(uint64_t *s)
{
    *s = *s * 6364136223846793005ull + 1442695040888963407ull;
    return *s >> 33;
}

static uint64_t sum_u64(const uint64_t *a, size_t n)
{
    uint64_t s = 0;
    for (size_t i = 0; i < n; ++i) s += a[i];
    return s;
}

static void complete_graph(uint32_t n, uint32_t k)
{
    const uint64_t m = (uint64_t)n * (n - 1) / 2;
    uint32_t *u = malloc(m * 4), *v = malloc(m * 4), *t = malloc(m * 4);
    uint64_t e = 0;
    for (uint32_t a = 0; a < n; ++a)
        for (uint32_t b = a + 1; b < n; ++b, ++e) {
            u[e] = a;
            v[e] = b;
            t[e] = 7u + (a == 0 ? (1u << k) : 0u);
        }
    orc_spec sp;
    memset(&sp, 0, sizeof(sp));
    sp.outputs = ORC_OUT_COUNT | ORC_OUT_CLOSE_HIST | ORC_OUT_OPEN_CLOSE;
    sp.n_labels = 1;
    orc_result *r = calloc(1, sizeof(orc_result));
    uint64_t nrec = 0;
    const int rc = oracle_survey(n, m, u, v, t, NULL, NULL, &sp, r, 2, NULL, 0, &nrec);
    check(rc == 0, "K_n survey returns 0");
    check(r->triangles == choose(n, 3), "K_n has C(n,3) triangles");
    check(r->close_hist[k] == choose(n - 1, 2), "K_n hist[k] = C(n-1,2)");
    check(r->close_hist[0] == choose(n - 1, 3), "K_n hist[0] = C(n-1,3)");
    check(sum_u64(r->open_close, 1024) == r->triangles, "K_n joint histogram sums to T");
    free(r);
    free(u);
    free(v);
    free(t);
}

static void random_multigraph(uint32_t n, uint64_t raw, int threads)
{
    uint64_t seed = 12345 + n;
    uint32_t *src = malloc(raw * 4), *dst = malloc(raw * 4), *ts = malloc(raw * 4);
    uint8_t *lab = malloc(n);
    for (uint64_t i = 0; i < raw; ++i) {
        src[i] = (uint32_t)(lcg(&seed) % n);
        dst[i] = (i % 17 == 0) ? src[i] : (uint32_t)(lcg(&seed) % n); /* some self-loops */
        ts[i] = (uint32_t)(lcg(&seed) & 0xfffff);
    }
    for (uint64_t i = 0; i + 1 < raw; i += 29) { /* reversed duplicates with later times */
        src[i + 1] = dst[i];
        dst[i + 1] = src[i];
        ts[i + 1] = ts[i] + 1;
    }
    for (uint32_t x = 0; x < n; ++x) lab[x] = (uint8_t)(lcg(&seed) % 4);
    uint32_t *u = malloc(raw * 4), *v = malloc(raw * 4), *t = malloc(raw * 4);
    uint8_t *d = malloc(raw);
    const int64_t m = oracle_clean(n, raw, src, dst, ts, u, v, t, d);
    check(m > 0, "clean keeps edges");
    /* brute force over vertex triples of the adjacency matrix */
    uint8_t *adj = calloc((size_t)n * n, 1);
    for (uint64_t i = 0; i < raw; ++i)
        if (src[i] != dst[i]) adj[(size_t)src[i] * n + dst[i]] = adj[(size_t)dst[i] * n + src[i]] = 1;
    uint64_t brute = 0;
    for (uint32_t a = 0; a < n; ++a)
        for (uint32_t b = a + 1; b < n; ++b) {
            if (!adj[(size_t)a * n + b]) continue;
            for (uint32_t c = b + 1; c < n; ++c) brute += adj[(size_t)a * n + c] & adj[(size_t)b * n + c];
        }
    orc_spec sp;
    memset(&sp, 0, sizeof(sp));
    sp.outputs = ORC_OUT_COUNT | ORC_OUT_CLOSE_HIST | ORC_OUT_LABEL_TABLE | ORC_OUT_SPREAD | ORC_OUT_OPEN_CLOSE |
                 ORC_OUT_MAX_EDGE | ORC_OUT_DEGREE_TABLE | ORC_OUT_DIRECTED;
    sp.n_labels = 4;
    sp.spread_lt = 1u << 19;
    sp.max_edge_shift = 10;
    orc_result *r = calloc(1, sizeof(orc_result));
    uint64_t nrec = 0;
    orc_tri *rec = calloc(brute + 1, sizeof(orc_tri));
    int rc = oracle_survey(n, (uint64_t)m, u, v, t, d, lab, &sp, r, threads, rec, brute + 1, &nrec);
    check(rc == 0, "survey returns 0");
    check(r->triangles == brute, "triangle count equals the brute force");
    check(nrec == brute, "one record per triangle");
    check(sum_u64(r->close_hist, 32) == brute, "closure histogram sums to T");
    check(sum_u64(r->label_table, ORC_TABLE_MAX) == brute, "label table sums to T");
    check(sum_u64(r->open_close, 1024) == brute, "joint histogram sums to T");
    check(sum_u64(r->degree_table, ORC_DEGREE_MAX) == brute, "degree table sums to T");
    check(sum_u64(r->directed, 7) == brute, "directed census sums to T");
    check(r->spread_count <= brute, "spread count at most T");
    {
        /* Algorithm 3's values: one per distinct-label triangle, as many as
         * the binned output counts, each the largest time of a record */
        const uint64_t want = sum_u64(r->max_edge, 1024);
        uint32_t *mv = calloc(want + 1, sizeof(uint32_t));
        uint64_t got = 0, distinct = 0;
        orc_result *r2 = calloc(1, sizeof(orc_result));
        memset(&sp, 0, sizeof(sp));
        sp.n_labels = 4;
        rc = oracle_max_edge_values(n, (uint64_t)m, u, v, t, lab, &sp, r2, threads, mv, want + 1, &got);
        check(rc == 0, "max-edge values return 0");
        check(got == want, "one value per distinct-label triangle");
        for (uint64_t i = 0; i < nrec; ++i) {
            const orc_tri *x = &rec[i];
            if (x->l_a == x->l_b || x->l_b == x->l_c || x->l_a == x->l_c) continue;
            ++distinct;
        }
        check(distinct == want, "distinct-label records match the values");
        free(r2);
        free(mv);
    }
    uint64_t *vc = calloc(n, 8), *ec = calloc((size_t)m, 8);
    memset(&sp, 0, sizeof(sp));
    sp.n_labels = 4;
    rc = oracle_participation(n, (uint64_t)m, u, v, t, lab, &sp, vc, ec, threads);
    check(rc == 0, "participation returns 0");
    check(sum_u64(vc, n) == 3 * brute, "vertex participation sums to 3T");
    check(sum_u64(ec, (size_t)m) == 3 * brute, "edge participation sums to 3T");
    free(vc);
    free(ec);
    free(rec);
    free(r);
    free(adj);
    free(u);
    free(v);
    free(t);
    free(d);
    free(src);
    free(dst);
    free(ts);
    free(lab);
}

static void degenerate(void)
{
    uint32_t s[4] = {3, 3, 5, 5}, t4[4] = {1, 2, 3, 4};
    uint32_t u[4], v[4], t[4];
    int64_t m = oracle_clean(8, 4, s, s, t4, u, v, t, NULL);
    check(m == 0, "self-loops only: no edge");
    m = oracle_clean(8, 0, s, s, t4, u, v, t, NULL);
    check(m == 0, "no raw edges: no edge");
    orc_spec sp;
    memset(&sp, 0, sizeof(sp));
    sp.outputs = ORC_OUT_COUNT | ORC_OUT_CLOSE_HIST;
    sp.n_labels = 1;
    orc_result *r = calloc(1, sizeof(orc_result));
    uint64_t nrec = 0;
    const int rc = oracle_survey(8, 0, u, v, t, NULL, NULL, &sp, r, 1, NULL, 0, &nrec);
    check(rc == 0 && r->triangles == 0, "empty graph: no triangle");
    free(r);
}

int main(void)
{
    complete_graph(12, 5);
    complete_graph(3, 2);
    random_multigraph(180, 5000, 1);
    random_multigraph(240, 9000, 4);
    degenerate();
    printf(failures ? "FAILED\n" : "PASSED\n");
    return failures ? 1 : 0;
}
