/*
 * mhs_kernelcpu.c -- the sequential reduction KernelCPU (Section 4.2,
 * Algorithms 4, 5 and 6) as a second, independent CPU implementation of
 * exhaustive DP + MD.
 *
 * TEST INFRASTRUCTURE ONLY, like the rest of this directory: it cross-checks
 * the round-synchronous oracle (mhs_oracle.c) and serves as the paper's own
 * serial comparator.  It shares no code with mhs_oracle.c: where that file
 * tests supersedence and domination with sorted-set differences and
 * inclusions, this one keeps the intersection-count matrices
 *
 *   I^E_ij = |e_i n e_j|        (the product A A^T, Section 4.1)
 *   I^V_ij = |E(v_i) n E(v_j)|  (the product A^T A, Section 4.1)
 *
 * up to date under deletions, as Algorithm 6 does, and reads the rules off
 * them:
 *   DP: e_i supersedes e_j  <=>  f(e_i) - (I^E_ii - I^E_ij) >= f(e_j)
 *   MD: v_i dominates v_j   <=>  I^V_ij = I^V_jj
 *
 * The matrices are stored sparsely: row i holds, sorted by column, every
 * column that shares at least one vertex (hyperedge) with i in the input;
 * all other entries are zero and stay zero.
 *
 * Algorithm 6 builds both matrices, marks everything alive and every index
 * as a candidate, then alternates Algorithm 4 (DP restricted to candidate
 * superseders P^E) and Algorithm 5 (MD restricted to candidate victims P^V)
 * while something is deleted.  Algorithm 4 decides against the matrices as
 * they were when it started and applies all its deletions afterwards, so a
 * hyperedge deleted in the same pass still supersedes; the same holds for
 * Algorithm 5.  Each loop iteration therefore deletes exactly what one round
 * of Algorithm 3 deletes, and the per-iteration deletion sets are compared
 * with those of the round-synchronous oracle.
 *
 * Reading taken (isolated vertices): Algorithm 5 starts the countdown at the
 * largest demand over E(v_j) and deletes v_j when it reaches zero, which a
 * vertex in no alive hyperedge (countdown 0 at the start) would never do.
 * Algorithm 2 deletes such a vertex (the conjunction over an empty set is
 * true), and so does this implementation: a countdown that starts at zero
 * deletes the vertex at once.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* A sparse symmetric count matrix over `rows` indices. */
typedef struct {
    int64_t *ptr;  /* rows + 1 */
    int32_t *col;  /* sorted per row */
    int32_t *val;
} kc_counts;

static void kc_free(kc_counts *M)
{
    free(M->ptr);
    free(M->col);
    free(M->val);
    memset(M, 0, sizeof(*M));
}

static int kc_cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Builds M_ij = |{k : i in L_k and j in L_k}| for the lists L_k given in
 * CSR form (lptr, lidx, nl lists) over `rows` indices, with the transposed
 * lists (tptr, tidx) giving for each index i the lists containing it.
 * Row i collects the members of every list through i, then counts repeats. */
static int kc_build(int32_t rows, const int64_t *tptr, const int32_t *tidx,
                    const int64_t *lptr, const int32_t *lidx, kc_counts *M)
{
    memset(M, 0, sizeof(*M));
    M->ptr = (int64_t *)calloc((size_t)rows + 1, sizeof(int64_t));
    if (!M->ptr) return -1;
    /* pass 1: sizes of the distinct column sets */
    int64_t scratch_cap = 16;
    int32_t *scratch = (int32_t *)malloc((size_t)scratch_cap * sizeof(int32_t));
    if (!scratch) return -1;
    int64_t total = 0;
    for (int pass = 0; pass < 2; pass++) {
        if (pass == 1) {
            M->col = (int32_t *)malloc((size_t)(total > 0 ? total : 1) * sizeof(int32_t));
            M->val = (int32_t *)malloc((size_t)(total > 0 ? total : 1) * sizeof(int32_t));
            if (!M->col || !M->val) { free(scratch); return -1; }
        }
        total = 0;
        for (int32_t i = 0; i < rows; i++) {
            int64_t len = 0;
            for (int64_t p = tptr[i]; p < tptr[i + 1]; p++) {
                int32_t k = tidx[p];
                len += lptr[k + 1] - lptr[k];
            }
            if (len > scratch_cap) {
                free(scratch);
                scratch_cap = len;
                scratch = (int32_t *)malloc((size_t)scratch_cap * sizeof(int32_t));
                if (!scratch) return -1;
            }
            int64_t w = 0;
            for (int64_t p = tptr[i]; p < tptr[i + 1]; p++) {
                int32_t k = tidx[p];
                for (int64_t q = lptr[k]; q < lptr[k + 1]; q++) scratch[w++] = lidx[q];
            }
            qsort(scratch, (size_t)w, sizeof(int32_t), kc_cmp_i32);
            M->ptr[i] = total;
            for (int64_t a = 0; a < w;) {
                int64_t b = a;
                while (b < w && scratch[b] == scratch[a]) b++;
                if (pass == 1) {
                    M->col[total] = scratch[a];
                    M->val[total] = (int32_t)(b - a);
                }
                total++;
                a = b;
            }
        }
        M->ptr[rows] = total;
    }
    free(scratch);
    return 0;
}

/* Entry (i, j), zero if j never shared anything with i. */
static int32_t *kc_at(const kc_counts *M, int32_t i, int32_t j)
{
    int64_t lo = M->ptr[i], hi = M->ptr[i + 1];
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (M->col[mid] < j) lo = mid + 1;
        else hi = mid;
    }
    return (lo < M->ptr[i + 1] && M->col[lo] == j) ? &M->val[lo] : NULL;
}

static int32_t kc_get(const kc_counts *M, int32_t i, int32_t j)
{
    int32_t *p = kc_at(M, i, j);
    return p ? *p : 0;
}

static void kc_dec(kc_counts *M, int32_t i, int32_t j)
{
    int32_t *p = kc_at(M, i, j);
    if (p) *p -= 1;
}

/* A candidate list with membership flags (each index at most once). */
typedef struct {
    int32_t *idx;
    uint8_t *in;
    int32_t len;
} kc_list;

static void kc_push(kc_list *L, int32_t i)
{
    if (!L->in[i]) {
        L->in[i] = 1;
        L->idx[L->len++] = i;
    }
}

static void kc_clear(kc_list *L)
{
    for (int32_t t = 0; t < L->len; t++) L->in[L->idx[t]] = 0;
    L->len = 0;
}

typedef struct {
    int32_t n, m;
    const int64_t *eptr;  /* hyperedge -> vertices */
    const int32_t *evtx;
    int64_t *vptr;        /* vertex -> hyperedges */
    int32_t *vedg;
    const int32_t *f;
    kc_counts IE, IV;
    uint8_t *RE, *RV;     /* 1 = alive */
    kc_list PE, PV;       /* candidate superseders / candidate victims */
    int32_t *Q;           /* deletions of the current pass */
} kc_state;

/* Algorithm 4: DP with superseders drawn from P^E.  Returns the number of
 * hyperedges deleted; marks them with `round` in death_e. */
static int32_t kc_alg4(kc_state *S, int32_t round, int32_t *death_e)
{
    int32_t q = 0;
    for (int32_t j = 0; j < S->m; j++) {
        if (!S->RE[j]) continue;
        for (int32_t t = 0; t < S->PE.len; t++) {
            int32_t i = S->PE.idx[t];
            if (i == j || !S->RE[i]) continue;
            int32_t xij = kc_get(&S->IE, i, j);
            int Dij = S->f[i] - (kc_get(&S->IE, i, i) - xij) >= S->f[j];
            int Dji = S->f[j] - (kc_get(&S->IE, j, j) - xij) >= S->f[i];
            if (Dij && (!Dji || i < j)) {
                S->Q[q++] = j;
                break;
            }
        }
    }
    for (int32_t t = 0; t < q; t++) {
        int32_t j = S->Q[t];
        S->RE[j] = 0;
        death_e[j] = round;
        /* e_j leaves E(v_i) n E(v_k) for every pair of its alive vertices */
        for (int64_t a = S->eptr[j]; a < S->eptr[j + 1]; a++) {
            int32_t vi = S->evtx[a];
            if (!S->RV[vi]) continue;
            for (int64_t b = S->eptr[j]; b < S->eptr[j + 1]; b++) {
                int32_t vk = S->evtx[b];
                if (S->RV[vk]) kc_dec(&S->IV, vi, vk);
            }
            kc_push(&S->PV, vi);
        }
    }
    kc_clear(&S->PE);
    return q;
}

/* Algorithm 5: MD for the candidate victims in P^V.  Returns the number of
 * vertices deleted; marks them with `round` in death_v. */
static int32_t kc_alg5(kc_state *S, int32_t round, int32_t *death_v)
{
    int32_t q = 0;
    for (int32_t t = 0; t < S->PV.len; t++) {
        int32_t j = S->PV.idx[t];
        if (!S->RV[j]) continue;
        int32_t c = 0;
        for (int64_t p = S->vptr[j]; p < S->vptr[j + 1]; p++) {
            int32_t e = S->vedg[p];
            if (S->RE[e] && S->f[e] > c) c = S->f[e];
        }
        if (c == 0) {  /* no alive hyperedge: deleted, as in Algorithm 2 */
            S->Q[q++] = j;
            continue;
        }
        int32_t djj = kc_get(&S->IV, j, j);
        for (int32_t i = 0; i < S->n; i++) {
            if (i == j || !S->RV[i]) continue;
            int32_t yij = kc_get(&S->IV, i, j);
            if (yij == djj && (yij != kc_get(&S->IV, i, i) || i < j)) {
                if (--c == 0) {
                    S->Q[q++] = j;
                    break;
                }
            }
        }
    }
    for (int32_t t = 0; t < q; t++) {
        int32_t j = S->Q[t];
        S->RV[j] = 0;
        death_v[j] = round;
        /* v_j leaves e_i n e_k for every pair of its alive hyperedges */
        for (int64_t a = S->vptr[j]; a < S->vptr[j + 1]; a++) {
            int32_t ei = S->vedg[a];
            if (!S->RE[ei]) continue;
            for (int64_t b = S->vptr[j]; b < S->vptr[j + 1]; b++) {
                int32_t ek = S->vedg[b];
                if (S->RE[ek]) kc_dec(&S->IE, ei, ek);
            }
            kc_push(&S->PE, ei);
        }
    }
    kc_clear(&S->PV);
    return q;
}

/* Algorithm 6 on a valid instance (the caller validates).  death_e[m] and
 * death_v[n] receive the 1-based iteration of deletion (0 = kept), *rounds
 * the number of iterations that deleted something.  Returns 0, or -1 when
 * memory runs out. */
int mhs_kernelcpu_run(int32_t n, int32_t m, const int64_t *edge_ptr, const int32_t *edge_vtx,
                      const int32_t *demand, int32_t *death_e, int32_t *death_v, int32_t *rounds)
{
    kc_state S;
    memset(&S, 0, sizeof(S));
    S.n = n;
    S.m = m;
    S.eptr = edge_ptr;
    S.evtx = edge_vtx;
    S.f = demand;
    int rc = -1;
    int64_t nnz = m > 0 ? edge_ptr[m] : 0;
    S.vptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    S.vedg = (int32_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
    S.RE = (uint8_t *)malloc((size_t)(m > 0 ? m : 1));
    S.RV = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
    S.PE.idx = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    S.PE.in = (uint8_t *)calloc((size_t)(m > 0 ? m : 1), 1);
    S.PV.idx = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    S.PV.in = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    S.Q = (int32_t *)malloc((size_t)((n > m ? n : m) > 0 ? (n > m ? n : m) : 1) * sizeof(int32_t));
    int64_t *fill = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    if (!S.vptr || !S.vedg || !S.RE || !S.RV || !S.PE.idx || !S.PE.in || !S.PV.idx || !S.PV.in || !S.Q || !fill)
        goto out;
    /* E(v) lists, ascending by hyperedge */
    for (int64_t p = 0; p < nnz; p++) S.vptr[edge_vtx[p] + 1]++;
    for (int32_t v = 0; v < n; v++) S.vptr[v + 1] += S.vptr[v];
    memcpy(fill, S.vptr, ((size_t)n + 1) * sizeof(int64_t));
    for (int32_t e = 0; e < m; e++)
        for (int64_t p = edge_ptr[e]; p < edge_ptr[e + 1]; p++) S.vedg[fill[edge_vtx[p]]++] = e;
    /* I^E from the E(v) lists, I^V from the hyperedges */
    if (kc_build(m, edge_ptr, edge_vtx, S.vptr, S.vedg, &S.IE)) goto out;
    if (kc_build(n, S.vptr, S.vedg, edge_ptr, edge_vtx, &S.IV)) goto out;
    memset(S.RE, 1, (size_t)(m > 0 ? m : 1));
    memset(S.RV, 1, (size_t)(n > 0 ? n : 1));
    for (int32_t e = 0; e < m; e++) { kc_push(&S.PE, e); death_e[e] = 0; }
    for (int32_t v = 0; v < n; v++) { kc_push(&S.PV, v); death_v[v] = 0; }
    int32_t it = 0;
    for (;;) {
        int32_t r = it + 1;
        int32_t de = kc_alg4(&S, r, death_e);
        int32_t dv = kc_alg5(&S, r, death_v);
        if (de == 0 && dv == 0) break;
        it = r;
    }
    *rounds = it;
    rc = 0;
out:
    free(fill);
    kc_free(&S.IE);
    kc_free(&S.IV);
    free(S.vptr);
    free(S.vedg);
    free(S.RE);
    free(S.RV);
    free(S.PE.idx);
    free(S.PE.in);
    free(S.PV.idx);
    free(S.PV.in);
    free(S.Q);
    return rc;
}
