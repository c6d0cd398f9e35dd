/*
 * mhs_oracle.c -- CPU oracle for the round-synchronous DP + MD reduction of
 * Multiple Hitting Set (van Bevern, Kirilin, Skachkov, Smirnov, Tsidulko,
 * "Serial and parallel kernelization of Multiple Hitting Set parameterized by
 * the Dilworth number, implemented on the GPU", arXiv 2109.06042).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load or call this library.  The HIP
 * product library shares no code, header, table or helper with it and never
 * calls it.
 *
 * Plain, single threaded, written from the set definitions rather than from
 * matrix products:
 *
 *   supersedes(i, j)  <=>  f(e_i) - |e_i \ e_j| >= f(e_j)
 *                          (Section 3.1, definition of supersedence)
 *   dominates(i, j)   <=>  E(v_j) is a subset of E(v_i), i != j
 *                          (Section 3.1, definition of Dom)
 *
 * One DP pass follows Algorithm 1 (Section 4.1): every ordered pair (i, j)
 * of distinct alive hyperedges is tested against the hypergraph as it was when
 * the pass started; e_j is deleted if some e_i supersedes it and e_j does not
 * supersede e_i back or i < j (the lower index survives among mutually
 * superseding hyperedges).  Hyperedges deleted in the same pass still count
 * as superseders, because Algorithm 1 never consults R_i.
 *
 * One MD pass follows Algorithm 2 (Section 4.1): D_ij = 1 iff v_i dominates
 * v_j and (v_j does not dominate v_i or i < j); C_j counts the i with
 * D_ij = 1; v_j is deleted iff C_j >= f(e) for every alive e containing v_j.
 * A vertex in no alive hyperedge is deleted (the conjunction over an empty set
 * is true).  Vertices deleted in the same pass still count in C_j.
 *
 * The driver follows Algorithm 3 (Section 4.1): DP pass, then MD pass on the
 * result, repeated while the hypergraph changes.  `rounds` counts the
 * iterations that deleted something; the final iteration that changes nothing
 * is not counted.  For every hyperedge and vertex the driver records the
 * round (1-based) in which it was deleted, 0 if it survives; this is the
 * per-round deletion trace.
 *
 * Two candidate modes give the same answer:
 *   MHS_ORACLE_ALLPAIRS -- every ordered pair, as written in Algorithms 1/2.
 *   MHS_ORACLE_PRUNED   -- DP tests only hyperedges i that share an alive
 *     vertex with e_j: if they share none then |e_i \ e_j| = |e_i| >= f(e_i)
 *     (every alive hyperedge keeps at least f(e) alive vertices, the
 *     invariant behind Lemma 4.3(i)), so f(e_i) - |e_i \ e_j| <= 0 < f(e_j).
 *     MD tests only vertices of one hyperedge of E(v_j): a dominator lies in
 *     every hyperedge of E(v_j).
 * With the superedge rule SE in place of DP (e_i a subset of e_j and
 * f(e_i) >= f(e_j), Section 3.1) the same candidates suffice: a subset of e_j
 * with at least one alive vertex shares that vertex with e_j.
 * Equality of the two modes is checked by the tests on small instances.
 *
 * KernelGPU-FE (Section 5.1, implementation details) alternates the DP + MD
 * reduction with the full-edge rule FE (Section 3.1) until neither applies.
 * mhs_oracle_run_fe takes it round by round: every iteration runs one DP and
 * one MD pass; an iteration in which both delete nothing (a DP + MD
 * fixpoint) runs one FE pass instead, which is exhaustive by itself (see
 * mhs_oracle_fe_pass); the reduction stops at the first iteration in which
 * nothing is deleted at all.  FE changes demands, so the passes read a
 * working copy of them.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MHS_ORACLE_ALLPAIRS 0
#define MHS_ORACLE_PRUNED 1

/* ------------------------------------------------------------------ input */

/* Returns 0 if the CSR is a valid instance, a negative code otherwise:
 *  -1 bad sizes / edge_ptr, -2 vertex out of range, -3 hyperedge not strictly
 *  increasing, -4 empty hyperedge, -5 demand outside [1, |e|]. */
int mhs_oracle_validate(int32_t n, int32_t m, const int64_t *edge_ptr,
                        const int32_t *edge_vtx, const int32_t *demand)
{
    if (n < 0 || m < 0) return -1;
    if (m > 0 && (!edge_ptr || edge_ptr[0] != 0)) return -1;
    for (int32_t e = 0; e < m; e++) {
        int64_t a = edge_ptr[e], b = edge_ptr[e + 1];
        if (b < a) return -1;
        if (b == a) return -4;
        for (int64_t p = a; p < b; p++) {
            if (edge_vtx[p] < 0 || edge_vtx[p] >= n) return -2;
            if (p > a && edge_vtx[p] <= edge_vtx[p - 1]) return -3;
        }
        if (demand[e] < 1 || (int64_t)demand[e] > b - a) return -5;
    }
    return 0;
}

/* ----------------------------------------------------- alive-set adjacency */

/* cur(e): the alive vertices of alive hyperedge e, ascending.
 * inc(v): the alive hyperedges containing alive vertex v, ascending. */
typedef struct {
    int64_t *cptr; int32_t *cvtx;   /* cur lists, indexed by hyperedge */
    int64_t *iptr; int32_t *iedg;   /* inc lists, indexed by vertex */
} adjacency;

static int build_adjacency(int32_t n, int32_t m, const int64_t *edge_ptr,
                           const int32_t *edge_vtx, const uint8_t *alive_v,
                           const uint8_t *alive_e, adjacency *A)
{
    int64_t nnz = m > 0 ? edge_ptr[m] : 0;
    A->cptr = (int64_t *)calloc((size_t)m + 1, sizeof(int64_t));
    A->cvtx = (int32_t *)malloc(((size_t)nnz + 1) * sizeof(int32_t));
    A->iptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    A->iedg = (int32_t *)malloc(((size_t)nnz + 1) * sizeof(int32_t));
    if (!A->cptr || !A->cvtx || !A->iptr || !A->iedg) return -1;
    int64_t q = 0;
    for (int32_t e = 0; e < m; e++) {
        A->cptr[e] = q;
        if (alive_e[e])
            for (int64_t p = edge_ptr[e]; p < edge_ptr[e + 1]; p++)
                if (alive_v[edge_vtx[p]]) {
                    A->cvtx[q++] = edge_vtx[p];
                    A->iptr[edge_vtx[p] + 1]++;
                }
    }
    A->cptr[m] = q;
    for (int32_t v = 0; v < n; v++) A->iptr[v + 1] += A->iptr[v];
    int64_t *fill = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    if (!fill) return -1;
    memcpy(fill, A->iptr, ((size_t)n + 1) * sizeof(int64_t));
    for (int32_t e = 0; e < m; e++)          /* ascending e: inc lists sorted */
        for (int64_t p = A->cptr[e]; p < A->cptr[e + 1]; p++)
            A->iedg[fill[A->cvtx[p]]++] = e;
    free(fill);
    return 0;
}

static void free_adjacency(adjacency *A)
{
    free(A->cptr); free(A->cvtx); free(A->iptr); free(A->iedg);
}

/* |a \ b| for ascending lists a and b, by a merge walk. */
static int64_t set_minus_size(const int32_t *a, int64_t na, const int32_t *b, int64_t nb)
{
    int64_t ia = 0, ib = 0, out = 0;
    while (ia < na) {
        if (ib >= nb || a[ia] < b[ib]) { out++; ia++; }
        else if (a[ia] == b[ib]) { ia++; ib++; }
        else ib++;
    }
    return out;
}

/* Is ascending list a a subset of ascending list b? */
static int is_subset(const int32_t *a, int64_t na, const int32_t *b, int64_t nb)
{
    if (na > nb) return 0;
    return set_minus_size(a, na, b, nb) == 0;
}

/* Edge rules.  MHS_RULE_DP: e_i supersedes e_j on the current hypergraph,
 * f(e_i) - |e_i \ e_j| >= f(e_j) (definition of supersedence, Section 3.1).
 * MHS_RULE_SE: e_i is a subset of e_j and f(e_i) >= f(e_j) (superedge rule,
 * Section 3.1). */
#define MHS_RULE_DP 0
#define MHS_RULE_SE 1
static int g_edge_rule = MHS_RULE_DP;

static int supersedes(const adjacency *A, const int32_t *demand, int32_t i, int32_t j)
{
    int64_t d = set_minus_size(A->cvtx + A->cptr[i], A->cptr[i + 1] - A->cptr[i],
                               A->cvtx + A->cptr[j], A->cptr[j + 1] - A->cptr[j]);
    if (g_edge_rule == MHS_RULE_SE) return d == 0 && demand[i] >= demand[j];
    return (int64_t)demand[i] - d >= (int64_t)demand[j];
}

/* v_i dominates v_j on the current hypergraph: E(v_j) subset of E(v_i). */
static int dominates(const adjacency *A, int32_t i, int32_t j)
{
    return is_subset(A->iedg + A->iptr[j], A->iptr[j + 1] - A->iptr[j],
                     A->iedg + A->iptr[i], A->iptr[i + 1] - A->iptr[i]);
}

/* ------------------------------------------------------------- one DP pass */

/* Algorithm 1: writes kill_e[j] = 1 for each alive hyperedge deleted by one
 * exhaustive DP pass; returns the number deleted, or -1 on allocation failure. */
int64_t mhs_oracle_dp_pass(int32_t n, int32_t m, const int64_t *edge_ptr,
                           const int32_t *edge_vtx, const int32_t *demand,
                           const uint8_t *alive_v, const uint8_t *alive_e,
                           uint8_t *kill_e, int mode)
{
    adjacency A;
    if (build_adjacency(n, m, edge_ptr, edge_vtx, alive_v, alive_e, &A)) return -1;
    int64_t killed = 0;
    int32_t *stamp = NULL;
    if (mode == MHS_ORACLE_PRUNED) {
        stamp = (int32_t *)malloc(((size_t)m + 1) * sizeof(int32_t));
        for (int32_t e = 0; e < m; e++) stamp[e] = -1;
    }
    for (int32_t j = 0; j < m; j++) {
        kill_e[j] = 0;
        if (!alive_e[j]) continue;
        if (mode == MHS_ORACLE_ALLPAIRS) {
            for (int32_t i = 0; i < m && !kill_e[j]; i++) {
                if (i == j || !alive_e[i]) continue;
                if (supersedes(&A, demand, i, j) && (!supersedes(&A, demand, j, i) || i < j))
                    kill_e[j] = 1;
            }
        } else {
            for (int64_t p = A.cptr[j]; p < A.cptr[j + 1] && !kill_e[j]; p++) {
                int32_t v = A.cvtx[p];
                for (int64_t q = A.iptr[v]; q < A.iptr[v + 1]; q++) {
                    int32_t i = A.iedg[q];
                    if (i == j || stamp[i] == j) continue;
                    stamp[i] = j;
                    if (supersedes(&A, demand, i, j) && (!supersedes(&A, demand, j, i) || i < j)) {
                        kill_e[j] = 1;
                        break;
                    }
                }
            }
        }
        killed += kill_e[j];
    }
    free(stamp);
    free_adjacency(&A);
    return killed;
}

/* ------------------------------------------------------------- one MD pass */

/* Algorithm 2: writes kill_v[j] = 1 for each alive vertex deleted by one
 * exhaustive MD pass; returns the number deleted, or -1 on allocation failure. */
int64_t mhs_oracle_md_pass(int32_t n, int32_t m, const int64_t *edge_ptr,
                           const int32_t *edge_vtx, const int32_t *demand,
                           const uint8_t *alive_v, const uint8_t *alive_e,
                           uint8_t *kill_v, int mode)
{
    adjacency A;
    if (build_adjacency(n, m, edge_ptr, edge_vtx, alive_v, alive_e, &A)) return -1;
    int64_t killed = 0;
    for (int32_t j = 0; j < n; j++) {
        kill_v[j] = 0;
        if (!alive_v[j]) continue;
        int64_t dj = A.iptr[j + 1] - A.iptr[j];
        int32_t maxf = 0;                       /* max over the empty set: 0 */
        for (int64_t q = A.iptr[j]; q < A.iptr[j + 1]; q++)
            if (demand[A.iedg[q]] > maxf) maxf = demand[A.iedg[q]];
        int64_t c = 0;
        if (c >= maxf) {                        /* isolated vertex */
            kill_v[j] = 1;
        } else if (mode == MHS_ORACLE_ALLPAIRS) {
            for (int32_t i = 0; i < n && c < maxf; i++) {
                if (i == j || !alive_v[i]) continue;
                if (dominates(&A, i, j) && (!dominates(&A, j, i) || i < j)) c++;
            }
            kill_v[j] = c >= maxf;
        } else {
            int32_t estar = A.iedg[A.iptr[j]];  /* any hyperedge of E(v_j) */
            (void)dj;
            for (int64_t p = A.cptr[estar]; p < A.cptr[estar + 1] && c < maxf; p++) {
                int32_t i = A.cvtx[p];
                if (i == j) continue;
                if (dominates(&A, i, j) && (!dominates(&A, j, i) || i < j)) c++;
            }
            kill_v[j] = c >= maxf;
        }
        killed += kill_v[j];
    }
    free_adjacency(&A);
    return killed;
}

/* ------------------------------------------------------------ Algorithm 3 */

/* ------------------------------------------------------------- one FE pass */

/* FE (Section 3.1): a hyperedge e with |e| = f(e) forces all its vertices into
 * every solution: they are deleted, k drops by their number, and every
 * hyperedge loses one unit of demand per forced vertex it contains, being
 * deleted when its demand reaches 0.  Forcing a vertex removes it from every
 * hyperedge together with one unit of demand, so |e| - f(e) never changes and
 * one pass over the hyperedges that are full at its start is exhaustive: F
 * is the union of their alive vertices.
 * In/out: demand (current demands; deleted hyperedges keep what is left).
 * Out: forced_v[v] = 1 for v in F, kill_e[e] = 1 for deleted hyperedges.
 * Returns |F| + number of deleted hyperedges, or -1 on allocation failure. */
int64_t mhs_oracle_fe_pass(int32_t n, int32_t m, const int64_t *edge_ptr,
                           const int32_t *edge_vtx, int32_t *demand,
                           const uint8_t *alive_v, const uint8_t *alive_e,
                           uint8_t *forced_v, uint8_t *kill_e)
{
    adjacency A;
    if (build_adjacency(n, m, edge_ptr, edge_vtx, alive_v, alive_e, &A)) return -1;
    int64_t changed = 0;
    for (int32_t v = 0; v < n; v++) forced_v[v] = 0;
    for (int32_t e = 0; e < m; e++) {
        kill_e[e] = 0;
        if (alive_e[e] && A.cptr[e + 1] - A.cptr[e] == (int64_t)demand[e])
            for (int64_t p = A.cptr[e]; p < A.cptr[e + 1]; p++) forced_v[A.cvtx[p]] = 1;
    }
    for (int32_t v = 0; v < n; v++) changed += forced_v[v];
    if (changed) {
        for (int32_t e = 0; e < m; e++) {
            if (!alive_e[e]) continue;
            int64_t t = 0;
            for (int64_t p = A.cptr[e]; p < A.cptr[e + 1]; p++) t += forced_v[A.cvtx[p]];
            demand[e] -= (int32_t)t;
            if (demand[e] <= 0) { kill_e[e] = 1; changed++; }
        }
    }
    free_adjacency(&A);
    return changed;
}

/* Selects the edge rule of the passes and runs below: MHS_RULE_DP (default)
 * or MHS_RULE_SE.  Returns the previous rule.  Not thread safe. */
int mhs_oracle_set_edge_rule(int rule)
{
    int old = g_edge_rule;
    g_edge_rule = rule == MHS_RULE_SE ? MHS_RULE_SE : MHS_RULE_DP;
    return old;
}

/* Runs DP then MD until nothing changes (or max_rounds productive rounds).
 * death_e[m], death_v[n]: round of deletion (1-based), 0 for survivors.
 * *rounds: number of productive rounds.  Returns 0, or the negative
 * validation code, or -100 on allocation failure. */
int mhs_oracle_run(int32_t n, int32_t m, const int64_t *edge_ptr,
                   const int32_t *edge_vtx, const int32_t *demand, int mode,
                   int32_t max_rounds, int32_t *death_e, int32_t *death_v,
                   int32_t *rounds)
{
    int rc = mhs_oracle_validate(n, m, edge_ptr, edge_vtx, demand);
    if (rc) return rc;
    uint8_t *alive_v = (uint8_t *)malloc((size_t)n + 1);
    uint8_t *alive_e = (uint8_t *)malloc((size_t)m + 1);
    uint8_t *kill_v = (uint8_t *)malloc((size_t)n + 1);
    uint8_t *kill_e = (uint8_t *)malloc((size_t)m + 1);
    if (!alive_v || !alive_e || !kill_v || !kill_e) return -100;
    memset(alive_v, 1, (size_t)n);
    memset(alive_e, 1, (size_t)m);
    for (int32_t e = 0; e < m; e++) death_e[e] = 0;
    for (int32_t v = 0; v < n; v++) death_v[v] = 0;
    int32_t r = 0;
    while (max_rounds < 0 || r < max_rounds) {
        int64_t ke = mhs_oracle_dp_pass(n, m, edge_ptr, edge_vtx, demand,
                                        alive_v, alive_e, kill_e, mode);
        if (ke < 0) return -100;
        for (int32_t e = 0; e < m; e++)
            if (kill_e[e]) { alive_e[e] = 0; death_e[e] = r + 1; }
        int64_t kv = mhs_oracle_md_pass(n, m, edge_ptr, edge_vtx, demand,
                                        alive_v, alive_e, kill_v, mode);
        if (kv < 0) return -100;
        for (int32_t v = 0; v < n; v++)
            if (kill_v[v]) { alive_v[v] = 0; death_v[v] = r + 1; }
        if (ke == 0 && kv == 0) break;
        r++;
    }
    *rounds = r;
    free(alive_v); free(alive_e); free(kill_v); free(kill_e);
    return 0;
}

/* KernelGPU-FE: DP + MD rounds, with an FE pass in every iteration that
 * deletes nothing by DP and MD, until an iteration deletes nothing at all.
 * As mhs_oracle_run, plus forced_v[n] (1 for vertices forced into the
 * solution by FE; their death round is the FE iteration), demand_out[m]
 * (demands at the end), *n_forced.  Returns 0 or a negative code. */
int mhs_oracle_run_fe(int32_t n, int32_t m, const int64_t *edge_ptr,
                      const int32_t *edge_vtx, const int32_t *demand, int mode,
                      int32_t max_rounds, int32_t *death_e, int32_t *death_v,
                      uint8_t *forced_v, int32_t *demand_out, int32_t *rounds,
                      int64_t *n_forced)
{
    int rc = mhs_oracle_validate(n, m, edge_ptr, edge_vtx, demand);
    if (rc) return rc;
    uint8_t *alive_v = (uint8_t *)malloc((size_t)n + 1);
    uint8_t *alive_e = (uint8_t *)malloc((size_t)m + 1);
    uint8_t *kill_v = (uint8_t *)malloc((size_t)n + 1);
    uint8_t *kill_e = (uint8_t *)malloc((size_t)m + 1);
    uint8_t *fv = (uint8_t *)malloc((size_t)n + 1);
    if (!alive_v || !alive_e || !kill_v || !kill_e || !fv) return -100;
    memset(alive_v, 1, (size_t)n);
    memset(alive_e, 1, (size_t)m);
    for (int32_t e = 0; e < m; e++) { death_e[e] = 0; demand_out[e] = demand[e]; }
    for (int32_t v = 0; v < n; v++) { death_v[v] = 0; forced_v[v] = 0; }
    int32_t r = 0;
    int64_t nf = 0;
    while (max_rounds < 0 || r < max_rounds) {
        int64_t ke = mhs_oracle_dp_pass(n, m, edge_ptr, edge_vtx, demand_out,
                                        alive_v, alive_e, kill_e, mode);
        if (ke < 0) return -100;
        for (int32_t e = 0; e < m; e++)
            if (kill_e[e]) { alive_e[e] = 0; death_e[e] = r + 1; }
        int64_t kv = mhs_oracle_md_pass(n, m, edge_ptr, edge_vtx, demand_out,
                                        alive_v, alive_e, kill_v, mode);
        if (kv < 0) return -100;
        for (int32_t v = 0; v < n; v++)
            if (kill_v[v]) { alive_v[v] = 0; death_v[v] = r + 1; }
        if (ke == 0 && kv == 0) {
            int64_t c = mhs_oracle_fe_pass(n, m, edge_ptr, edge_vtx, demand_out,
                                           alive_v, alive_e, fv, kill_e);
            if (c < 0) return -100;
            if (c == 0) break;
            for (int32_t v = 0; v < n; v++)
                if (fv[v]) { alive_v[v] = 0; death_v[v] = r + 1; forced_v[v] = 1; nf++; }
            for (int32_t e = 0; e < m; e++)
                if (kill_e[e]) { alive_e[e] = 0; death_e[e] = r + 1; }
        }
        r++;
    }
    *rounds = r;
    *n_forced = nf;
    free(alive_v); free(alive_e); free(kill_v); free(kill_e); free(fv);
    return 0;
}
