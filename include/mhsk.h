/*
 * mhsk.h -- C ABI of the MI355X Multiple Hitting Set kernelization library.
 *
 * The library reduces Multiple Hitting Set instances (problem definition,
 * Section 1: hypergraph H = (V, E), demands f: E -> {1..alpha}, budget k) by
 * exhaustive, round-synchronous application of the demand-pushing rule DP
 * (Section 3.1, generalising Weihe's hyperedge rule W2) and the
 * multiple-domination rule MD (Section 3.1, generalising Weihe's vertex rule
 * W1), in the order of Algorithm 3 (Section 4.1): each round runs one DP pass
 * (Algorithm 1) and then one MD pass (Algorithm 2) on its result, until a
 * round deletes nothing.
 *
 *   DP pass: e_j is deleted iff some alive e_i != e_j supersedes it,
 *            f(e_i) - |e_i \ e_j| >= f(e_j), and e_j does not supersede e_i
 *            or i < j (of two mutually superseding hyperedges the lower
 *            original id survives).  All tests read the state at the start of
 *            the pass.
 *   MD pass: v_j is deleted iff the number C_j of alive v_i != v_j with
 *            E(v_j) subset of E(v_i) and (E(v_i) not subset of E(v_j) or
 *            i < j) is at least the largest demand of an alive hyperedge
 *            containing v_j; a vertex in no alive hyperedge is deleted.
 *
 * Both passes are evaluated from the intersection counts of the 0/1
 * incidence matrix A with itself (equations mat-trick1 and mat-trick2,
 * Section 4): |e_i & e_j| = (A A^T)_ij and |E(v_i) & E(v_j)| = (A^T A)_ij.
 * On the GPU these products are int8 MFMA contractions whose epilogue applies
 * the tests; the count matrices are never stored.
 *
 * Conventions shared by every entry point:
 *  - Every function returns an int status (MHS_OK = 0, negative on error) or
 *    is void; nothing throws across the ABI.  mhs_last_error() returns a
 *    thread-local message for the last non-OK status of the calling thread.
 *  - Ids are 0-based original ids.  Hyperedges are given in CSR form.
 *  - Device memory is always the caller's: the caller passes one workspace
 *    of at least the size reported by the matching *_workspace_bytes call.
 *    The library allocates host memory only (results, staging tables).
 *  - `hip_stream` is a hipStream_t (NULL = the default stream).  mhs_run and
 *    mhs_run_batch are synchronous: when they return, all their work on that
 *    stream has finished and the workspace may be reused.
 *  - The library runs on the HIP device that is current on the calling
 *    thread; the workspace must live on that device.
 */
#ifndef MHSK_H
#define MHSK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
enum {
    MHS_OK = 0,
    MHS_EINVAL = -1,   /* malformed instance, bad argument or reserved flag */
    MHS_ENOSPC = -2,   /* workspace / arena smaller than required, or no host
                          memory for a server request's copy */
    MHS_EDEVICE = -3,  /* a HIP runtime call failed */
    MHS_EAGAIN = -4,   /* server: nothing to return yet */
    MHS_EREJECT = -5   /* server: request can never fit the arena */
};

/* ----------------------------------------------------------------- flags */
#define MHS_VARIANT_AUTO   0u        /* contraction kernel chosen by the library */
#define MHS_VARIANT_INT8   1u        /* int8 MFMA (v_mfma_i32_16x16x64_i8) */
#define MHS_VARIANT_BITSET 2u        /* bit-packed operands, AND + popcount on the vector ALU */
#define MHS_VARIANT_SPARSE 3u        /* nonzero product terms only, hash-counted per victim */
#define MHS_VARIANT_HYBRID 4u        /* per instance: int8 MFMA tiles for instances whose hyperedges
                                        span under 5% of the vertex ids (banded tiles), sparse
                                        counts otherwise; device-resident inputs take int8 */
/* Instances with n or m of 2^29 or more take sparse counts whatever the
 * variant (dense tiles encode counts below 2^29). */
#define MHS_VARIANT_MASK   0xffu
#define MHS_TRACE_ROUNDS   (1u << 8)  /* keep the per-round deletion lists: every result
                                         carries them (each element's deletion round,
                                         mhs_result_round / mhs_result_deaths), so the
                                         flag is accepted and changes nothing */
#define MHS_INPUT_DEVICE   (1u << 12) /* instance arrays are device pointers */
#define MHS_NO_GRAPH       (1u << 9)  /* launch every round's kernels directly */
#define MHS_PROFILE        (1u << 10) /* time the contraction kernels with events */
#define MHS_GRAPH          (1u << 11) /* capture a round once into a hipGraph and replay it */
/* Neither MHS_GRAPH nor MHS_NO_GRAPH: direct launches for one instance
 * (mhs_run: a graph boundary costs the device more than the host needs to
 * launch a round's kernels), hipGraph replay for a set (mhs_run_batch,
 * mhs_tune).  Both: MHS_EINVAL. */
/* Persistent contraction grid: 2^k workgroups per compute unit (k = 0..4);
 * 0 (no bits) = library default (4 per CU).  Set by the autotuner. */
#define MHS_GRID_LOG2(k)   ((((uint32_t)(k)) + 1u) << 24)
#define MHS_GRID_MASK      (0xfu << 24)
/* Operand staging of the int8 MFMA contraction: k = 0 tiles staged in LDS
 * through registers, 1 fragments loaded straight from HBM into registers,
 * 2 asynchronous global-to-LDS copies through a 4-stage ring; 0 (no bits) =
 * library default (k = 0).  Results are identical; set by the autotuner. */
#define MHS_GEMM_SCHED(k)  ((((uint32_t)(k)) + 1u) << 20)
#define MHS_GEMM_SCHED_MASK (0x3u << 20)
#define MHS_RULE_SE        (1u << 16) /* edge phase applies the superedge rule SE
                                         (Section 3.1: delete e_j if some e_i is a
                                         subset of it with f(e_i) >= f(e_j); same
                                         tie break) instead of DP: the paper's
                                         SE + MD combination of Theorem 3.4 */
#define MHS_RULE_FE        (1u << 17) /* alternate the reduction with the full-edge
                                         rule FE (Section 3.1; the paper's
                                         KernelGPU-FE, Section 5.1): a round in
                                         which the edge rule and MD delete nothing
                                         runs one FE pass: the alive vertices of
                                         every hyperedge with |e| = f(e) are forced
                                         into the solution and deleted, every
                                         hyperedge loses one unit of demand per
                                         forced vertex and goes at demand 0; the
                                         reduction stops at the first round that
                                         deletes nothing.  k_out = k - forced. */

/* ------------------------------------------------------------- instances */
/*
 * One instance (problem definition, Section 1).
 *   n, m      number of vertices (ids 0..n-1) and hyperedges (0..m-1), >= 0.
 *   edge_ptr  m+1 entries, edge_ptr[0] = 0, nondecreasing; nnz = edge_ptr[m]
 *             (nnz < 2^31).  May be NULL when m = 0.
 *   edge_vtx  nnz vertex ids; within each hyperedge strictly increasing and in
 *             [0, n).  Every hyperedge is nonempty.
 *   demand    m demands, 1 <= demand[e] <= |e|.
 *   k         budget; DP and MD never change it (k_out = k).
 *   nnz       optional: edge_ptr[m] if the caller knows it, else 0.  Only
 *             used for device inputs, where it spares a device-to-host read
 *             before the reduction starts; a wrong value is rejected by the
 *             device-side check (MHS_EINVAL).
 * Arrays are host pointers unless MHS_INPUT_DEVICE is set, in which case they
 * are device pointers on the current device; they stay owned by the caller
 * and are only read.  Identical hyperedges are allowed (distinct ids).
 * Validation failures return MHS_EINVAL (for device inputs the check runs on
 * the device before any reduction).
 */
typedef struct {
    int32_t n, m;
    const int64_t *edge_ptr;
    const int32_t *edge_vtx;
    const int32_t *demand;
    int64_t k;
    int64_t nnz;
} mhs_instance;

/* Summary of one result (Algorithm 3 output). */
typedef struct {
    int32_t n_kept;    /* surviving vertices */
    int32_t m_kept;    /* surviving hyperedges */
    int32_t n_forced;  /* vertices forced into the solution (MHS_RULE_FE; else 0) */
    int32_t rounds;    /* productive rounds: iterations that deleted something */
    int64_t k_out;     /* k - n_forced */
} mhs_summary;

/* Timing and work counters of one run.  The step timings and the dense
 * kernels' work counters (issued_ops, blob_bytes, encode_bytes) are filled
 * when MHS_PROFILE is set (0 otherwise: their atomics stay off the timed
 * path); iterations, gemm_launches, terms and total_ms always. */
typedef struct {
    int32_t iterations;        /* rounds executed, including the final no-change one */
    int32_t gemm_launches;     /* contraction kernel launches */
    double gemm_ms;            /* summed event time of the contraction kernels
                                  (dense tiles and sparse counting) */
    double edge_gemm_ms;       /* ... of which DP (A A^T) phases */
    double vertex_gemm_ms;     /* ... of which MD (A^T A) phases */
    double rows_ms;            /* rows, windows and tile encoding, both phases */
    double compact_ms;         /* deletion decisions and compaction */
    double round_end_ms;       /* fixpoint bookkeeping */
    double issued_ops;         /* int8 MFMA multiply-add ops issued (2 per MAC) */
    double edge_issued_ops;
    double vertex_issued_ops;
    double blob_bytes;         /* bytes of encoded incidence tiles written */
    double encode_bytes;       /* algorithmic HBM bytes of the rows/encode kernels:
                                  37 per row + 8 per scanned entry + blob bytes */
    double terms;              /* nonzero product terms visited (sparse variant) */
    double total_ms;           /* wall time of the call on the host */
    double sparse_ms;          /* summed event time of the sparse counting kernels
                                  (part of gemm_ms; sparse members only) */
    double edge_sparse_ms;     /* ... of which edge phases */
    double vertex_sparse_ms;   /* ... of which vertex phases */
} mhs_stats;

typedef struct mhs_result mhs_result;  /* opaque, library-owned host object */
typedef struct mhs_server mhs_server;  /* opaque */

/* ------------------------------------------------------------ one-shot */
/* Device workspace (bytes) mhs_run needs for an instance of this shape. */
size_t mhs_workspace_bytes(int32_t n, int32_t m, int64_t nnz, uint32_t flags);

/* Reduce one instance to the fixpoint of Algorithm 3.  On MHS_OK, *out holds
 * a new result (free with mhs_result_free); otherwise *out is NULL. */
int mhs_run(const mhs_instance *inst, uint32_t flags, void *d_ws, size_t ws_bytes,
            void *hip_stream, mhs_result **out);

/* --------------------------------------------------------------- batched */
/* Device workspace for reducing `count` instances together (0 for an
 * invalid shape, or for device instances without their nnz). */
size_t mhs_batch_workspace_bytes(const mhs_instance *insts, int32_t count, uint32_t flags);

/* Reduce `count` independent instances together: every round runs one DP
 * phase and one MD phase over all instances that have not reached their
 * fixpoint, each phase as one launch per kernel over the whole set (the
 * contraction a persistent grid over the set's tile pairs); rounds are
 * replayed from hipGraphs.  outs[i] receives instance i's result, identical
 * to what mhs_run returns for it alone.
 * Host instances cross the bus in one compact upload.  With
 * MHS_INPUT_DEVICE every instance's arrays are device pointers read in
 * place (they must stay valid and unchanged until the call returns) and
 * every instance with m > 0 must give its nnz (MHS_EINVAL otherwise); the
 * hybrid rule then takes each instance's span sum from a device pass.
 * Validation failures name the first bad instance ("instance i: ..."). */
int mhs_run_batch(const mhs_instance *insts, int32_t count, uint32_t flags, void *d_ws,
                  size_t ws_bytes, void *hip_stream, mhs_result **outs);

/* mhs_run_batch with the results written straight into caller arrays (no
 * result objects): the arrays are concatenated in instance order as
 * mhs_results_take writes them -- death_e and demand hold every instance's
 * m entries one after the other (sum of m), death_v and forced their n
 * entries (sum of n), sums[i] and stats[i] instance i's summary and stats.
 * Any output may be NULL to skip it; all are host memory the caller owns.
 * Same inputs, flags, workspace and errors as mhs_run_batch. */
int mhs_run_batch_into(const mhs_instance *insts, int32_t count, uint32_t flags, void *d_ws,
                       size_t ws_bytes, void *hip_stream, mhs_summary *sums, mhs_stats *stats,
                       int32_t *death_e, int32_t *death_v, int32_t *demand, uint8_t *forced);

/* -------------------------------------------------------------- autotune */
typedef struct {
    uint32_t best_flags;   /* variant and grid bits of the fastest candidate */
    int32_t candidates;    /* candidates timed */
    double best_ms;        /* its wall time on the sample (best of three batched runs) */
    double default_ms;     /* wall time of the int8 default on the sample (likewise) */
} mhs_tune_report;

/* Schedule autotuner.  Times every candidate (contraction variant: int8
 * MFMA and the per-instance hybrid, each with the three operand stagings of
 * MHS_GEMM_SCHED, and bitset popcount, each with a persistent grid of 1, 2,
 * 4, 8 or 16 workgroups per CU; sparse counting: 36 candidates) on `count`
 * sample instances reduced as one batch (host arrays, or device arrays with
 * MHS_INPUT_DEVICE as for mhs_run_batch, which keeps the host-to-device
 * copies out of the timings; each candidate run once to warm up, then timed
 * as the best of three runs),
 * after checking that every candidate returns identical results; reports the
 * fastest and records it for the sample's size class (log2 of the mean
 * hyperedge count, mean hyperedge size and vertex count).  Later calls with
 * MHS_VARIANT_AUTO on a batch or instance of a recorded class use it; other
 * classes use the hybrid with 4 workgroups per CU.  `d_ws` must
 * hold mhs_batch_workspace_bytes of the sample (with the same flags).
 * Flags: 0, MHS_NO_GRAPH or MHS_GRAPH, MHS_RULE_SE / MHS_RULE_FE, and
 * MHS_INPUT_DEVICE. */
int mhs_tune(const mhs_instance *insts, int32_t count, uint32_t flags, void *d_ws, size_t ws_bytes,
             void *hip_stream, mhs_tune_report *report);
/* Forget every recorded class (AUTO falls back to the default). */
void mhs_tune_reset(void);

/* ------------------------------------------------------- no allocation */
/*
 * For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the one-instance
 * reduction of mhs_run, identical results, with its workspace in a static
 * device array of MHS_STATIC_SCRATCH_BYTES that the library holds on every
 * device it runs on until the process ends.  No device, pinned or mapped
 * memory is allocated, no event or graph is created: rounds are launched one
 * at a time on `hip_stream`, the active count is read after each, and the
 * call is synchronous on that stream.
 *   inst      host arrays, or device arrays with MHS_INPUT_DEVICE (the nnz
 *             hint spares one read of edge_ptr[m]).
 *   flags     as mhs_run, except MHS_PROFILE and MHS_GRAPH (MHS_EINVAL).
 *   summary   receives the result summary.
 *   death_e   host, m entries (may be NULL only when m = 0): deletion round of
 *             every hyperedge, 0 = kept (as mhs_result_deaths).
 *   death_v   host, n entries (may be NULL only when n = 0).
 * An instance whose workspace (mhs_workspace_bytes) exceeds the static
 * array is refused with MHS_ENOSPC before any device work.  Calls on one
 * device share its array, which keeps the last call's contents (the
 * reduction initializes everything it reads): calls from one process are
 * serialized per device by the library; calls that overlap on one GPU from
 * several processes race.
 */
#define MHS_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
int mhs_run_static(const mhs_instance *inst, uint32_t flags, void *hip_stream, mhs_summary *summary,
                   int32_t *death_e, int32_t *death_v);

/* --------------------------------------------------------------- results */
/* MHS_OK for a finished reduction; for a request the server could not
 * reduce, its error code (the message goes to mhs_last_error). */
int mhs_result_status(const mhs_result *r);
int mhs_result_summary(const mhs_result *r, mhs_summary *s);
int mhs_result_stats(const mhs_result *r, mhs_stats *s);
/* Copy surviving ids in ascending order; arrays sized from the summary
 * (any may be NULL to skip it). forced_v receives the n_forced forced ids. */
int mhs_result_copy(const mhs_result *r, int32_t *kept_v, int32_t *kept_e, int32_t *forced_v);
/* Per-element deletion round (1-based), 0 for survivors: death_e[m], death_v[n]. */
int mhs_result_deaths(const mhs_result *r, int32_t *death_e, int32_t *death_v);
/* Demand of every hyperedge at the end, m entries: its original demand
 * less the forced vertices it contained (MHS_RULE_FE); 0 for deleted ones. */
int mhs_result_demands(const mhs_result *r, int32_t *demand);
/* Forced flag of every vertex, n bytes (1 = forced into the solution). */
int mhs_result_forced(const mhs_result *r, uint8_t *forced);
/* Deletions of productive round r (1..rounds), ascending ids.  Two-call use:
 * with NULL arrays only the counts are written. */
int mhs_result_round(const mhs_result *r, int32_t round, int32_t *n_del_e, int32_t *del_e,
                     int32_t *n_del_v, int32_t *del_v);
void mhs_result_free(mhs_result *r);
/* Export `count` results with one call and free them (a batch's results
 * otherwise take a call per array and result).  Arrays are concatenated in
 * result order: death_e and demand hold the results' m entries each, one
 * result after the other (sum of m entries), death_v and forced their n
 * entries (sum of n); sums[i] and stats[i] receive result i's summary and
 * stats.  Any output may be NULL to skip it; the caller owns every output.
 * All rs[i] must be live results: if one is NULL nothing is written or freed
 * (MHS_EINVAL); on MHS_OK every result is freed and rs[i] set to NULL. */
int mhs_results_take(mhs_result **rs, int32_t count, mhs_summary *sums, mhs_stats *stats,
                     int32_t *death_e, int32_t *death_v, int32_t *demand, uint8_t *forced);

/* --------------------------------------------------------------- serving */
/*
 * Continuous batching.  The server owns a caller-provided device arena and a
 * host queue.  mhs_server_submit validates the request, keeps a compact
 * copy of it (32-bit offsets, 16-bit vertex ids when n <= 65536) and queues
 * it; a request whose footprint (mhs_workspace_bytes of the instance, host
 * input, plus its compact copy) exceeds the arena is rejected with
 * MHS_EREJECT.
 *
 * The server advances in steps, each queued on the server's stream by one
 * poll: the requests found finished by the previous step are read back and
 * their arena ranges and slots freed; queued requests are admitted in
 * arrival order while a slot and enough arena space are free (first fit,
 * never overcommitting), uploaded and prepared; one round (edge phase + MD
 * phase) runs over every resident instance in shared launches; the
 * instances' counters are copied back.  At most two steps are in flight.
 *
 * mhs_server_poll never waits for the device: it takes stock of the steps
 * that have completed, queues the next step when fewer than two are in
 * flight, and returns up to `cap` finished requests (ids and results, in the
 * order they finished; the results are the caller's, free each with
 * mhs_result_free).  It returns MHS_OK when it returns at least one result,
 * else MHS_EAGAIN (the message says whether the server is idle: nothing
 * queued, resident or in flight).  A result is identical to mhs_run's for
 * the same instance and flags, whatever else is resident.  A request the
 * device could not reduce (its counters carry an error) comes back as a
 * failed result: mhs_result_status returns its code (MHS_EINVAL,
 * MHS_ENOSPC or MHS_EDEVICE) and message, and every other accessor returns
 * the same code.
 *
 * mhs_server_drain queues steps, waiting for the device, until nothing is
 * queued, resident or in flight; the finished requests stay with the server
 * until a poll returns them.
 *
 * submit may be called from another thread than poll; poll, drain, pending,
 * arena_used and destroy must not run concurrently with each other.
 * destroy waits for the stream and frees the results nobody polled.
 * Flags: a variant (MHS_VARIANT_*, HYBRID included), MHS_GRID_LOG2,
 * MHS_RULE_SE, MHS_RULE_FE, MHS_TRACE_ROUNDS, MHS_GRAPH or MHS_NO_GRAPH
 * (rounds are launched directly either way).
 */
int mhs_server_create(void *d_arena, size_t arena_bytes, int32_t max_slots, uint32_t flags,
                      void *hip_stream, mhs_server **out);
int mhs_server_submit(mhs_server *s, const mhs_instance *inst, uint64_t request_id);
/* Take stock, queue the next step, return finished requests (non-blocking). */
int mhs_server_poll(mhs_server *s, int32_t cap, uint64_t *ids, mhs_result **results,
                    int32_t *n_done);
/* Run every queued and resident request to its fixpoint (blocking). */
int mhs_server_drain(mhs_server *s);
/* Number of queued (not yet admitted) and resident requests. */
int mhs_server_pending(const mhs_server *s, int32_t *queued, int32_t *resident);
/* Bytes of the arena currently reserved by resident requests. */
int mhs_server_arena_used(const mhs_server *s, size_t *used);
void mhs_server_destroy(mhs_server *s);

/* ------------------------------------------------------------------ misc */
const char *mhs_last_error(void);
/* Library version string. */
const char *mhs_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MHSK_H */
