// engine.h -- device-side state and host engine of the DP + MD round loop.
//
// A "set" holds any number of resident instances.  Every per-instance array
// lives in that instance's slice of caller-provided device memory; a
// device-resident table of DInst descriptors points at them.  Each round
// (Algorithm 3, Section 4.1) runs over all instances of the set that have not
// reached their fixpoint:
//
//   edge phase (Algorithm 1, DP):   rows and K windows -> tile offsets ->
//        encode A_E tiles -> fused A_E A_E^T contraction over the tile pairs with
//        the DP test -> stable edge compaction (death rounds, compact ids)
//   vertex phase (Algorithm 2, MD): rows (degrees, largest demands) and K
//        windows -> tile offsets -> encode A_V tiles -> fused A_V A_V^T
//        contraction over the tile pairs counting dominators -> MD test and stable
//        vertex compaction
//   round end: fixpoint detection.
//
// Launch geometries depend only on the set's original sizes, never on the
// alive counts (those live in device memory), so a round can be captured in
// a hipGraph once and replayed.  Workgroups map to (instance, tile) or
// (instance, block) through per-set prefix arrays and a binary search.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>
#include <vector>

namespace mhsk {

constexpr int kTile = 128;                       // rows per contraction tile
constexpr int kChunk = 64;                       // K elements per MFMA step
constexpr int kChunkBytes = kTile * kChunk;      // one tile x one chunk, int8
constexpr int kChunkBytesBits = kTile * 8;       // one tile x one chunk, bits
constexpr int kBlock = 1024;                     // rows per compaction block
constexpr int kCtr = 32;                         // per-instance counter words
constexpr int kFlagSlots = 8;                    // host-mapped round slots (sequence number mod 8)
constexpr int kMaxRoundsPerLaunch = kFlagSlots / 2;
// Members of a set with at most kLocalN vertices are prepared by workgroups
// of kLocalChunk incidences each that count and place in LDS (global
// atomics only per vertex and workgroup); single instances and larger ones
// count with global atomics per incidence.
constexpr int kLocalN = 8192;
constexpr int kLocalChunk = 16384;
// Slack classes of the sparse variant's round-1 list order: a table of
// kSlackClasses list positions per vertex in the blob.
constexpr int kSlackClasses = 16;

// Per-instance device counters (int32 words of DInst::ctr; 64-bit counters
// occupy two words starting at an even index).  Per-phase counters have an
// edge (E) and a vertex (V) copy; the round end resets them for the next
// iteration, so every phase kernel can rely on them being zero at its start.
enum Ctr : int {
  C_MA = 0,          // alive hyperedges
  C_NA = 1,          // alive vertices
  C_ROUND = 2,       // current iteration (1-based; the last one once done)
  C_DONE = 3,        // fixpoint reached
  C_KILLED_E = 4,    // hyperedges deleted in the current iteration
  C_KILLED_V = 5,    // vertices deleted in the current iteration
  C_ROUNDS = 6,      // productive rounds so far
  C_ERR = 7,         // validation / capacity error code (0 = ok)
  C_SPARE_8 = 8,     // unused (4 words)
  C_SPARE_12 = 12,   // unused (2 words)
  C_BLOB_SUM = 14,   // int64: blob bytes written, all phases
  C_CHUNKS_SUM_E = 16,  // int64: K chunks over all edge-phase items
  C_CHUNKS_SUM_V = 18,  // int64: K chunks over all vertex-phase items
  C_WIDE_E = 20,     // the edge phase's tile 0 window spans a quarter of K or more
  C_WIDE_V = 21,     // ... the vertex phase's (tile pairs are then taken row by row)
  C_PAIRS_SUM = 22,  // int64: nonzero product terms visited (sparse variant)
  C_ROWS_SUM = 24,   // int64: rows encoded by k_rows_encode, all phases
  C_ENTRIES_SUM = 26,  // int64: CSR / CSC entries those rows scanned
  C_NCOMP_E = 28,    // edge compactions so far (its parity selects the current erow list)
  C_NCOMP_V = 29,    // vertex compactions so far (parity selects the current vrow list)
  C_FE_FIRED = 30,   // the FE pass of the current round forced something
  C_NFORCED = 31,    // vertices forced into the solution by FE so far
};

// Global (set-wide) device counters.
enum GCtr : int {
  G_ANY = 3,       // instances still active after the last round end (words 0..2 unused)
  G_RSEQ = 4,      // round ends since the last prepare (selects the host flag slot)
  G_TICKET = 5,    // 5..8: block tickets of the round's four compaction launches
                   // (edge, vertex, FE edge, FE vertex)
  G_N = 16
};

// Error codes in C_ERR (validation codes match the host validator).
enum ErrCode : int {
  E_PTR = 1, E_RANGE = 2, E_ORDER = 3, E_EMPTY = 4, E_DEMAND = 5, E_CAPACITY = 100, E_STALL = 101
};

struct DInst {
  int32_t n, m;
  int64_t nnz;
  const int64_t* eptr;   // m+1, input CSR (read in place)
  const int32_t* evtx;   // nnz
  const int32_t* dem;    // m
  int32_t* vptr;         // n+1, CSC built on the device
  int32_t* vedg;         // nnz
  int32_t* vend;         // n: CSC fill cursors while preparing; then the end of
                         // v's alive-first list: [vptr[v], vend[v]) holds every
                         // alive hyperedge of v (the rest of the list is dead)
  int32_t* death_e;      // m: round of deletion, 0 = alive
  int32_t* death_v;      // n
  int32_t* erow[2];      // m each: alive hyperedges in slot order (parity buffers)
  int32_t* vrow[2];      // n each: alive vertices in id order
  int32_t* ecol;         // m: original hyperedge -> compact index, -1 if deleted
  int32_t* vcol;         // n: original vertex -> compact index, -1 if deleted
  int32_t* rs;           // R: |e| (edge phase) or |E(v)| (vertex phase), per compact row
  int32_t* rf;           // R: f(e) or the largest demand over E(v)
  int32_t* rid;          // R: original id
  int32_t* cnt;          // n: dominator counts C_j
  uint8_t* kill;         // R: deletion flag per compact row
  int32_t* esz;          // m: alive size of each alive hyperedge (sparse variant)
  int32_t* vdeg;         // n: alive degree of each alive vertex (sparse variant)
  uint8_t* eslk;         // m: |e| - f(e) of each alive hyperedge, capped at 254; 255 once
                         // deleted (sparse variant: partner filter of the edge phase)
  int32_t* tkl;          // T: first K chunk of a tile's window
  int32_t* tkh;          // T: one past its last K chunk
  int64_t* toff;         // T: byte offset of the tile in blob
  uint64_t* bstat;       // B: per compaction block status word (epoch | kind | count)
  int8_t* blob;          // encoded incidence tiles
  int64_t blob_cap;
  int32_t* ctr;          // kCtr counters
  int32_t* fw;           // m: working demands (FE lowers them; equal to dem otherwise)
  uint8_t* forced;       // n: forced into the solution by FE
  int32_t variant;       // 1 int8 MFMA, 2 bitset popcount (dense tiles), 3 sparse counts
  int32_t rule_se;       // edge phase applies the superedge rule SE instead of DP
  int32_t rule_fe;       // FE pass in every round that DP and MD leave unchanged
  int32_t prep_lds;      // prepared by workgroups counting in LDS (k_prep_lcount / k_prep_lfill)
};

// Per-instance slice layout (byte offsets from the slice start).
struct InstLayout {
  size_t bytes = 0;
  bool staged = false;   // slice holds a copy of host input
  size_t off_in_ptr = 0, off_in_vtx = 0, off_in_dem = 0;
  size_t off_in_cmp = 0;   // compact upload (stage_compact), 0 if none
  size_t off_ctr, off_death_e, off_death_v, off_forced, off_fw;
  size_t off_vptr, off_vedg, off_vend;
  size_t off_erow0, off_erow1, off_vrow0, off_vrow1, off_ecol, off_vcol;
  size_t off_rs, off_rf, off_rid, off_cnt, off_kill, off_esz, off_vdeg, off_eslk;
  size_t off_tkl, off_tkh, off_toff, off_bstat, off_blob;
  int64_t blob_cap = 0;
};

// stage_input: the slice holds a copy of host input (the arrays as the
// kernels read them); stage_compact: also room for the compact upload they
// are widened from on the device (the server's requests).
InstLayout inst_layout(int32_t n, int32_t m, int64_t nnz, bool stage_input, bool stage_compact = false);
// Device bytes of a set's control block for `ninst` instances.
size_t set_control_bytes(int32_t ninst);

// Prefix arrays over the instances of a set (ninst + 1 each) counting the
// work units each round's launches cover: dense tiles, sparse tiles, blocks
// of kBlock rows and contraction candidates (tile pairs J >= I of the dense
// tiles, T (T + 1) / 2), per phase.  The host fills them from the full sizes;
// every round end recounts them from the alive rows, so grids and persistent
// loops cover only alive work.
enum AliveWork : int {
  AP_ETD = 0, AP_VTD = 1, AP_ETS = 2, AP_VTS = 3, AP_EB = 4, AP_VB = 5, AP_EP = 6, AP_VP = 7, AP_N = 8
};

// Launch context of one set.
struct LaunchCtx {
  hipStream_t stream = nullptr;
  DInst* insts = nullptr;        // device table [ninst]
  int32_t ninst = 0;
  // prefix arrays [ninst+1] over instances: edge tiles, vertex tiles,
  // edge blocks, vertex blocks
  int32_t* etp = nullptr;
  int32_t* vtp = nullptr;
  int32_t* ebp = nullptr;
  int32_t* vbp = nullptr;
  int32_t* lpb = nullptr;        // [ninst+1] prefix of LDS-prepare workgroups
  int32_t n_lblocks = 0;         // their total
  int32_t* gbp = nullptr;        // [ninst+1] prefix of kBlock-hyperedge blocks of the other members
  int32_t n_gblocks = 0;         // their total (the global-atomic prepare's blocks)
  int32_t prep_long = 0;         // those members' hyperedges are long on average: more lanes each
  int32_t max_local_n = 0;       // largest vertex count among those members
  int32_t* ap = nullptr;         // AP_N prefix arrays of alive work units
  int32_t n_etiles = 0, n_vtiles = 0, n_eblocks = 0, n_vblocks = 0;
  int32_t cus = 256;             // compute units of the device (persistent grids)
  int32_t* gctr = nullptr;       // G_N global counters
  int32_t gemm_grid = 0;         // persistent contraction grid
  int32_t variant = 1;           // dense tile kernel of the set: 1 int8 MFMA, 2 bitset popcount
  int32_t has_dense = 1;         // some member uses dense tiles
  int32_t has_sparse = 0;        // some member uses sparse counts
  int32_t has_fe = 0;            // some member applies the full-edge rule
  int32_t rule_se = 0;           // the members apply SE instead of DP (one rule per set)
  int32_t sparse_force_range = 0;  // sparse variant: always count over dense id ranges
  int32_t sparse_big = 0;          // sparse counting with the big victim tables: some sparse
                                   // member's hyperedges have many product terms each
  int32_t gemm_lds = 0;            // int8 variant kernel: 0 direct loads, 1 LDS via registers, 2 async copies
  int32_t fuse_end = 0;            // one instance, no FE: the vertex compaction ends the round
  int32_t count_work = 0;          // profiled runs: the dense kernels add to the work counters
                                   // (rows, entries, blob bytes, contraction chunks)
  int32_t* out = nullptr;        // gather target
  int64_t* ooff = nullptr;       // [ninst] int32 offsets into out
  // host-mapped pinned int32[2 kFlagSlots] (or null): each round end stores
  // its sequence number and active count into slot pair G_RSEQ mod
  // kFlagSlots, so the host polls without a copy or an event
  int32_t* hflag = nullptr;
};

// Widening of one instance's compact upload (batched host inputs cross the
// bus as 32-bit offsets and, when n <= 65536, 16-bit vertex ids) into the
// arrays the kernels read: edge_ptr as int64, edge_vtx as int32, demand.
struct WidenJob {
  const int32_t* sptr;   // m+1 offsets
  const void* svtx;      // nnz ids, uint16 if vtx16 else int32
  const int32_t* sdem;   // m demands
  int64_t* dptr;
  int32_t* dvtx;
  int32_t* ddem;
  int64_t nnz;
  int32_t m, vtx16;
};
constexpr int kWidenBlocks = 64;   // workgroups per instance
void launch_widen(hipStream_t stream, const WidenJob* jobs, int count);

void launch_prepare(const LaunchCtx& c);
// Steps of a phase (vertex = false: edge phase / DP, true: vertex phase / MD).
void launch_rows(const LaunchCtx& c, bool vertex);         // rows, windows, encode
void launch_rows_sparse(const LaunchCtx& c, bool vertex);  // the sparse members' rows
void launch_rows_dense(const LaunchCtx& c, bool vertex);   // the dense members' rows and tiles
void launch_contraction(const LaunchCtx& c, bool vertex);  // tile pairs, fused contraction + test
// ... its two parts: sparse counting (members of the sparse variant), then
// the dense tile contraction (int8 / bitset members)
void launch_contraction_sparse(const LaunchCtx& c, bool vertex);
void launch_contraction_dense(const LaunchCtx& c, bool vertex);
void launch_compact(const LaunchCtx& c, bool vertex);      // deletion decision, compaction
void launch_fe(const LaunchCtx& c);                        // FE pass and its compactions
void launch_round_end(const LaunchCtx& c);
void launch_delay(hipStream_t stream, long long ticks);
// Where k_gather writes a set's results in c.out: the members' counters and
// their kept hyperedge and vertex counts (int32 words at word offsets ctr
// and kept), then death_e, death_v and the final demands (0 for a deleted
// hyperedge), each concatenated over the members, at byte offsets de_b,
// dv_b, dem_b, as int32 or, with `narrow`, as uint16 (the host picks it when
// every value fits: rounds run and vertex counts below 2^16, and a demand
// never exceeds its hyperedge's size), then the forced flags as bytes.
struct GatherLayout {
  int64_t ctr, kept, de_b, dv_b, dem_b, forced_b;
  int32_t narrow;
};
// c.ooff holds the members' hyperedge offsets (ninst + 1) then their vertex
// offsets (ninst + 1) in those arrays.
void launch_gather(const LaunchCtx& c, const GatherLayout& g);
void launch_gather_ctr(const LaunchCtx& c);
// Per instance, the sum over its hyperedges of (last id - first id + 1)
// added to spans[x] (zeroed by the caller).
void launch_span(const LaunchCtx& c, unsigned long long* spans);

}  // namespace mhsk
