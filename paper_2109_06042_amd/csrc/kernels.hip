// kernels.hip -- gfx950 kernels of the DP + MD round loop.
//
// Data layout (per instance, see engine.h):
//  * The input CSR (edge_ptr int64, edge_vtx int32, demand int32) is read in
//    place; a CSC (vptr, vedg) is built once on the device.
//  * Alive hyperedges / vertices are kept as stable compact lists (erow,
//    vrow) in "slot order": hyperedges sorted by their first vertex, so that
//    interval-like instances give banded incidence tiles; vertices by id.
//    The tie breaks of Algorithms 1 and 2 always compare ORIGINAL ids (rid),
//    so the slot order changes nothing in the result.
//  * A phase's contraction operand is the compact incidence matrix (rows =
//    alive hyperedges and K = alive vertices for A A^T; rows = alive vertices
//    and K = alive hyperedges for A^T A), cut into tiles of 128 rows.  Each
//    tile stores only its K window [tkl, tkh) in chunks of 64 (every column
//    outside the window is zero in all of the tile's rows), already in the
//    operand order of v_mfma_i32_16x16x64_i8: for chunk c and 16-row block
//    rb a 1 KiB block in which lane l = 16*g + (row % 16) owns bytes
//    k = 16*g .. 16*g+15 of its row.  A wave loads one fragment with one
//    coalesced 16-byte load per lane.
//  * Tile pairs whose windows do not overlap have a zero product block.  Every
//    alive hyperedge keeps at least f(e) alive vertices, so a zero
//    intersection never satisfies supersedence (f_i - s_i <= 0 < f_j), and a
//    zero vertex-pair count only matches an isolated vertex, which MD deletes
//    anyway: such pairs are skipped.  Both products are symmetric, so only
//    tile pairs I <= J are computed and the epilogue tests both directions.
#include "engine.h"

namespace mhsk {

typedef int v4i __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Orders a wave's LDS accesses (LDS operations of one wave complete in
// issue order; this keeps the compiler from moving them across).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Kernel-side view of an instance descriptor: the same fields as DInst with
// every array in the global address space.  Loads and stores through it
// compile to global_* instructions; through generic pointers they would be
// flat_* instructions, which count in the LDS wait counter too, so that
// every wait for an LDS access would also wait for the global loads in
// flight.
#define GLOBAL __attribute__((address_space(1)))
struct KInst {
  int32_t n, m;
  int64_t nnz;
  const GLOBAL int64_t* eptr;
  const GLOBAL int32_t* evtx;
  const GLOBAL int32_t* dem;
  GLOBAL int32_t* vptr;
  GLOBAL int32_t* vedg;
  GLOBAL int32_t* vend;
  GLOBAL int32_t* death_e;
  GLOBAL int32_t* death_v;
  GLOBAL int32_t* erow[2];
  GLOBAL int32_t* vrow[2];
  GLOBAL int32_t* ecol;
  GLOBAL int32_t* vcol;
  GLOBAL int32_t* rs;
  GLOBAL int32_t* rf;
  GLOBAL int32_t* rid;
  GLOBAL int32_t* cnt;
  GLOBAL uint8_t* kill;
  GLOBAL int32_t* esz;
  GLOBAL int32_t* vdeg;
  GLOBAL uint8_t* eslk;
  GLOBAL int32_t* tkl;
  GLOBAL int32_t* tkh;
  GLOBAL int64_t* toff;
  GLOBAL uint64_t* bstat;
  GLOBAL int8_t* blob;
  int64_t blob_cap;
  GLOBAL int32_t* ctr;
  GLOBAL int32_t* fw;
  GLOBAL uint8_t* forced;
  int32_t variant;
  int32_t rule_se;
  int32_t rule_fe;
  int32_t prep_lds;
};

template <class T>
__device__ __forceinline__ GLOBAL T* gptr(T* p) { return (GLOBAL T*)p; }
template <class T>
__device__ __forceinline__ const GLOBAL T* gptr(const T* p) { return (const GLOBAL T*)p; }

__device__ __forceinline__ KInst kview(const DInst& d) {
  KInst k;
  k.n = d.n; k.m = d.m; k.nnz = d.nnz;
  k.eptr = gptr(d.eptr); k.evtx = gptr(d.evtx); k.dem = gptr(d.dem);
  k.vptr = gptr(d.vptr); k.vedg = gptr(d.vedg); k.vend = gptr(d.vend);
  k.death_e = gptr(d.death_e); k.death_v = gptr(d.death_v);
  k.erow[0] = gptr(d.erow[0]); k.erow[1] = gptr(d.erow[1]);
  k.vrow[0] = gptr(d.vrow[0]); k.vrow[1] = gptr(d.vrow[1]);
  k.ecol = gptr(d.ecol); k.vcol = gptr(d.vcol);
  k.rs = gptr(d.rs); k.rf = gptr(d.rf); k.rid = gptr(d.rid); k.cnt = gptr(d.cnt);
  k.kill = gptr(d.kill); k.esz = gptr(d.esz); k.vdeg = gptr(d.vdeg); k.eslk = gptr(d.eslk);
  k.tkl = gptr(d.tkl); k.tkh = gptr(d.tkh); k.toff = gptr(d.toff); k.bstat = gptr(d.bstat);
  k.blob = gptr(d.blob); k.blob_cap = d.blob_cap;
  k.ctr = gptr(d.ctr); k.fw = gptr(d.fw); k.forced = gptr(d.forced);
  k.variant = d.variant; k.rule_se = d.rule_se; k.rule_fe = d.rule_fe; k.prep_lds = d.prep_lds;
  return k;
}

// Device-scope relaxed atomics on global memory (what atomicAdd and
// atomicCAS do on generic pointers, as global_atomic_* instructions).
template <class T>
__device__ __forceinline__ T gadd(GLOBAL T* p, T v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ T gcas(GLOBAL T* p, T expected, T desired) {
  __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
  return expected;
}

// Largest x in [0, n) with prefix[x] <= g (prefix[0] = 0, prefix[n] > g).
__device__ __forceinline__ int find_owner(const int32_t* prefix, int n, int g) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ------------------------------------------------------------ block scans
// Exclusive scan of one int per thread (blockDim a multiple of 64, at most
// 1024); returns the prefix, writes the block total.  Each wave scans the
// wave totals itself (lane w reads wave w's, a 16-lane shuffle scan), so no
// thread makes a serial pass over them.  `sh` needs blockDim/64 ints.
__device__ int block_exscan(int v, int* sh, int* total) {
  const int lane = lane_id();
  const int wid = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[wid] = x;
  __syncthreads();
  int t = lane < nw ? sh[lane] : 0;
#pragma unroll
  for (int o = 1; o < 16; o <<= 1) {
    const int y = __shfl_up(t, o, 64);
    if (lane >= o) t += y;
  }
  const int before = wid > 0 ? __shfl(t, wid - 1, 64) : 0;
  *total = __shfl(t, nw - 1, 64);
  __syncthreads();   // sh is read by every wave before a next scan writes it
  return before + x - v;
}

__device__ __forceinline__ int wave_min(int x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = min(x, __shfl_xor(x, o, 64));
  return x;
}
__device__ __forceinline__ int wave_max(int x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = max(x, __shfl_xor(x, o, 64));
  return x;
}

__device__ __forceinline__ bool inst_idle(const GLOBAL int32_t* ctr) {
  return ctr[C_DONE] != 0 || ctr[C_ERR] != 0;
}

// Members of a set choose dense tiles (int8 / bitset) or sparse counts.
__device__ __forceinline__ bool is_sparse(const KInst& I) { return I.variant == 3; }

__device__ __forceinline__ void set_err(GLOBAL int32_t* ctr, int code) {
  gcas(&ctr[C_ERR], 0, code);
}

__device__ __forceinline__ long long& ctr64(int32_t* ctr, int idx) {
  return *reinterpret_cast<long long*>(ctr + idx);
}

// Words that blocks of one launch exchange (status words, published
// windows) are read and written as device-scope atomics, so no block sees a
// stale cached copy.
__device__ __forceinline__ uint64_t st_load(const GLOBAL uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_store(GLOBAL uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
constexpr long long kSpinMax = 1ll << 20;     // bound on polls of another block's word (about a second)

// Work units of a launch map to (instance, unit) through a prefix over the
// instances, held in LDS when it fits (kPrefLds entries).
constexpr int kPrefLds = 1024;

__device__ __forceinline__ const int32_t* cache_prefix(const int32_t* g, int ninst, int32_t* s) {
  if (ninst > 1 && ninst < kPrefLds) {
    for (int i = threadIdx.x; i <= ninst; i += blockDim.x) s[i] = g[i];
    __syncthreads();
    return s;
  }
  return g;
}

// (w is the same for the whole workgroup: the owner goes to a scalar
// register, and the instance's descriptor with it)
__device__ __forceinline__ int unit_owner(const int32_t* pf, int ninst, int w) {
  return ninst == 1 ? 0 : __builtin_amdgcn_readfirstlane(find_owner(pf, ninst, w));
}

// Workgroups are dealt to the eight XCDs in turn (workgroup b to XCD b mod
// 8).  xcd_remap(b, n) gives workgroup b < n the logical index that puts
// consecutive logical indices on one XCD (XCD x takes a contiguous run of
// about n / 8), so the units of one instance share an L2.
__device__ __forceinline__ int xcd_remap(int b, int n) {
  const int q = n >> 3, r = n & 7, x = b & 7, k = b >> 3;
  return x * q + min(x, r) + k;
}

// A persistent loop's share of `total` units when they are split into eight
// contiguous runs, one per XCD, each walked by that XCD's workgroups in
// turn: units *first, *first + *step, ... below *end.  Sets of one and grids
// of fewer than eight workgroups keep the plain stride over all units.
__device__ __forceinline__ void xcd_share(int64_t total, bool split, int64_t* first, int64_t* end, int* step) {
  const int G = gridDim.x, b = blockIdx.x;
  if (!split || G < 8) {
    *first = b;
    *end = total;
    *step = G;
    return;
  }
  const int x = b & 7;
  const int64_t q = total >> 3, r = total & 7;
  const int64_t s = x * q + min<int64_t>(x, r);
  *first = s + (b >> 3);
  *end = s + q + (x < r ? 1 : 0);
  *step = (G >> 3) + (x < (G & 7) ? 1 : 0);
}

// The two parity buffers of the compact row lists, chosen by a select
// rather than an index, so a descriptor copy stays in registers.
__device__ __forceinline__ GLOBAL int32_t* erow_list(const KInst& I, int k) { return k ? I.erow[1] : I.erow[0]; }
__device__ __forceinline__ GLOBAL int32_t* vrow_list(const KInst& I, int k) { return k ? I.vrow[1] : I.vrow[0]; }

// ---------------------------------------------------------------- prepare
// One launch for the counters and the per-vertex state: thread g of the
// grid initializes instance g's counters and compaction status words (the
// global counters: thread 0), and workgroup b < nvb the vertices of block b
// (prefix `vbp` over the instances).
__global__ __launch_bounds__(kBlock) void k_prep_init(const DInst* __restrict__ insts, int ninst,
                                                      const int32_t* vbp, int nvb, int32_t* gctr) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g == 0)
    for (int i = 0; i < G_N; ++i) gctr[i] = 0;
  if (g < ninst) {
    const KInst I = kview(insts[g]);
    for (int i = 0; i < kCtr; ++i) I.ctr[i] = 0;
    I.ctr[C_MA] = I.m;
    I.ctr[C_NA] = I.n;
    I.ctr[C_ROUND] = 1;
    if (I.m > 0 && I.eptr[0] != 0) I.ctr[C_ERR] = E_PTR;
    // compaction status words: a zero word is "not ready" in every epoch
    const int nbk = (max(I.n, I.m) + kBlock - 1) / kBlock;
    for (int b = 0; b < nbk; ++b) I.bstat[b] = 0;
  }
  if ((int)blockIdx.x >= nvb) return;
  // per vertex: clear CSC counts and sort buckets, initial vertex state
  const int x = unit_owner(vbp, ninst, blockIdx.x);
  const KInst I = kview(insts[x]);
  const int v = (blockIdx.x - vbp[x]) * kBlock + threadIdx.x;
  if (v >= I.n) return;
  I.vend[v] = 0;
  I.rs[v] = 0;
  I.death_v[v] = 0;
  I.forced[v] = 0;
  I.vcol[v] = v;
  I.vrow[0][v] = v;
}

// The per-hyperedge prepare kernels give each hyperedge L lanes that stride
// over its entries (kPrepLanes, or kPrepLanesLong for sets whose
// hyperedges are long on average), and launch L workgroups per kBlock
// hyperedges, so no lane walks a long serial chain of dependent atomics.
constexpr int kPrepLanes = 8;
constexpr int kPrepLanesLong = 64;

template <int L>
__device__ __forceinline__ int prep_edge(const int32_t* ebp, int ninst, int* x) {
  const int blk = blockIdx.x / L;
  *x = unit_owner(ebp, ninst, blk);
  return (blk - ebp[*x]) * kBlock + (blockIdx.x % L) * (kBlock / L) + threadIdx.x / L;
}

// Size of the first-vertex bucket of vertex v (bucket starts in rid after
// the scan).
__device__ __forceinline__ int bucket_size(const KInst& I, int v) {
  return (v + 1 < I.n ? I.rid[v + 1] : I.m) - I.rid[v];
}
constexpr int kSortBucket = 256;   // larger buckets keep their arrival order

// The LDS prepare gives each hyperedge kLdsLanes lanes: the members it
// serves have short hyperedges on average, and with eight lanes each about
// half of them idled (count and fill 2.07 -> 1.67 ms on the 512-instance
// batch with four).
constexpr int kLdsLanes = 4;
// First bad entry of hyperedge e (kLdsLanes lanes stride over it, the same
// checks as k_prep_edges): 0 or an ErrCode, on every lane of the group.
__device__ __forceinline__ int edge_check(const KInst& I, int e, int sub, int64_t* pa, int64_t* pb) {
  int code = 0;
  const int64_t a = I.eptr[e], b = I.eptr[e + 1];
  if (a < 0 || b < a || b > I.nnz || (e == I.m - 1 && b != I.nnz)) code = E_PTR;
  else if (b == a) code = E_EMPTY;
  else if (I.dem[e] < 1 || (int64_t)I.dem[e] > b - a) code = E_DEMAND;
  int64_t bad = INT64_MAX;
  if (!code) {
    for (int64_t p = a + sub; p < b; p += kLdsLanes) {
      const int v = I.evtx[p];
      int c = 0;
      if (v < 0 || v >= I.n) c = E_RANGE;
      else if (p > a) {
        const int u = I.evtx[p - 1];
        if (u >= 0 && u < I.n && u >= v) c = E_ORDER;
      }
      if (c) { bad = ((p - a) << 4) | c; break; }
    }
  }
#pragma unroll
  for (int o = kLdsLanes / 2; o > 0; o >>= 1) {
    const int64_t y = __shfl_xor(bad, o, kLdsLanes);
    bad = y < bad ? y : bad;
  }
  if (!code && bad != INT64_MAX) code = (int)(bad & 15);
  *pa = a;
  *pb = b;
  return code;
}

// LDS prepare of small members of a set (prep_lds): workgroup g of G of an
// instance (prefix `lpb`) takes hyperedges [m g / G, m (g + 1) / G).  The
// count kernel validates them and counts degrees and first-vertex buckets
// in LDS, then adds each nonzero count to the instance's global totals
// (vend, rs) with one atomic, whose old value is the workgroup's offset in
// that vertex's list or bucket: kept in the tile blob region, which is free
// until the first round (n ints per workgroup for the lists, then n per
// workgroup for the buckets).  k_prep_scan turns the totals into starts
// (and, for these members, vend into list ends); the fill kernel starts its
// LDS cursors at start + offset and places its entries.  Dynamic LDS: 2 n
// ints.
__device__ __forceinline__ void lds_range(const int32_t* lpb, int ninst, int* x, int* g, int* G, int* e0, int* e1,
                                          const DInst* __restrict__ insts, KInst* I) {
  // an instance's workgroups share an XCD: the runs they place next to each
  // other in its vertex lists then meet in one L2 instead of reaching HBM
  // as partial lines
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  *x = unit_owner(lpb, ninst, b);
  *I = kview(insts[*x]);
  *g = b - lpb[*x];
  *G = lpb[*x + 1] - lpb[*x];
  *e0 = (int)((int64_t)I->m * *g / *G);
  *e1 = (int)((int64_t)I->m * (*g + 1) / *G);
}

__global__ __launch_bounds__(1024) void k_prep_lcount(const DInst* __restrict__ insts, int ninst,
                                                       const int32_t* lpb) {
  extern __shared__ int s_lds[];
  int x, g, G, e0, e1;
  KInst I;
  lds_range(lpb, ninst, &x, &g, &G, &e0, &e1, insts, &I);
  if (I.ctr[C_ERR]) return;
  const int n = I.n, tid = threadIdx.x, sub = tid % kLdsLanes;
  int* s_deg = s_lds;
  int* s_bk = s_lds + n;
  for (int v = tid; v < n; v += blockDim.x) { s_deg[v] = 0; s_bk[v] = 0; }
  __syncthreads();
  constexpr int EPB = 1024 / kLdsLanes;   // hyperedges per pass
  for (int eb = e0; eb < e1; eb += EPB) {
    const int e = eb + tid / kLdsLanes;
    if (e >= e1) break;
    if (sub == 0) {
      I.death_e[e] = 0;
      I.ecol[e] = -1;
      I.fw[e] = I.dem[e];
    }
    int64_t a, b;
    const int code = edge_check(I, e, sub, &a, &b);
    if (code) {
      if (sub == 0) set_err(I.ctr, code);
      continue;
    }
    if (sub == 0) I.eslk[e] = (uint8_t)min((int)(b - a) - I.dem[e], 254);
    for (int64_t p = a + sub; p < b; p += kLdsLanes) atomicAdd(&s_deg[I.evtx[p]], 1);
    if (sub == 0) atomicAdd(&s_bk[I.evtx[a]], 1);
  }
  __syncthreads();
  GLOBAL int32_t* ofs = reinterpret_cast<GLOBAL int32_t*>(I.blob);
  for (int v = tid; v < n; v += blockDim.x) {
    const int d = s_deg[v], k = s_bk[v];
    if (d) ofs[(int64_t)g * n + v] = gadd(&I.vend[v], d);
    if (k) ofs[(int64_t)(G + g) * n + v] = gadd(&I.rs[v], k);
  }
}

// The fill stages a workgroup's entries in LDS sorted by vertex (local
// counts, their scan, placement at local cursors) and writes them out in
// that order, so the entries it adds to one vertex list leave as one run
// from consecutive lanes rather than as single words at scattered times.  A
// workgroup with more than kFillStage incidences places its entries
// directly.  Dynamic LDS: 2 n ints + kFillStage (n <= kLocalN = 8192).
constexpr int kFillStage = 16384;
__global__ __launch_bounds__(1024) void k_prep_lfill(const DInst* __restrict__ insts, int ninst,
                                                      const int32_t* lpb) {
  extern __shared__ int s_lds[];
  __shared__ int s_sh[16];
  int x, g, G, e0, e1;
  KInst I;
  lds_range(lpb, ninst, &x, &g, &G, &e0, &e1, insts, &I);
  if (I.ctr[C_ERR]) return;
  const int n = I.n, tid = threadIdx.x, sub = tid % kLdsLanes;
  int* s_cur = s_lds;
  int* s_bk = s_lds + n;
  int* s_stage = s_lds + 2 * n;
  // this workgroup's offsets in the lists and buckets (a vertex absent from
  // its hyperedges reads an offset it never uses)
  const GLOBAL int32_t* ofs = reinterpret_cast<const GLOBAL int32_t*>(I.blob);
  const int L = e1 > e0 ? (int)(I.eptr[e1] - I.eptr[e0]) : 0;
  const bool staged = L <= kFillStage;
  for (int v = tid; v < n; v += blockDim.x) {
    s_cur[v] = staged ? 0 : I.vptr[v] + ofs[(int64_t)g * n + v];
    s_bk[v] = I.rid[v] + ofs[(int64_t)(G + g) * n + v];
  }
  __syncthreads();
  const bool sp = is_sparse(I);
  constexpr int EPB = 1024 / kLdsLanes;
  if (staged) {
    for (int eb = e0; eb < e1; eb += EPB) {
      const int e = eb + tid / kLdsLanes;
      if (e >= e1) break;
      const int64_t a = I.eptr[e], b = I.eptr[e + 1];
      for (int64_t p = a + sub; p < b; p += kLdsLanes) atomicAdd(&s_cur[I.evtx[p]], 1);
    }
    __syncthreads();
    // exclusive scan of the local counts in place, eight vertices per thread
    {
      const int v0 = tid * 8;
      int c[8], sum = 0;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        c[k] = v0 + k < n ? s_cur[v0 + k] : 0;
        sum += c[k];
      }
      int tot;
      int run = block_exscan(sum, s_sh, &tot);
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        if (v0 + k < n) s_cur[v0 + k] = run;
        run += c[k];
      }
    }
    __syncthreads();
  }
  for (int eb = e0; eb < e1; eb += EPB) {
    const int e = eb + tid / kLdsLanes;
    if (e >= e1) break;
    const int64_t a = I.eptr[e], b = I.eptr[e + 1];
    for (int64_t p = a + sub; p < b; p += kLdsLanes) {
      const int pos = atomicAdd(&s_cur[I.evtx[p]], 1);
      if (staged) s_stage[pos] = e;
      else I.vedg[pos] = e;
    }
    if (sub == 0) {
      const int v = I.evtx[a];
      const int pos = atomicAdd(&s_bk[v], 1);
      erow_list(I, (sp || bucket_size(I, v) > kSortBucket) ? 0 : 1)[pos] = e;
    }
  }
  if (!staged) return;
  __syncthreads();
  // s_cur[v] is now the local end of v's run: the run holding local
  // position i is the first vertex whose end exceeds i
  for (int i = tid; i < L; i += blockDim.x) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (s_cur[mid] > i) hi = mid; else lo = mid + 1;
    }
    const int start = lo > 0 ? s_cur[lo - 1] : 0;
    I.vedg[I.vptr[lo] + ofs[(int64_t)g * n + lo] + (i - start)] = s_stage[i];
  }
}

// per hyperedge of the members not prepared in LDS (prefix `gbp` over their
// blocks of kBlock hyperedges): validation, CSC degree count, first-vertex
// bucket count.  The error reported for a hyperedge is that of its first bad
// entry (a pointer, size or demand error before any entry).
template <int L>
__global__ __launch_bounds__(kBlock) void k_prep_edges(const DInst* __restrict__ insts, int ninst, const int32_t* gbp) {
  int x;
  const int e = prep_edge<L>(gbp, ninst, &x);
  const KInst I = kview(insts[x]);
  if (I.prep_lds) return;
  const int sub = threadIdx.x % L;
  const bool mine = e < I.m;
  int64_t a = 0, b = 0;
  int code = 0;
  if (mine) {
    if (sub == 0) {
      I.death_e[e] = 0;
      I.ecol[e] = -1;
      I.fw[e] = I.dem[e];
    }
    a = I.eptr[e];
    b = I.eptr[e + 1];
    if (a < 0 || b < a || b > I.nnz || (e == I.m - 1 && b != I.nnz)) code = E_PTR;
    else if (b == a) code = E_EMPTY;
    else if (I.dem[e] < 1 || (int64_t)I.dem[e] > b - a) code = E_DEMAND;
  }
  // first bad entry of this lane's stride, as (offset << 4 | code)
  int64_t bad = INT64_MAX;
  if (mine && !code) {
    for (int64_t p = a + sub; p < b; p += L) {
      const int v = I.evtx[p];
      int c = 0;
      if (v < 0 || v >= I.n) c = E_RANGE;
      else if (p > a) {
        const int u = I.evtx[p - 1];
        if (u >= 0 && u < I.n && u >= v) c = E_ORDER;
      }
      if (c) { bad = ((p - a) << 4) | c; break; }
    }
  }
#pragma unroll
  for (int o = L / 2; o > 0; o >>= 1) {
    const int64_t y = __shfl_xor(bad, o, L);
    bad = y < bad ? y : bad;
  }
  if (!mine) return;
  if (!code && bad != INT64_MAX) code = (int)(bad & 15);
  if (code) {
    if (sub == 0) set_err(I.ctr, code);
    return;
  }
  if (sub == 0) I.eslk[e] = (uint8_t)min((int)(b - a) - I.dem[e], 254);
  for (int64_t p = a + sub; p < b; p += L) gadd(&I.vend[I.evtx[p]], 1);
  if (sub == 0) gadd(&I.rs[I.evtx[a]], 1);
}

// per instance: exclusive scans building vptr and the bucket starts, eight
// consecutive vertices per thread (two 16-byte loads and stores per array
// where all eight are in range); the 16 wave totals go through LDS and
// every wave adds those before it
__global__ __launch_bounds__(1024) void k_prep_scan(const DInst* __restrict__ insts) {
  constexpr int R = 8;
  __shared__ int s_wc[16], s_wb[16];
  const KInst I = kview(insts[blockIdx.x]);
  if (I.ctr[C_ERR]) {
    if (threadIdx.x == 0) I.ctr[C_DONE] = 1;
    return;
  }
  const int lane = lane_id(), wid = threadIdx.x >> 6;
  int carry_c = 0, carry_b = 0;
  for (int base = 0; base < I.n; base += 1024 * R) {
    const int v0 = base + threadIdx.x * R;
    const bool full = v0 + R <= I.n;
    int c[R], bk[R];
    if (full) {
      const v4i c0 = *reinterpret_cast<const GLOBAL v4i*>(I.vend + v0);
      const v4i c1 = *reinterpret_cast<const GLOBAL v4i*>(I.vend + v0 + 4);
      const v4i b0 = *reinterpret_cast<const GLOBAL v4i*>(I.rs + v0);
      const v4i b1 = *reinterpret_cast<const GLOBAL v4i*>(I.rs + v0 + 4);
      c[0] = c0.x; c[1] = c0.y; c[2] = c0.z; c[3] = c0.w; c[4] = c1.x; c[5] = c1.y; c[6] = c1.z; c[7] = c1.w;
      bk[0] = b0.x; bk[1] = b0.y; bk[2] = b0.z; bk[3] = b0.w; bk[4] = b1.x; bk[5] = b1.y; bk[6] = b1.z; bk[7] = b1.w;
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const bool in = v0 + r < I.n;
        c[r] = in ? I.vend[v0 + r] : 0;
        bk[r] = in ? I.rs[v0 + r] : 0;
      }
    }
    int sc = 0, sb = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) { sc += c[r]; sb += bk[r]; }
    int xc = sc, xb = sb;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int yc = __shfl_up(xc, o, 64), yb = __shfl_up(xb, o, 64);
      if (lane >= o) { xc += yc; xb += yb; }
    }
    if (lane == 63) { s_wc[wid] = xc; s_wb[wid] = xb; }
    __syncthreads();
    int pc = carry_c + xc - sc, pb = carry_b + xb - sb, tc = 0, tb = 0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int a = s_wc[q], e = s_wb[q];
      if (q < wid) { pc += a; pb += e; }
      tc += a;
      tb += e;
    }
    __syncthreads();   // the totals are read before the next chunk writes them
    // starts in vptr and rid; vend and rs are the fill's cursors (starts),
    // or for LDS-prepared members, which fill from their own cursors, the
    // list ends (rs then unused until the rows kernels overwrite it)
    const int le = I.prep_lds ? 1 : 0;
    int oc[R], ob[R], ec[R];
#pragma unroll
    for (int r = 0; r < R; ++r) { oc[r] = pc; ob[r] = pb; pc += c[r]; pb += bk[r]; ec[r] = le ? pc : oc[r]; }
    if (full) {
      const v4i o0 = v4i{oc[0], oc[1], oc[2], oc[3]}, o1 = v4i{oc[4], oc[5], oc[6], oc[7]};
      const v4i n0 = v4i{ec[0], ec[1], ec[2], ec[3]}, n1 = v4i{ec[4], ec[5], ec[6], ec[7]};
      const v4i p0 = v4i{ob[0], ob[1], ob[2], ob[3]}, p1 = v4i{ob[4], ob[5], ob[6], ob[7]};
      *reinterpret_cast<GLOBAL v4i*>(I.vptr + v0) = o0; *reinterpret_cast<GLOBAL v4i*>(I.vptr + v0 + 4) = o1;
      *reinterpret_cast<GLOBAL v4i*>(I.vend + v0) = n0; *reinterpret_cast<GLOBAL v4i*>(I.vend + v0 + 4) = n1;
      *reinterpret_cast<GLOBAL v4i*>(I.rid + v0) = p0; *reinterpret_cast<GLOBAL v4i*>(I.rid + v0 + 4) = p1;
      *reinterpret_cast<GLOBAL v4i*>(I.rs + v0) = p0; *reinterpret_cast<GLOBAL v4i*>(I.rs + v0 + 4) = p1;
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (v0 + r < I.n) { I.vptr[v0 + r] = oc[r]; I.vend[v0 + r] = ec[r]; I.rid[v0 + r] = ob[r]; I.rs[v0 + r] = ob[r]; }
    }
    carry_c += tc;
    carry_b += tb;
  }
  if (threadIdx.x == 0) I.vptr[I.n] = carry_c;
}

// per hyperedge of the members not prepared in LDS (prefix `gbp`): CSC fill
// (each list in arrival order: nothing depends on it) and bucket placement
// by first vertex.  Buckets up to kSortBucket are
// staged in erow[1] (free until the first compaction) and ordered by id in
// k_prep_rank; larger ones keep their arrival order in erow[0].
template <int L>
__global__ __launch_bounds__(kBlock) void k_prep_fill(const DInst* __restrict__ insts, int ninst, const int32_t* gbp) {
  int x;
  const int e = prep_edge<L>(gbp, ninst, &x);
  const KInst I = kview(insts[x]);
  if (I.ctr[C_ERR] || e >= I.m || I.prep_lds) return;
  const int sub = threadIdx.x % L;
  const int64_t a = I.eptr[e], b = I.eptr[e + 1];
  for (int64_t p = a + sub; p < b; p += L) {
    const int pos = gadd(&I.vend[I.evtx[p]], 1);
    I.vedg[pos] = e;
  }
  if (sub == 0) {
    const int v = I.evtx[a];
    const int pos = gadd(&I.rs[v], 1);
    erow_list(I, (is_sparse(I) || bucket_size(I, v) > kSortBucket) ? 0 : 1)[pos] = e;
  }
}

// per hyperedge of a small bucket: its rank among the bucket's hyperedges
// by id gives its slot, so the slot order is (first vertex, id).  The
// sparse variant keeps the arrival order: its counts do not depend on how
// rows fall into tiles.
__global__ void k_prep_rank(const DInst* __restrict__ insts, int ninst, const int32_t* ebp) {
  const int x = unit_owner(ebp, ninst, blockIdx.x);
  const KInst I = kview(insts[x]);
  if (I.ctr[C_ERR] || is_sparse(I)) return;
  const int e = (blockIdx.x - ebp[x]) * kBlock + threadIdx.x;
  if (e >= I.m) return;
  const int v = I.evtx[I.eptr[e]];
  const int n = bucket_size(I, v);
  if (n > kSortBucket) return;
  const int s = I.rid[v];
  const GLOBAL int32_t* st = I.erow[1];
  int rank = 0;
  for (int i = 0; i < n; ++i) rank += st[s + i] < e;
  I.erow[0][s + rank] = e;
}

// Round-1 slack order of the sparse members' vertex lists.  Before the
// first round every vertex is alive, so a hyperedge's slack |e| - f(e) is
// its input size minus its demand (the edge prepare stores it in eslk).  A
// hyperedge e_i can dominate e_j (D_ij under DP: f_i + X_ij >= f_j + s_i
// with X_ij <= s_j; under SE: e_i a subset of e_j with f_i >= f_j) only if
// its slack is at most e_j's.  So each list is reordered by slack class, a
// monotone map of the slack onto kSlackClasses classes, and the end of every
// class is kept in a table of kSlackClasses positions per vertex (in the
// blob, which sparse members use for nothing else): in round 1 a victim
// walks each list only up to the end of its own slack's class.  Later rounds
// walk whole lists (slacks only fall, so the first round's order bounds
// nothing then).  Lists longer than kSlackWide entries are left in place
// with every class ending at the list's end.
constexpr int kSlackR = 8;                        // entries per lane
constexpr int kSlackNarrow = 16 * kSlackR;        // lists sorted by 16 lanes
constexpr int kSlackWide = 64 * kSlackR;          // lists sorted by a wave
__device__ __forceinline__ int slack_class(int s) {
  return s < 8 ? s
               : 8 + (s >= 10) + (s >= 12) + (s >= 15) + (s >= 19) + (s >= 24) + (s >= 32) + (s >= 64);
}
// End of slack class c in vertex v's list: the table is class-major (n
// positions per class), so the victims of one class read one dense stripe.
__device__ __forceinline__ GLOBAL int32_t* slack_end(const KInst& I, int v, int c) {
  return reinterpret_cast<GLOBAL int32_t*>(I.blob) + (int64_t)c * I.n + v;
}

// A counting sort by slack class of the list [a, a + d) of vertex v (d <=
// GL kSlackR) by the GL lanes of a group, in place (every entry is in
// registers before any is written), with the group's class counters
// `cnt` and cursors `cur` in LDS.  `act` is the group's.  The order within
// a class is the cursors' (the counts and tests do not depend on it).
template <int GL>
__device__ __forceinline__ void slack_sort_list(const KInst& I, int v, int a, int d, bool act, int* cnt,
                                                int* cur) {
  const int gl = lane_id() & (GL - 1);
  if (gl < kSlackClasses) cnt[gl] = 0;
  wave_sync();
  int e[kSlackR], k[kSlackR];
#pragma unroll
  for (int u = 0; u < kSlackR; ++u) {
    const int p = u * GL + gl;
    e[u] = act && p < d ? I.vedg[a + p] : -1;
  }
#pragma unroll
  for (int u = 0; u < kSlackR; ++u) k[u] = e[u] >= 0 ? slack_class(I.eslk[e[u]]) : -1;
#pragma unroll
  for (int u = 0; u < kSlackR; ++u)
    if (k[u] >= 0) atomicAdd(&cnt[k[u]], 1);
  wave_sync();
  // class starts: an exclusive scan of the counts over the group's lanes
  const int x = gl < kSlackClasses ? cnt[gl] : 0;
  int incl = x;
#pragma unroll
  for (int o = 1; o < GL; o <<= 1) {
    const int y = __shfl_up(incl, o, GL);
    if (gl >= o) incl += y;
  }
  if (gl < kSlackClasses) {
    cur[gl] = a + incl - x;
    if (act) *slack_end(I, v, gl) = a + incl;
  }
  wave_sync();
#pragma unroll
  for (int u = 0; u < kSlackR; ++u)
    if (k[u] >= 0) I.vedg[atomicAdd(&cur[k[u]], 1)] = e[u];
  wave_sync();
}

// One workgroup per block of kBlock vertices (prefix `vbp`) of the sparse
// members: groups of 16 lanes take the lists of up to kSlackNarrow entries,
// four vertices per wave at a time; longer lists queue for whole waves.
__global__ __launch_bounds__(kBlock) void k_prep_slack(const DInst* __restrict__ insts, int ninst,
                                                       const int32_t* vbp) {
  __shared__ int s_q[kBlock];
  __shared__ int s_nq;
  __shared__ int s_cnt[kBlock / 16][kSlackClasses], s_cur[kBlock / 16][kSlackClasses];
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int x = unit_owner(vbp, ninst, blk);
  const KInst I = kview(insts[x]);
  if (I.ctr[C_ERR] || !is_sparse(I) || I.m == 0) return;
  const int w = threadIdx.x >> 6, lane = lane_id(), q = lane >> 4, gl = lane & 15;
  if (threadIdx.x == 0) s_nq = 0;
  __syncthreads();
  // the wave's 64 vertices: lane l loads the bounds of vertex l, group q
  // takes vertex 4 k + q at step k
  const int vw = (blk - vbp[x]) * kBlock + w * 64;
  const bool lin = vw + lane < I.n;
  const int la = lin ? I.vptr[vw + lane] : 0, ld = lin ? I.vend[vw + lane] - la : 0;
  for (int k = 0; k < 64; k += 4) {
    const int v = vw + k + q;
    const bool in = v < I.n;
    const int a = __shfl(la, k + q, 64), d = __shfl(ld, k + q, 64);
    if (in && d > kSlackNarrow && gl == 0) s_q[atomicAdd(&s_nq, 1)] = v;
    slack_sort_list<16>(I, v, a, d, in && d <= kSlackNarrow, s_cnt[w * 4 + q], s_cur[w * 4 + q]);
  }
  __syncthreads();
  const int nq = s_nq;
  for (int k = w; k < nq; k += kBlock / 64) {
    const int v = s_q[k];
    const int a = I.vptr[v], b = I.vend[v];
    if (b - a <= kSlackWide) {
      slack_sort_list<64>(I, v, a, b - a, true, s_cnt[w * 4], s_cur[w * 4]);
    } else if (lane < kSlackClasses) {
      *slack_end(I, v, lane) = b;
    }
  }
}

void launch_prepare(const LaunchCtx& c) {
  if (!c.ninst) return;
  const int grid = std::max(c.n_vblocks, (c.ninst + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_prep_init, dim3(grid), dim3(kBlock), 0, c.stream, c.insts, c.ninst, c.vbp, c.n_vblocks,
                     c.gctr);
  const size_t lds = (size_t)2 * c.max_local_n * sizeof(int);
  if (c.n_lblocks)
    hipLaunchKernelGGL(k_prep_lcount, dim3(c.n_lblocks), dim3(1024), lds, c.stream, c.insts, c.ninst, c.lpb);
  if (c.n_gblocks && c.prep_long)
    hipLaunchKernelGGL(k_prep_edges<kPrepLanesLong>, dim3(c.n_gblocks * kPrepLanesLong), dim3(kBlock), 0, c.stream,
                       c.insts, c.ninst, c.gbp);
  else if (c.n_gblocks)
    hipLaunchKernelGGL(k_prep_edges<kPrepLanes>, dim3(c.n_gblocks * kPrepLanes), dim3(kBlock), 0, c.stream,
                       c.insts, c.ninst, c.gbp);
  hipLaunchKernelGGL(k_prep_scan, dim3(c.ninst), dim3(1024), 0, c.stream, c.insts);
  if (c.n_lblocks)
    hipLaunchKernelGGL(k_prep_lfill, dim3(c.n_lblocks), dim3(1024), lds + (size_t)kFillStage * sizeof(int), c.stream,
                       c.insts, c.ninst, c.lpb);
  if (c.n_gblocks && c.prep_long)
    hipLaunchKernelGGL(k_prep_fill<kPrepLanesLong>, dim3(c.n_gblocks * kPrepLanesLong), dim3(kBlock), 0, c.stream,
                       c.insts, c.ninst, c.gbp);
  else if (c.n_gblocks)
    hipLaunchKernelGGL(k_prep_fill<kPrepLanes>, dim3(c.n_gblocks * kPrepLanes), dim3(kBlock), 0, c.stream,
                       c.insts, c.ninst, c.gbp);
  if (c.n_eblocks)
    hipLaunchKernelGGL(k_prep_rank, dim3(c.n_eblocks), dim3(kBlock), 0, c.stream, c.insts, c.ninst, c.ebp);
  if (c.has_sparse && c.n_vblocks)
    hipLaunchKernelGGL(k_prep_slack, dim3(c.n_vblocks), dim3(kBlock), 0, c.stream, c.insts, c.ninst, c.vbp);
}

// ------------------------------------------------- rows, windows, encode
// One workgroup of 1024 threads per (instance, tile of 128 compact rows) of
// the phase; LPR = 8 lanes share a row and stride over its entries, keeping
// up to RC of them in registers (8 for hyperedge rows, 16 for the longer
// vertex rows), so each entry is fetched once per round and a lane's loads
// are independent of each other:
//  1. per row: its alive entries (edge phase: compact ids vcol[v] of the
//     hyperedge's alive vertices; vertex phase: ecol[e] of the vertex's alive
//     hyperedges), s = |e| (the diagonal (A A^T)_ee) or d = |E(v)| (the
//     diagonal (A^T A)_vv), the demand f(e) or the largest demand over E(v)
//     (0 if empty), the original id; clears the row's kill flag and count.
//     Vertex rows also partition their hyperedge list in place, alive
//     hyperedges first, and shorten [vptr[v], vend[v]) to them: deletions
//     are final, so later rounds never scan a deleted hyperedge again;
//  2. the tile's K window [kl, kh) in chunks of 64 (its blob space is a
//     fixed stretch per tile);
//  3. zero the window, then set the entries: one byte each in the
//     v_mfma_i32_16x16x64_i8 operand order (int8 variant) or one bit each,
//     one 64-bit word per (chunk, row) (bitset variant).
constexpr int kRowsThreads = 1024;

// Blob address of K chunk c of tile t in a phase: each tile owns a stretch
// as long as the phase's widest possible window (every K chunk), and chunk c
// sits at the same place in it whatever the tile's window, so a reader needs
// neither the window start nor an allocation record.
template <bool VERTEX>
__device__ __forceinline__ int64_t phase_chunks(const KInst& I) {
  return ((VERTEX ? I.m : I.n) + kChunk - 1) / kChunk;
}
template <bool VERTEX, int CB>
__device__ __forceinline__ int64_t chunk_offset(const KInst& I, int t, int c) {
  return ((int64_t)t * phase_chunks<VERTEX>(I) + c) * CB;
}

template <bool VERTEX>
struct RowsCfg {
  static constexpr int LPR = 8;                       // lanes per row
  static constexpr int RPP = kRowsThreads / LPR;      // rows per pass
  static constexpr int NP = kTile / RPP;              // passes over the tile
  static constexpr int RC = VERTEX ? 16 : 8;          // entries cached per lane and pass
};

template <bool VERTEX>
__device__ __forceinline__ void row_range(const KInst& I, int cur, int r, int* id, int64_t* a, int64_t* b) {
  if (!VERTEX) {
    const int e = erow_list(I, cur)[r];
    *id = e;
    *a = I.eptr[e];
    *b = I.eptr[e + 1];
  } else {
    const int v = vrow_list(I, cur)[r];
    *id = v;
    *a = I.vptr[v];
    *b = I.vend[v];
  }
}

// Entry p of a row: the vertex (edge phase) or hyperedge (vertex phase) id.
template <bool VERTEX>
__device__ __forceinline__ int entry_key(const KInst& I, int64_t p) {
  return VERTEX ? I.vedg[p] : I.evtx[p];
}

// A row's entries beyond a lane's cache (positions p0, p0 + LPR, ... below
// b), four at a time with their loads issued together (a position past the
// end reads the row's last entry and is not passed on): f(column, demand)
// for each, the column -1 for a deleted entry.
template <bool VERTEX, int LPR, typename F>
__device__ __forceinline__ void spill_entries(const KInst& I, int64_t p0, int64_t b, F f) {
  const GLOBAL int32_t* cmap = VERTEX ? I.ecol : I.vcol;
  for (int64_t q = p0; q < b; q += 4 * LPR) {
    int key[4], col[4], dem[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) key[u] = entry_key<VERTEX>(I, min(q + u * LPR, b - 1));
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      col[u] = cmap[key[u]];
      dem[u] = VERTEX ? I.fw[key[u]] : 0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (q + u * LPR < b) f(col[u], dem[u]);
  }
}

template <int W>
__device__ __forceinline__ int group_sum(int x) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, W);
  return x;
}

template <int W>
__device__ __forceinline__ int group_exscan(int x) {
  int y = x;
#pragma unroll
  for (int o = 1; o < W; o <<= 1) {
    const int z = __shfl_up(y, o, W);
    if ((int)(threadIdx.x % W) >= o) y += z;
  }
  return y - x;
}

template <bool VERTEX, bool BITS>
__device__ void rows_tile(const KInst& I, int tile, int count) {
  using Cfg = RowsCfg<VERTEX>;
  constexpr int LPR = Cfg::LPR, RPP = Cfg::RPP, NP = Cfg::NP, RC = Cfg::RC;
  constexpr int NW = kRowsThreads / 64;
  static_assert(NP * RPP == kTile, "passes cover the tile");
  __shared__ int smin[NW], smax[NW], sscan[NW];
  __shared__ long long s_off;
  __shared__ int s_kl, s_kh;
  if (inst_idle(I.ctr) || is_sparse(I)) return;
  const int rows = VERTEX ? I.ctr[C_NA] : I.ctr[C_MA];
  if (tile * kTile >= rows) return;
  const int cur = I.ctr[VERTEX ? C_NCOMP_V : C_NCOMP_E] & 1;
  const int t = threadIdx.x;
  const int sub = t % LPR;            // lane within the row group
  int col[NP][RC];                    // cached compact columns (-1: deleted or none)
  int64_t ra[NP], rb[NP];
  bool spill[NP];                     // entries beyond the cache (reloaded later)
  bool gspill[NP];                    // some lane of the row group spilled (vertex rows)
  int rowid[NP];
  int kmin = INT32_MAX, kmax = -1, scanned = 0;
#pragma unroll
  for (int pass = 0; pass < NP; ++pass) {
    const int lr = pass * RPP + t / LPR;
    const int r = tile * kTile + lr;
    const bool valid = r < rows;
    int id = 0;
    int64_t a = 0, b = 0;
    if (valid) row_range<VERTEX>(I, cur, r, &id, &a, &b);
    ra[pass] = a;
    rb[pass] = b;
    rowid[pass] = id;
    gspill[pass] = false;
    int key[RC];
#pragma unroll
    for (int i = 0; i < RC; ++i) {
      const int64_t p = a + sub + (int64_t)i * LPR;
      key[i] = p < b ? entry_key<VERTEX>(I, p) : -1;
    }
    // Column (and demand) loads of all cached entries go out before any is
    // used, so one memory latency covers them; each is masked to the lanes
    // that have the entry.  Consuming a value next to its load (a select on
    // it, in particular) would make each entry wait for its own data.
    int dmv[RC];
    const GLOBAL int32_t* cmap = VERTEX ? I.ecol : I.vcol;
#pragma unroll
    for (int i = 0; i < RC; ++i) {
      col[pass][i] = -1;
      dmv[i] = 0;
      if (key[i] >= 0) {
        col[pass][i] = cmap[key[i]];
        if (VERTEX) dmv[i] = I.fw[key[i]];
      }
    }
    int cnt = 0, mf = 0, dead = 0;
#pragma unroll
    for (int i = 0; i < RC; ++i) {
      const int c = col[pass][i];
      const int alive = c >= 0;
      cnt += alive;
      dead += (key[i] >= 0) & !alive;
      mf = max(mf, dmv[i] & ~(c >> 31));
      kmin = min(kmin, alive ? c : INT32_MAX);
      kmax = max(kmax, c);
    }
    const int64_t rest = a + sub + (int64_t)RC * LPR;
    spill[pass] = rest < b;
    spill_entries<VERTEX, LPR>(I, rest, b, [&](int c, int dm) {
      if (c >= 0) { ++cnt; mf = max(mf, dm); kmin = min(kmin, c); kmax = max(kmax, c); }
    });
    if (VERTEX) {
      // alive-first partition of a fully cached list with deleted entries
      const int any_spill = group_sum<LPR>(spill[pass] ? 1 : 0);
      gspill[pass] = valid && any_spill > 0;
      const int alive_tot = group_sum<LPR>(cnt);
      const int dead_tot = group_sum<LPR>(dead);
      int ap = group_exscan<LPR>(cnt);
      int dp = alive_tot + group_exscan<LPR>(dead);
      if (valid && !any_spill && dead_tot > 0) {
#pragma unroll
        for (int i = 0; i < RC; ++i) {
          if (key[i] < 0) continue;
          if (col[pass][i] >= 0) I.vedg[a + ap++] = key[i];
          else I.vedg[a + dp++] = key[i];
        }
        if (sub == 0) I.vend[id] = (int32_t)(a + alive_tot);
      }
    }
    cnt = group_sum<LPR>(cnt);
#pragma unroll
    for (int o = LPR / 2; o > 0; o >>= 1) mf = max(mf, __shfl_xor(mf, o, LPR));
    if (valid && sub == 0) {
      scanned += (int)(b - a);
      I.rs[r] = cnt;
      I.rf[r] = VERTEX ? mf : I.fw[id];
      I.rid[r] = id;
      I.kill[r] = 0;
      if (VERTEX) I.cnt[r] = 0;
    }
  }
  kmin = wave_min(kmin);
  kmax = wave_max(kmax);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) scanned += __shfl_xor(scanned, o, 64);
  if (lane_id() == 0) { smin[t >> 6] = kmin; smax[t >> 6] = kmax; sscan[t >> 6] = scanned; }
  __syncthreads();
  constexpr int CB = BITS ? kChunkBytesBits : kChunkBytes;
  if (t == 0) {
    int lo = INT32_MAX, hi = -1, sc = 0;
    for (int w = 0; w < NW; ++w) { lo = min(lo, smin[w]); hi = max(hi, smax[w]); sc += sscan[w]; }
    if (count) {
      gadd(reinterpret_cast<GLOBAL unsigned long long*>(&I.ctr[C_ROWS_SUM]),
                (unsigned long long)min(kTile, rows - tile * kTile));
      gadd(reinterpret_cast<GLOBAL unsigned long long*>(&I.ctr[C_ENTRIES_SUM]), (unsigned long long)sc);
    }
    s_kl = s_kh = 0;
    I.tkl[tile] = 0;
    I.tkh[tile] = 0;
    if (hi >= 0) {
      // fixed place per (tile, chunk): no allocation round trip
      const int kl = lo / kChunk, kh = hi / kChunk + 1;
      const long long bytes = (long long)(kh - kl) * CB;
      const long long off = chunk_offset<VERTEX, CB>(I, tile, kl);
      if (off + bytes > I.blob_cap) {
        set_err(I.ctr, E_CAPACITY);
      } else {
        I.tkl[tile] = kl;
        I.tkh[tile] = kh;
        I.toff[tile] = off;
        if (tile == 0) {
          const int kalive = VERTEX ? I.ctr[C_MA] : I.ctr[C_NA];
          I.ctr[VERTEX ? C_WIDE_V : C_WIDE_E] = (int64_t)(kh - kl) * kChunk * 4 >= kalive ? 1 : 0;
        }
        s_kl = kl;
        s_kh = kh;
        s_off = off;
        if (count) gadd(reinterpret_cast<GLOBAL unsigned long long*>(&I.ctr[C_BLOB_SUM]), (unsigned long long)bytes);
      }
    }
  }
  __syncthreads();
  const int kl = s_kl, kh = s_kh;
  if (kh <= kl) return;
  GLOBAL int8_t* base = I.blob + s_off;
  const int64_t bytes = (int64_t)(kh - kl) * CB;
  const v4i z = {0, 0, 0, 0};
  for (int64_t o = (int64_t)t * 16; o < bytes; o += (int64_t)kRowsThreads * 16) *(v4i*)(base + o) = z;
  __syncthreads();
  const int k0 = kl * kChunk;
  auto set_entry = [&](int lr, int c) {
    const int k = c - k0;
    if (BITS) {
      // lanes of one row may share a word: atomic OR on its 32-bit half
      GLOBAL unsigned* w = reinterpret_cast<GLOBAL unsigned*>(base + ((int64_t)(k >> 6) * kTile + lr) * 8);
      __hip_atomic_fetch_or(w + ((k >> 5) & 1), 1u << (k & 31), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      const int kk = k & (kChunk - 1);
      base[(int64_t)(k >> 6) * kChunkBytes + (lr >> 4) * 1024 + (lr & 15) * 16 + (kk >> 4) * 256 + (kk & 15)] = 1;
    }
  };
#pragma unroll
  for (int pass = 0; pass < NP; ++pass) {
    const int lr = pass * RPP + t / LPR;
    if (tile * kTile + lr >= rows) continue;
#pragma unroll
    for (int i = 0; i < RC; ++i)
      if (col[pass][i] >= 0) set_entry(lr, col[pass][i]);
    if (spill[pass]) {
      // a spilled list is not partitioned yet: its range is unchanged
      spill_entries<VERTEX, LPR>(I, ra[pass] + sub + (int64_t)RC * LPR, rb[pass], [&](int c, int) {
        if (c >= 0) set_entry(lr, c);
      });
    }
  }
  if (VERTEX) {
    // Lists longer than the cache are compacted to their alive entries
    // now, in place and in order (the row group walks the list 4 x LPR
    // entries at a time; each alive entry moves to a position at or before
    // the one it was read from, in a step whose loads all precede its
    // stores), so later rounds scan only what is alive and usually fit the
    // cache.  Deleted entries are not kept: deletions are final.
#pragma unroll
    for (int pass = 0; pass < NP; ++pass) {
      if (!gspill[pass]) continue;
      const int64_t a = ra[pass], b = rb[pass];
      int w = 0;
      for (int64_t q0 = a; q0 < b; q0 += 4 * LPR) {
        int key[4], al[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int64_t p = q0 + u * LPR + sub;
          key[u] = p < b ? I.vedg[p] : -1;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          al[u] = 0;
          if (key[u] >= 0) al[u] = I.ecol[key[u]] >= 0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int pos = w + group_exscan<LPR>(al[u]);
          if (al[u]) I.vedg[a + pos] = key[u];
          w += group_sum<LPR>(al[u]);
        }
      }
      if (sub == 0) I.vend[rowid[pass]] = (int32_t)(a + w);
    }
  }
}

// Persistent over the phase's alive dense tiles (prefix `ap` over the
// instances); the workgroup finishes one tile before taking the next.
template <bool VERTEX, bool BITS>
__global__ __launch_bounds__(kRowsThreads) void k_rows_encode(const DInst* __restrict__ insts, int ninst, const int32_t* ap, int count) {
  __shared__ int32_t s_pf[kPrefLds];
  const int32_t* pf = cache_prefix(ap, ninst, s_pf);
  int64_t w0, end;
  int st;
  xcd_share(pf[ninst], ninst > 1, &w0, &end, &st);
  for (int w = (int)w0; w < end; w += st) {
    const int x = unit_owner(pf, ninst, w);
    const KInst I = kview(insts[x]);   // by value: fields load once, ahead of their uses
    rows_tile<VERTEX, BITS>(I, w - pf[x], count);
    __syncthreads();
  }
}

// ------------------------------------------------------- epilogue test
// The phase's test on one pair (row i, column j, i != j) with intersection
// count x; `col` collects the verdict on j, `row` the one on i (the mirrored
// pair, off-diagonal tiles only).
//  DP (Algorithm 1): D_ij = [f_i + x >= f_j + s_i], i.e. f(e_i) - |e_i \ e_j| >= f(e_j);
//                    e_j is deleted if D_ij and (not D_ji or id_i < id_j).
//  MD (Algorithm 2): dom_ij = [x == d_j] and ([x != d_i] or id_i < id_j);
//                    C_j counts the dominators.
//  SE (superedge rule, Section 3.1, in place of DP when rule_se is set):
//                    D_ij = [x == s_i] and f_i >= f_j (e_i a subset of e_j),
//                    with the same tie break.
template <bool VERTEX>
__device__ __forceinline__ void pair_test(int x, int s_i, int f_i, int id_i, int s_j, int f_j, int id_j,
                                          bool diag, bool se, int& col, int& row) {
  if (!VERTEX) {
    const bool dij = se ? (x == s_i && f_i >= f_j) : (f_i + x >= f_j + s_i);
    const bool dji = se ? (x == s_j && f_j >= f_i) : (f_j + x >= f_i + s_j);
    if (dij && (!dji || id_i < id_j)) col = 1;
    if (!diag && dji && (!dij || id_j < id_i)) row = 1;
  } else {
    col += (x == s_j && (x != s_i || id_i < id_j)) ? 1 : 0;
    if (!diag) row += (x == s_i && (x != s_j || id_j < id_i)) ? 1 : 0;
  }
}

// ------------------------------------------------ tile-pair candidates
// A phase contracts every pair of dense tiles (I, J), J >= I, of an
// instance whose K windows [tkl, tkh) overlap, over the common chunks.  The
// contraction enumerates the candidates itself.  With T tiles, candidate
// number u T - u (u - 1) / 2 + v (0 <= v < T - u) is
//  - pair (v, v + u), diagonal by diagonal, when the windows are narrow
//    (banded instances, where only the first diagonals overlap: they are
//    the first candidates and spread over the whole grid), or
//  - pair (u, u + v), row by row, when tile 0's window spans a quarter of K
//    or more (C_WIDE_E / C_WIDE_V, set by the rows kernel): the workgroups
//    running together then share row tile u, whose operand chunks come from
//    cache, and the contraction streams the other operand only.
// A set numbers its instances' candidates one after the other through the
// prefix of their counts T (T + 1) / 2 (AP_EP / AP_VP, recounted at every
// round end).  Workgroup b of a grid of G examines candidates b, b + G,
// b + 2G, ..., one per thread and blockDim at a time, collects the
// overlapping pairs in LDS and computes them one after the other.
constexpr int kPairThreads = 256;     // workgroup size of every contraction kernel

// First candidate of diagonal / row u.
__device__ __forceinline__ int64_t line_start(int64_t u, int T) { return u * T - u * (u - 1) / 2; }

// Candidate q (0 <= q < T (T + 1) / 2) of an instance with T tiles -> its
// line u and place v on it.
__device__ __forceinline__ void pair_decode(int64_t q, int T, int* u, int* v) {
  // u is the largest with line_start(u) <= q: the smaller root of
  // u^2 - (2T + 1) u + 2q = 0, rounded down, then corrected by one step
  // either way for rounding
  const double b = 2.0 * T + 1.0;
  int i = (int)((b - sqrt(b * b - 8.0 * (double)q)) * 0.5);
  i = max(0, min(i, T - 1));
  if (i + 1 < T && line_start(i + 1, T) <= q) ++i;
  if (i > 0 && line_start(i, T) > q) --i;
  *u = i;
  *v = (int)(q - line_start(i, T));
}

// Alive rows of the phase (0 for an instance that is done, failed or uses
// sparse counts).  The four words load together: no branch between them.
template <bool VERTEX>
__device__ __forceinline__ int phase_rows(const KInst& I) {
  const GLOBAL int32_t* c = I.ctr;
  const int done = c[C_DONE], err = c[C_ERR], rows = VERTEX ? c[C_NA] : c[C_MA];
  return (done | err | (I.variant == 3)) ? 0 : rows;
}

// Examine candidate q of instance x (numbered over T tiles); an overlapping
// pair of alive tiles (both below `alive_tiles`) goes to the LDS list.  The
// windows of both readings of q load at once, before the order flag and the
// alive count arrive.
template <bool VERTEX>
__device__ __forceinline__ void collect_pair(const KInst& I, int x, int64_t q, int T, int alive_tiles, int count,
                                             int* s_n, int4* s_it, int* s_ix) {
  int u, v;
  pair_decode(q, T, &u, &v);
  const int wide = I.ctr[VERTEX ? C_WIDE_V : C_WIDE_E];
  // diagonal reading (v, u + v), row reading (u, u + v): J is u + v in both
  const int tj = u + v;
  const int kl_d = I.tkl[v], kh_d = I.tkh[v], kl_r = I.tkl[u], kh_r = I.tkh[u];
  const int klj = I.tkl[tj], khj = I.tkh[tj];
  const int ti = wide ? u : v;
  const int lo = max(wide ? kl_r : kl_d, klj), hi = min(wide ? kh_r : kh_d, khj);
  if (tj >= alive_tiles || lo >= hi) return;
  const int k = atomicAdd(s_n, 1);
  s_it[k] = make_int4(ti, tj, lo, hi);
  s_ix[k] = x;
  if (count)
    gadd(reinterpret_cast<GLOBAL unsigned long long*>(&I.ctr[VERTEX ? C_CHUNKS_SUM_V : C_CHUNKS_SUM_E]),
              (unsigned long long)(hi - lo));
}

// Persistent loop of a contraction kernel: body(I, TI, TJ, c0, c1, rows)
// runs for every overlapping pair, the whole workgroup together, with a
// barrier after each (rows: the phase's alive rows of that instance).
//  - A set of one numbers its candidates over the tiles it had when
//    prepared (a fixed count, known without reading device state), so the
//    window loads need not wait for the alive count; pairs beyond the alive
//    tiles are dropped.  Its descriptor loads once.
//  - A set numbers them over the alive tiles through `pp`, the prefix of the
//    instances' counts recounted at every round end.
// `count` adds the pairs' chunks to the work counters (profiled runs: the
// atomics stay off the timed path otherwise).
template <bool VERTEX, typename F>
__device__ __forceinline__ void for_each_pair(const DInst* insts, int ninst, const int32_t* pp, int count,
                                              F&& body) {
  __shared__ int32_t s_pref[kPrefLds];
  __shared__ int4 s_it[kPairThreads];
  __shared__ int s_ix[kPairThreads];
  __shared__ int s_n;
  const int64_t step = (int64_t)gridDim.x * kPairThreads;
  if (ninst == 1) {
    const KInst I = kview(insts[0]);
    const int T = ((VERTEX ? I.n : I.m) + kTile - 1) / kTile;
    const int64_t total = (int64_t)T * (T + 1) / 2;
    const int rows = phase_rows<VERTEX>(I);
    const int alive_tiles = (rows + kTile - 1) / kTile;
    // every pair of alive tiles lies on the first alive_tiles lines (rows or
    // diagonals); the first batch does not wait for that bound
    const int64_t bound = line_start(alive_tiles, T);
    for (int64_t first = blockIdx.x; first < total && (first == blockIdx.x || first < bound); first += step) {
      if (threadIdx.x == 0) s_n = 0;
      __syncthreads();
      const int64_t q = first + (int64_t)threadIdx.x * gridDim.x;
      if (q < total) collect_pair<VERTEX>(I, 0, q, T, alive_tiles, count, &s_n, s_it, s_ix);
      __syncthreads();
      const int n = s_n;
      for (int k = 0; k < n; ++k) {
        const int4 w = s_it[k];
        body(I, w.x, w.y, w.z, w.w, rows);
        __syncthreads();
      }
    }
    return;
  }
  const int32_t* pf = cache_prefix(pp, ninst, s_pref);
  int64_t f0, end;
  int st;
  xcd_share(pf[ninst], true, &f0, &end, &st);
  for (int64_t first = f0; first < end; first += (int64_t)st * kPairThreads) {
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    const int64_t p = first + (int64_t)threadIdx.x * st;
    if (p < end) {
      const int x = find_owner(pf, ninst, (int)p);
      const KInst I = kview(insts[x]);   // per thread: only the fields it needs load
      const int at = (phase_rows<VERTEX>(I) + kTile - 1) / kTile;
      const int64_t q = p - pf[x];
      // (q beyond the count only for an instance that stopped this round)
      if (q < (int64_t)at * (at + 1) / 2) collect_pair<VERTEX>(I, x, q, at, at, count, &s_n, s_it, s_ix);
    }
    __syncthreads();
    const int n = s_n;
    for (int k = 0; k < n; ++k) {
      const int4 w = s_it[k];
      const KInst I = kview(insts[__builtin_amdgcn_readfirstlane(s_ix[k])]);
      body(I, w.x, w.y, w.z, w.w, phase_rows<VERTEX>(I));
      __syncthreads();
    }
  }
}

// Epilogue parameters of an item's row tile TI (threads 0..127) and column
// tile TJ (threads 128..255): size or degree (-1 beyond the alive rows),
// demand or largest demand, original id.  Loaded with the operands, kept in
// LDS at [0, 128) for rows and [128, 256) for columns.
__device__ __forceinline__ int3 load_params(const KInst& I, int rows, int TI, int TJ) {
  const int t = threadIdx.x;
  const int g = (t < kTile ? TI : TJ) * kTile + (t & (kTile - 1));
  return g < rows ? make_int3(I.rs[g], I.rf[g], I.rid[g]) : make_int3(-1, 0, 0);
}

struct EpiParams {
  int s[2 * kTile], f[2 * kTile], id[2 * kTile];
};

__device__ __forceinline__ void store_params(EpiParams& P, int3 v) {
  const int t = threadIdx.x;
  if (t < 2 * kTile) { P.s[t] = v.x; P.f[t] = v.y; P.id[t] = v.z; }
}

// Flush the per-tile verdicts collected in LDS to global memory (kill
// flags or dominator counts) and clear them for the next item.
// Verdicts on rows beyond the alive rows are dropped.
template <bool VERTEX>
__device__ __forceinline__ void flush_tile(const KInst& I, int TI, int TJ, int rows, int* s_col, int* s_row) {
  const int tid = threadIdx.x;
  if (tid < kTile) {
    const int v = s_col[tid];
    if (v) {
      const int g = TJ * kTile + tid;
      if (g < rows) {
        if (!VERTEX) I.kill[g] = 1;
        else gadd(&I.cnt[g], v);
      }
      s_col[tid] = 0;
    }
  } else if (tid < 2 * kTile) {
    const int t = tid - kTile;
    const int v = s_row[t];
    if (v) {
      const int g = TI * kTile + t;
      if (g < rows) {
        if (!VERTEX) I.kill[g] = 1;
        else gadd(&I.cnt[g], v);
      }
      s_row[t] = 0;
    }
  }
}

// ---------------------------------------------------- fused contraction
// Epilogue parameters of the MFMA kernels, one int4 {s, f, id, a} per row
// of the item's row tile ([0, 128)) and column tile ([128, 256)): size or
// degree, demand or largest demand, original id, and a = s - f (DP).  Rows
// beyond the alive rows get values that make every test with them false for
// the alive rows, so the tests need no validity branch (DP: a = f = kBig,
// beyond any count; SE: s = kBig; MD: s = 0 and id = INT32_MAX, so a count of 0
// meets no degree of an alive vertex and no tie break); their own verdicts
// are dropped by flush_tile.  Requires counts below kBig.
constexpr int kBig = 1 << 29;

struct MfmaParams {
  int4 p[2 * kTile];
};

template <bool VERTEX>
__device__ __forceinline__ void store_mfma_params(MfmaParams& P, int3 v, bool se) {
  const int t = threadIdx.x;
  if (t >= 2 * kTile) return;
  int4 r;
  if (v.x >= 0) r = make_int4(v.x, v.y, v.z, v.x - v.y);
  else if (VERTEX) r = make_int4(0, 0, INT32_MAX, 0);
  else if (se) r = make_int4(kBig, 0, 0, 0);
  else r = make_int4(0, kBig, 0, kBig);
  P.p[t] = r;
}

// Lane masks (0 or -1) from the sign of a difference, shifted in an asm
// statement the compiler does not see through, so they stay vector integers:
// as comparisons they would become 64-bit scalar lane masks, which the 64
// tests of a lane keep live in numbers that spill.  Operands differ by less
// than 2^31.
__device__ __forceinline__ int m_lt(int a, int b) {
  const int d = (int)((unsigned)a - (unsigned)b);
  int r;
  asm("v_ashrrev_i32 %0, 31, %1" : "=v"(r) : "v"(d));
  return r;
}
__device__ __forceinline__ int m_ge(int a, int b) { return ~m_lt(a, b); }
__device__ __forceinline__ int m_eq(int a, int b) { return m_ge(a, b) & m_ge(b, a); }

// One pair's verdicts as masks (0 / -1) from its count x and the packed
// parameters of the row (rp) and column (cp) it joins: c on the column, r on
// the row.  RULE 0: DP, 1: SE, 2: MD.
template <int RULE>
__device__ __forceinline__ void pair_rule(int x, const int4& rp, const int4& cp, int& c, int& r) {
  const int lt = m_lt(rp.z, cp.z);
  int dij, dji;
  if (RULE == 2) {
    dij = m_eq(x, cp.x);   // (column j's test: x == d_j)
    dji = m_eq(x, rp.x);
  } else if (RULE == 1) {
    dij = m_eq(x, rp.x) & m_ge(rp.y, cp.y);
    dji = m_eq(x, cp.x) & m_ge(cp.y, rp.y);
  } else {
    dij = m_ge(x, rp.w + cp.y);
    dji = m_ge(x, cp.w + rp.y);
  }
  c = dij & (~dji | lt);
  r = dji & (~dij | ~lt);
}

// The phase's test on the 64 x 64 block of one wave of an MFMA tile pair
// (accumulator layout of v_mfma_i32_16x16x64_i8: lane l holds rows
// 4*(l/16)..+3 of column l%16 of each 16 x 16 block), as straight-line
// integer arithmetic on the counts x (the same tests as pair_test):
//  DP: D_ij = [x >= a_i + f_j]   (f_i + x >= f_j + s_i)
//  SE: D_ij = [x == s_i] and f_i >= f_j
//      column j gets D_ij and (not D_ji or id_i < id_j); row i the mirror
//  MD: column j gets [x == s_j] and ([x != s_i] or id_i < id_j); row i the mirror
// Verdicts are summed as integers (a flag is a nonzero sum).  A diagonal tile (TI == TJ) holds
// both orders of every pair: only column verdicts are taken there, and the
// self pair is masked.  Verdicts collect in s_col / s_row for flush_tile.
template <bool VERTEX, int RULE>
__device__ __forceinline__ void mfma_epilogue_rule(int TI, int TJ, const v4i (&acc)[4][4], const MfmaParams& P,
                                                   int* s_col, int* s_row, int wr, int wc, int lane) {
  const int offd = TI != TJ ? -1 : 0;
  // the self pair of a diagonal tile: block i == j, element q == selfq
  const int selfq = (TI == TJ && wr == wc) ? (lane & 15) - (lane >> 4) * 4 : -1;
  int4 cp[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) cp[j] = P.p[kTile + wc * 64 + j * 16 + (lane & 15)];
  int colacc[4] = {0, 0, 0, 0};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int lr = wr * 64 + i * 16 + (lane >> 4) * 4 + q;
      const int4 rp = P.p[lr];
      const int okd = ~m_eq(q, selfq);   // for the block i == j
      int rowacc = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        int c, r;
        pair_rule<RULE>(acc[i][j][q], rp, cp[j], c, r);
        if (i == j) {
          c &= okd;
          r &= okd;
        }
        colacc[j] -= c;          // masks are -1: subtracting counts them
        rowacc -= r & offd;
      }
      if (rowacc) {
        if (!VERTEX) s_row[lr] = 1;
        else atomicAdd(&s_row[lr], rowacc);
      }
      // one row of tests at a time: left to itself the scheduler hoists the
      // tests of all 64 pairs and runs out of registers
      __builtin_amdgcn_sched_barrier(0);
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (!colacc[j]) continue;
    const int lc = wc * 64 + j * 16 + (lane & 15);
    if (!VERTEX) s_col[lc] = 1;
    else atomicAdd(&s_col[lc], colacc[j]);
  }
}

// SE: the edge-phase kernels are instantiated per rule (a set applies one
// rule), so each holds the registers of one test only.
template <bool VERTEX, bool SE>
__device__ __forceinline__ void mfma_epilogue(int TI, int TJ, const v4i (&acc)[4][4], const MfmaParams& P,
                                              int* s_col, int* s_row, int wr, int wc, int lane) {
  mfma_epilogue_rule<VERTEX, VERTEX ? 2 : (SE ? 1 : 0)>(TI, TJ, acc, P, s_col, s_row, wr, wc, lane);
}

// Persistent over the overlapping tile pairs (for_each_pair); for each
// pair (I, J) it computes the 128 x 128 block X = A_I A_J^T over the common K chunks with
// v_mfma_i32_16x16x64_i8 (4 waves of 64 x 64, 4 x 4 MFMA blocks per wave),
// then applies the phase's test to X in registers; X never leaves them.
//  DP (Algorithm 1):  D_ij = [f_i + X_ij >= f_j + s_i], i.e.
//                     f(e_i) - (|e_i| - |e_i & e_j|) >= f(e_j);
//                     e_j deleted if D_ij and (not D_ji or id_i < id_j), i != j
//  MD (Algorithm 2):  dom_ij = [X_ij == d_j] and ([X_ij != d_i] or id_i < id_j),
//                     i != j;  C_j += dom_ij
// Accumulator layout of the 16x16 MFMA: lane l holds rows 4*(l/16)..+3 of
// column l%16.
template <bool VERTEX, bool SE>
__global__ __launch_bounds__(kPairThreads, 2) void k_gemm(const DInst* __restrict__ insts, int ninst, const int32_t* pp, int count) {
  __shared__ int s_col[kTile];
  __shared__ int s_row[kTile];
  __shared__ MfmaParams s_par;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = tid >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  if (tid < kTile) { s_col[tid] = 0; s_row[tid] = 0; }
  for_each_pair<VERTEX>(insts, ninst, pp, count, [&](const KInst& I, int TI, int TJ, int c0, int c1, int rows) {
    const int3 par = load_params(I, rows, TI, TJ);
    const GLOBAL int8_t* pa = I.blob + chunk_offset<VERTEX, kChunkBytes>(I, TI, c0) + (wr * 4) * 1024 + lane * 16;
    const GLOBAL int8_t* pb = I.blob + chunk_offset<VERTEX, kChunkBytes>(I, TJ, c0) + (wc * 4) * 1024 + lane * 16;
    v4i acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = v4i{0, 0, 0, 0};
    v4i a[4], b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) { a[i] = *(const v4i*)(pa + i * 1024); b[i] = *(const v4i*)(pb + i * 1024); }
    store_mfma_params<VERTEX>(s_par, par, SE);
    for (int c = c0; c < c1; ++c) {
      v4i an[4], bn[4];
      const bool more = c + 1 < c1;
      if (more) {
        pa += kChunkBytes;
        pb += kChunkBytes;
#pragma unroll
        for (int i = 0; i < 4; ++i) { an[i] = *(const v4i*)(pa + i * 1024); bn[i] = *(const v4i*)(pb + i * 1024); }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[i], b[j], acc[i][j], 0, 0, 0);
      if (more) {
#pragma unroll
        for (int i = 0; i < 4; ++i) { a[i] = an[i]; b[i] = bn[i]; }
      }
    }
    __syncthreads();   // staged epilogue parameters
    // ---- epilogue: the phase's test on the 64 x 64 block of this wave
    mfma_epilogue<VERTEX, SE>(TI, TJ, acc, s_par, s_col, s_row, wr, wc, lane);
    __syncthreads();
    flush_tile<VERTEX>(I, TI, TJ, rows, s_col, s_row);
  });
}

// LDS-staged form of k_gemm: the workgroup copies each K chunk of both tiles
// (8 KiB each, already in operand order) into LDS once, so every fragment is
// fetched from L2 once per workgroup instead of once per wave; the next
// chunk is prefetched into registers while the MFMAs run on the current one
// (two LDS stages, one barrier per chunk).
template <bool VERTEX, bool SE>
__global__ __launch_bounds__(kPairThreads, 2) void k_gemm_lds(const DInst* __restrict__ insts, int ninst, const int32_t* pp, int count) {
  __shared__ int s_col[kTile];
  __shared__ int s_row[kTile];
  __shared__ MfmaParams s_par;
  __shared__ v4i sA[2][512];
  __shared__ v4i sB[2][512];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = tid >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  if (tid < kTile) { s_col[tid] = 0; s_row[tid] = 0; }
  for_each_pair<VERTEX>(insts, ninst, pp, count, [&](const KInst& I, int TI, int TJ, int c0, int c1, int rows) {
    const int3 par = load_params(I, rows, TI, TJ);
    const GLOBAL v4i* ga = reinterpret_cast<const GLOBAL v4i*>(I.blob + chunk_offset<VERTEX, kChunkBytes>(I, TI, c0));
    const GLOBAL v4i* gb = reinterpret_cast<const GLOBAL v4i*>(I.blob + chunk_offset<VERTEX, kChunkBytes>(I, TJ, c0));
    v4i ra0 = ga[tid], ra1 = ga[tid + 256], rb0 = gb[tid], rb1 = gb[tid + 256];
    sA[0][tid] = ra0; sA[0][tid + 256] = ra1;
    sB[0][tid] = rb0; sB[0][tid + 256] = rb1;
    store_mfma_params<VERTEX>(s_par, par, SE);
    __syncthreads();
    v4i acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = v4i{0, 0, 0, 0};
    for (int c = c0; c < c1; ++c) {
      const int st = (c - c0) & 1;
      const bool more = c + 1 < c1;
      if (more) {
        ga += 512;
        gb += 512;
        ra0 = ga[tid]; ra1 = ga[tid + 256];
        rb0 = gb[tid]; rb1 = gb[tid + 256];
      }
      v4i a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        a[i] = sA[st][(wr * 4 + i) * 64 + lane];
        b[i] = sB[st][(wc * 4 + i) * 64 + lane];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[i], b[j], acc[i][j], 0, 0, 0);
      if (more) {
        sA[st ^ 1][tid] = ra0; sA[st ^ 1][tid + 256] = ra1;
        sB[st ^ 1][tid] = rb0; sB[st ^ 1][tid + 256] = rb1;
      }
      __syncthreads();
    }
    mfma_epilogue<VERTEX, SE>(TI, TJ, acc, s_par, s_col, s_row, wr, wc, lane);
    __syncthreads();
    flush_tile<VERTEX>(I, TI, TJ, rows, s_col, s_row);
  });
}

// Asynchronous-copy form of k_gemm_lds: operand chunks go from global memory
// straight into LDS (global_load_lds_dwordx4, no register staging) through a
// ring of kAsyncStages stages, so up to kAsyncStages - 1 chunks are in flight
// while the MFMAs run on the current one.  Each thread issues four 16-byte
// copies per chunk (two per operand); a wave's 64 copies fill one 1 KiB
// fragment block, which is exactly the operand order in the blob.
constexpr int kAsyncStages = 4;

__device__ __forceinline__ void copy_to_lds(const GLOBAL v4i* src, v4i* dst_wave_base) {
  __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1)))*)src,
                                   (void __attribute__((address_space(3)))*)dst_wave_base, 16, 0, 0);
}

// Waits until at most n of this thread's vector-memory operations are in
// flight (n <= 12 here; exp and lgkm counters not waited on).
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 16, "vmcnt field");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8));
}

template <bool VERTEX, bool SE>
__global__ __launch_bounds__(kPairThreads, 2) void k_gemm_async(const DInst* __restrict__ insts, int ninst, const int32_t* pp, int count) {
  __shared__ int s_col[kTile];
  __shared__ int s_row[kTile];
  __shared__ MfmaParams s_par;
  __shared__ v4i sA[kAsyncStages][512];
  __shared__ v4i sB[kAsyncStages][512];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = tid >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  if (tid < kTile) { s_col[tid] = 0; s_row[tid] = 0; }
  for_each_pair<VERTEX>(insts, ninst, pp, count, [&](const KInst& I, int TI, int TJ, int c0, int c1, int rows) {
    const int3 par = load_params(I, rows, TI, TJ);
    const GLOBAL v4i* ga = reinterpret_cast<const GLOBAL v4i*>(I.blob + chunk_offset<VERTEX, kChunkBytes>(I, TI, c0));
    const GLOBAL v4i* gb = reinterpret_cast<const GLOBAL v4i*>(I.blob + chunk_offset<VERTEX, kChunkBytes>(I, TJ, c0));
    // chunk k of the item (0-based) into stage k % kAsyncStages
    auto issue = [&](int k) {
      const int st = k % kAsyncStages;
      const GLOBAL v4i* a = ga + (int64_t)k * 512;
      const GLOBAL v4i* b = gb + (int64_t)k * 512;
      copy_to_lds(a + tid, &sA[st][wid * 64]);
      copy_to_lds(a + tid + 256, &sA[st][256 + wid * 64]);
      copy_to_lds(b + tid, &sB[st][wid * 64]);
      copy_to_lds(b + tid + 256, &sB[st][256 + wid * 64]);
    };
    const int nk = c1 - c0;
#pragma unroll
    for (int k = 0; k < kAsyncStages - 1; ++k)
      if (k < nk) issue(k);
    store_mfma_params<VERTEX>(s_par, par, SE);
    v4i acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = v4i{0, 0, 0, 0};
    for (int k = 0; k < nk; ++k) {
      if (k + kAsyncStages - 1 < nk) issue(k + kAsyncStages - 1);
      // chunks issued after chunk k may stay in flight (4 copies each)
      const int after = __builtin_amdgcn_readfirstlane(min(kAsyncStages - 1, nk - 1 - k));
      if (after >= 3) wait_vm<12>();
      else if (after == 2) wait_vm<8>();
      else if (after == 1) wait_vm<4>();
      else wait_vm<0>();
      // every thread's copies of chunk k have landed; a plain barrier (no
      // memory fence, which would wait for the later chunks too) publishes them
      __builtin_amdgcn_s_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");   // LDS reads stay below the barrier
      const int st = k % kAsyncStages;
      v4i a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        a[i] = sA[st][(wr * 4 + i) * 64 + lane];
        b[i] = sB[st][(wc * 4 + i) * 64 + lane];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[i], b[j], acc[i][j], 0, 0, 0);
      // every wave has read stage st (its fragments are in registers) before
      // the next iteration refills the stage of chunk k - 1... k + 3
      __builtin_amdgcn_s_waitcnt((15 & 15) | (7 << 4) | (0 << 8));   // lgkmcnt(0): LDS reads done
      __builtin_amdgcn_s_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");   // copies stay below the barrier
    }
    mfma_epilogue<VERTEX, SE>(TI, TJ, acc, s_par, s_col, s_row, wr, wc, lane);
    __syncthreads();
    flush_tile<VERTEX>(I, TI, TJ, rows, s_col, s_row);
  });
}

// Bitset variant: X_ij = sum over 64-bit chunks of popcount(a_i & b_j) on
// the vector ALU.  Each thread owns an 8 x 8 block of the 128 x 128 tile
// pair; up to kStage chunks of both tiles are staged in LDS (rows padded by
// one word per 8 so the 16 column groups of a wave hit distinct banks).
constexpr int kStage = 16;
constexpr int kPadRows = kTile + kTile / 8;
__device__ __forceinline__ int pad_row(int p) { return p + (p >> 3); }

template <bool VERTEX>
__global__ __launch_bounds__(kPairThreads) void k_gemm_bits(const DInst* __restrict__ insts, int ninst, const int32_t* pp, int count) {
  __shared__ int s_col[kTile];
  __shared__ int s_row[kTile];
  __shared__ EpiParams s_par;
  __shared__ uint64_t sa[kStage * kPadRows];
  __shared__ uint64_t sb[kStage * kPadRows];
  const int tid = threadIdx.x;
  const int ty = tid >> 4, tx = tid & 15;
  if (tid < kTile) { s_col[tid] = 0; s_row[tid] = 0; }
  for_each_pair<VERTEX>(insts, ninst, pp, count, [&](const KInst& I, int TI, int TJ, int c0, int c1, int rows) {
    const int3 par = load_params(I, rows, TI, TJ);
    const GLOBAL uint64_t* A = reinterpret_cast<const GLOBAL uint64_t*>(I.blob + chunk_offset<VERTEX, kChunkBytesBits>(I, TI, c0));
    const GLOBAL uint64_t* B = reinterpret_cast<const GLOBAL uint64_t*>(I.blob + chunk_offset<VERTEX, kChunkBytesBits>(I, TJ, c0));
    int acc[8][8];
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[r][q] = 0;
    store_params(s_par, par);   // ordered before the epilogue by the staging barriers
    for (int c = c0; c < c1; c += kStage) {
      const int ns = min(kStage, c1 - c);
      for (int wv = tid; wv < ns * kTile; wv += 256) {
        const int ch = wv >> 7, row = wv & (kTile - 1);
        sa[ch * kPadRows + pad_row(row)] = A[wv];
        sb[ch * kPadRows + pad_row(row)] = B[wv];
      }
      __syncthreads();
      for (int st = 0; st < ns; ++st) {
        uint64_t a[8], b[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          a[r] = sa[st * kPadRows + pad_row(ty * 8 + r)];
          b[r] = sb[st * kPadRows + pad_row(tx * 8 + r)];
        }
#pragma unroll
        for (int r = 0; r < 8; ++r)
#pragma unroll
          for (int q = 0; q < 8; ++q) acc[r][q] += __popcll(a[r] & b[q]);
      }
      __syncthreads();
      A += (int64_t)ns * kTile;
      B += (int64_t)ns * kTile;
    }
    const bool diag = TI == TJ;
    int cs[8], cf[8], cid[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int lc = kTile + tx * 8 + q;
      cs[q] = s_par.s[lc];
      cf[q] = s_par.f[lc];
      cid[q] = s_par.id[lc];
    }
    int colacc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int lr = ty * 8 + r;
      const int rs_ = s_par.s[lr];
      if (rs_ < 0) continue;
      const int rf_ = s_par.f[lr], rid_ = s_par.id[lr];
      int rowacc = 0;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int lc = tx * 8 + q;
        if (cs[q] < 0 || (diag && lr == lc)) continue;
        pair_test<VERTEX>(acc[r][q], rs_, rf_, rid_, cs[q], cf[q], cid[q], diag, I.rule_se != 0, colacc[q], rowacc);
      }
      if (rowacc) {
        if (!VERTEX) s_row[lr] = 1;
        else atomicAdd(&s_row[lr], rowacc);
      }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (!colacc[q]) continue;
      const int lc = tx * 8 + q;
      if (!VERTEX) s_col[lc] = 1;
      else atomicAdd(&s_col[lc], colacc[q]);
    }
    __syncthreads();
    flush_tile<VERTEX>(I, TI, TJ, rows, s_col, s_row);
  });
}

// ------------------------------------------------------ sparse variant
// Variant 3: the nonzero entries of row j of A A^T (edge phase) or of A^T A
// (vertex phase) only.  One wave per victim j enumerates the product terms
// -- for every alive vertex v of e_j every alive hyperedge containing v, or
// for every alive hyperedge e of v_j every alive vertex of e -- counts them
// per partner in an LDS hash table, and applies the same DP / MD test as the
// dense epilogue to every partner with a nonzero count (a zero count never
// passes either test, see the layout notes at the top).  When the terms
// exceed half the table they are split over passes by a hash of the partner
// id; if a pass still overflows, the victim is recounted over dense ranges
// of partner ids, which cannot overflow.
__device__ __forceinline__ unsigned hmix(unsigned x) {
  x ^= x >> 16;
  x *= 0x7feb352dU;
  x ^= x >> 15;
  x *= 0x846ca68bU;
  x ^= x >> 16;
  return x;
}

// Per compact row: alive size / degree by original id (the partner tests
// need them for every partner), epilogue parameters, cleared flags; vertex
// rows shorten their hyperedge list [vptr[v], vend[v]) to the alive ones.
template <bool VERTEX>
__device__ void sp_rows_block(const KInst& I, int blk) {
  if (inst_idle(I.ctr) || !is_sparse(I)) return;
  const int rows = VERTEX ? I.ctr[C_NA] : I.ctr[C_MA];
  const int r = blk * kBlock + threadIdx.x;
  if (r >= rows) return;
  const int cur = I.ctr[VERTEX ? C_NCOMP_V : C_NCOMP_E] & 1;
  if (!VERTEX) {
    const int e = erow_list(I, cur)[r];
    int sz = 0;
    // alive size, eight entries at a time with their loads issued together
    const int pa = (int)I.eptr[e], pq = (int)I.eptr[e + 1];
    for (int p0 = pa; p0 < pq; p0 += 8) {
      int vv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) vv[u] = I.evtx[min(p0 + u, pq - 1)];
#pragma unroll
      for (int u = 0; u < 8; ++u) sz += (p0 + u < pq && I.vcol[vv[u]] >= 0) ? 1 : 0;
    }
    const int fe = I.fw[e];
    I.esz[e] = sz;
    I.eslk[e] = (uint8_t)min(sz - fe, 254);
    I.rs[r] = sz;
    I.rf[r] = fe;
    I.rid[r] = e;
  } else {
    const int v = vrow_list(I, cur)[r];
    int d = 0, mf = 0;
    // keep only the alive hyperedges of v at the front of its list, eight
    // entries at a time: a chunk is read whole (its loads issued together,
    // then its hyperedges' states) before its alive entries are written at
    // or before their old positions, so the partition stays in place and a
    // chunk costs two round trips instead of two per entry; deletions are
    // final
    constexpr int C = 8;
    const int a = I.vptr[v], q = I.vend[v];
    for (int p0 = a; p0 < q; p0 += C) {
      int e[C], c[C], f[C];
#pragma unroll
      for (int u = 0; u < C; ++u) e[u] = I.vedg[min(p0 + u, q - 1)];
#pragma unroll
      for (int u = 0; u < C; ++u) {
        c[u] = I.ecol[e[u]];
        f[u] = I.fw[e[u]];
      }
#pragma unroll
      for (int u = 0; u < C; ++u)
        if (p0 + u < q && c[u] >= 0) {
          I.vedg[a + d] = e[u];
          ++d;
          mf = max(mf, f[u]);
        }
    }
    I.vend[v] = a + d;
    I.vdeg[v] = d;
    I.rs[r] = d;
    I.rf[r] = mf;
    I.rid[r] = v;
    I.cnt[r] = 0;
  }
  I.kill[r] = 0;
}

// Persistent over the phase's blocks of kBlock rows (prefix `bp`).
template <bool VERTEX>
__global__ __launch_bounds__(kBlock) void k_sp_rows(const DInst* __restrict__ insts, int ninst, const int32_t* bp) {
  __shared__ int32_t s_pf[kPrefLds];
  const int32_t* pf = cache_prefix(bp, ninst, s_pf);
  int64_t w0, end;
  int st;
  xcd_share(pf[ninst], ninst > 1, &w0, &end, &st);
  for (int w = (int)w0; w < end; w += st) {
    const int x = unit_owner(pf, ninst, w);
    const KInst I = kview(insts[x]);
    sp_rows_block<VERTEX>(I, w - pf[x]);
  }
}

// Outer list of victim j: the alive vertices of e_j (edge phase) or the
// alive hyperedges of v_j (vertex phase); inner list of an outer element:
// the hyperedges containing the vertex, or the vertices of the hyperedge.
// Positions are 32-bit: an instance holds fewer than 2^31 incidences (the
// library rejects more).
template <bool VERTEX>
__device__ __forceinline__ void outer_range(const KInst& I, int j, int* a, int* b) {
  if (!VERTEX) { *a = I.eptr[j]; *b = I.eptr[j + 1]; }
  else { *a = I.vptr[j]; *b = I.vend[j]; }
}
// Edge phase: with cls >= 0 (round 1) the inner list of vertex v ends at
// the end of slack class cls (k_prep_slack), else at the list's end.
template <bool VERTEX>
__device__ __forceinline__ bool outer_elem(const KInst& I, int p, int* ia, int* ib, int cls = -1) {
  if (!VERTEX) {
    const int v = I.evtx[p];
    if (I.vcol[v] < 0) return false;
    *ia = I.vptr[v];
    *ib = cls < 0 ? I.vend[v] : *slack_end(I, v, cls);
  } else {
    const int e = I.vedg[p];
    if (I.ecol[e] < 0) return false;
    *ia = I.eptr[e];
    *ib = I.eptr[e + 1];
  }
  return true;
}
// Partner id at inner position q, or -1 if it is not alive.
template <bool VERTEX>
__device__ __forceinline__ int inner_partner(const KInst& I, int q) {
  if (!VERTEX) {
    const int e = I.vedg[q];
    return I.death_e[e] == 0 ? e : -1;
  }
  const int v = I.evtx[q];
  return I.vcol[v] >= 0 ? v : -1;
}

// Wave-level scans of one int per lane.
__device__ __forceinline__ int wave_exscan(int v, int* total) {
  const int lane = lane_id();
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  *total = __shfl(x, 63, 64);
  return x - v;
}
__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Enumerates the victim's product terms (partner ids; j itself and dead
// partners filtered out) and calls f(partner) for each, the lanes of one
// wave cooperating: outer elements 64 at a time, their inner lists split
// over the lanes through a prefix of their lengths.
template <bool VERTEX, typename F>
__device__ void wave_for_each_term(const KInst& I, int j, int32_t* s_start, int* s_pref, int cls, F f) {
  const int lane = lane_id();
  int oa, ob;
  outer_range<VERTEX>(I, j, &oa, &ob);
  for (int base = oa; base < ob; base += 64) {
    const int p = base + lane;
    int ia = 0, ib = 0;
    if (p < ob && !outer_elem<VERTEX>(I, p, &ia, &ib, cls)) ia = ib = 0;
    const int len = p < ob ? (int)(ib - ia) : 0;
    int tot;
    const int pre = wave_exscan(len, &tot);
    s_start[lane] = (int32_t)ia;
    s_pref[lane] = pre;
    wave_sync();
    for (int t = lane; t < tot; t += 64) {
      int lo = 0, hi = 63;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_pref[mid] <= t) lo = mid; else hi = mid - 1;
      }
      const int partner = inner_partner<VERTEX>(I, s_start[lo] + (t - s_pref[lo]));
      if (partner >= 0 && partner != j) f(partner);
    }
    wave_sync();
  }
}

// The same enumeration with all threads of the block cooperating (outer
// lists 256 elements at a time), for victims with many terms.
template <bool VERTEX, typename F>
__device__ void block_for_each_term(const KInst& I, int j, int32_t* s_start, int* s_pref, int* sh, int cls, F f) {
  int oa, ob;
  outer_range<VERTEX>(I, j, &oa, &ob);
  for (int base = oa; base < ob; base += blockDim.x) {
    const int p = base + threadIdx.x;
    int ia = 0, ib = 0;
    if (p < ob && !outer_elem<VERTEX>(I, p, &ia, &ib, cls)) ia = ib = 0;
    const int len = p < ob ? (int)(ib - ia) : 0;
    int tot;
    const int pre = block_exscan(len, sh, &tot);
    s_start[threadIdx.x] = (int32_t)ia;
    s_pref[threadIdx.x] = pre;
    __syncthreads();
    for (int t = threadIdx.x; t < tot; t += blockDim.x) {
      int lo = 0, hi = (int)blockDim.x - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_pref[mid] <= t) lo = mid; else hi = mid - 1;
      }
      const int partner = inner_partner<VERTEX>(I, s_start[lo] + (t - s_pref[lo]));
      if (partner >= 0 && partner != j) f(partner);
    }
    __syncthreads();
  }
}

// Victim tables hold packed words (partner << cb | count), cb the bit width
// of the victim's alive size s_j: a partner is counted at most once per
// alive outer element, so no count exceeds s_j < 2^cb and none reaches the
// key bits.  A victim packs when its partner ids fit the other 32 - cb bits
// (then no word equals the empty mark); others count over dense ranges.
constexpr unsigned kEmpty = 0xffffffffu;

__device__ __forceinline__ int count_bits(int sj) { return 32 - __clz(max(sj, 1)); }
__device__ __forceinline__ bool packs(int nid, int cb) { return ((uint64_t)nid << cb) < (1ull << 32); }
// Smallest power of two >= x, for x >= 1.
__device__ __forceinline__ int pow2_at_least(int x) { return x <= 1 ? 1 : 1 << (32 - __clz(x - 1)); }

// Adds one term of `partner` to a table of `slots` packed words if the
// partner falls in pass `pass` of `passes`; sets *over if no slot is left.
__device__ __forceinline__ void hash_insert(unsigned* tab, int slots, int cb, int passes, int pass, int partner,
                                            int* over) {
  if (passes > 1 && (int)(hmix((unsigned)partner * 2654435761u) % (unsigned)passes) != pass) return;
  const unsigned key = (unsigned)partner << cb;
  unsigned h = hmix((unsigned)partner) & (unsigned)(slots - 1);
  for (int probe = 0; probe < slots; ++probe) {
    const unsigned prev = atomicCAS(&tab[h], kEmpty, key | 1u);
    if (prev == kEmpty) return;
    if ((prev >> cb) == (unsigned)partner) { atomicAdd(&tab[h], 1u); return; }
    h = (h + 1) & (unsigned)(slots - 1);
  }
  *over = 1;
}

// The terms of a victim whose outer list fits one wave (K <= 64 elements;
// s_start / s_pref hold each element's inner start and the exclusive prefix
// of the inner lengths, tot their sum): U terms per lane per step, each
// found by a search over the prefix and its two dependent loads issued
// together with the others'; f(partner, state) takes each counted term with
// the partner's state as loaded (its slack byte or its compact id).
// Edge phase: partners whose slack |e_i| - f(e_i) exceeds slack_cap are
// skipped (slack 255 marks a deleted hyperedge).  Under DP the victim's own
// slack is passed: X_ij <= s_j, so D_ij (f_i + X_ij >= f_j + s_i) needs
// s_i - f_i <= s_j - f_j, and such a partner cannot delete e_j (either way
// round: D_ji is only asked of partners with D_ij).  Under SE 254 passes
// every alive partner.
template <bool VERTEX, typename F>
__device__ __forceinline__ void wave_terms_one(const KInst& I, int j, int K, int tot, const int32_t* s_start,
                                               const int* s_pref, int slack_cap, F f) {
  constexpr int U = 4;
  const int lane = lane_id();
  const int top = K > 1 ? 1 << (31 - __clz(K - 1)) : 0;
  for (int t0 = 0; t0 < tot; t0 += 64 * U) {
    int lo[U];
#pragma unroll
    for (int u = 0; u < U; ++u) lo[u] = 0;
    for (int step = top; step > 0; step >>= 1) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int t = t0 + u * 64 + lane;
        const int mid = lo[u] + step;
        if (mid < K && s_pref[mid] <= t) lo[u] = mid;
      }
    }
    // every lane issues its U loads of each stage together, unconditionally
    // (position 0, which exists whenever there are terms, stands in for a
    // lane past the end), so the two dependent stages cost two round trips
    int el[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = t0 + u * 64 + lane;
      const int q = t < tot ? s_start[lo[u]] + (t - s_pref[lo[u]]) : 0;
      el[u] = VERTEX ? I.evtx[q] : I.vedg[q];
    }
    int alive[U];
#pragma unroll
    for (int u = 0; u < U; ++u) alive[u] = VERTEX ? I.vcol[el[u]] : (int)I.eslk[el[u]];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool ok = t0 + u * 64 + lane < tot && (VERTEX ? alive[u] >= 0 : alive[u] <= slack_cap);
      el[u] = ok ? el[u] : -1;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (el[u] >= 0 && el[u] != j) f(el[u], alive[u]);
  }
}

// Segments of GL lanes (16 or 32) of a wave: exclusive scan of one int per
// lane, with the segment total.
template <int GL>
__device__ __forceinline__ int group_exscan(int v, int* total) {
  const int gl = lane_id() & (GL - 1);
  int x = v;
#pragma unroll
  for (int o = 1; o < GL; o <<= 1) {
    const int y = __shfl_up(x, o, GL);
    if (gl >= o) x += y;
  }
  *total = __shfl(x, GL - 1, GL);
  return x - v;
}
// The terms of a group victim (K <= GL outer elements; g_start / g_pref
// hold their inner starts and the exclusive prefix of the inner lengths, tot
// their sum), U per lane per step, found by a search over the prefix, the
// loads of each stage issued together (clamped positions stand in for lanes
// past the end), the edge-phase slack filter as in wave_terms_one.  With
// `probe` (a DP victim that any partner of slack 0 deletes, see sp_groups)
// the walk stops after the step that meets such a partner and returns true.
// *visited receives the number of terms walked.
template <bool VERTEX, int GL, typename F>
__device__ __forceinline__ bool group_terms(const KInst& I, int j, int K, int tot, const int32_t* g_start,
                                            const int* g_pref, int slack_cap, bool probe, int* visited, F f) {
  *visited = tot;
  constexpr int U = 4;
  const int gl = lane_id() & (GL - 1);
  const int top = K > 1 ? 1 << (31 - __clz(K - 1)) : 0;
  for (int t0 = 0; t0 < tot; t0 += GL * U) {
    int lo[U];
#pragma unroll
    for (int u = 0; u < U; ++u) lo[u] = 0;
    for (int step = top; step > 0; step >>= 1) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int t = t0 + u * GL + gl;
        const int mid = lo[u] + step;
        if (mid < K && g_pref[mid] <= t) lo[u] = mid;
      }
    }
    int el[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = t0 + u * GL + gl;
      const int q = t < tot ? g_start[lo[u]] + (t - g_pref[lo[u]]) : 0;
      el[u] = VERTEX ? I.evtx[q] : I.vedg[q];
    }
    int alive[U];
#pragma unroll
    for (int u = 0; u < U; ++u) alive[u] = VERTEX ? I.vcol[el[u]] : (int)I.eslk[el[u]];
    int zero = 0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool ok = t0 + u * GL + gl < tot && (VERTEX ? alive[u] >= 0 : alive[u] <= slack_cap);
      if (ok && el[u] != j) {
        f(el[u], alive[u]);
        zero |= (!VERTEX && alive[u] == 0) ? 1 : 0;
      }
    }
    // group-uniform: the loop bound and `probe` are the group's
    if (probe && group_sum<GL>(zero) > 0) {
      *visited = min(tot, t0 + GL * U);
      return true;
    }
  }
  return false;
}

// The test of partner i (count c) against victim j, the partner's size and
// demand (edge phase) or degree (vertex phase) already loaded into pa, pb:
// DP or SE in the edge phase (any partner deletes), MD in the vertex phase
// (the dominators are counted).
template <bool VERTEX>
__device__ __forceinline__ int pair_verdict(const KInst& I, int i, int c, int pa, int pb, int sj, int fj, int j) {
  if (!VERTEX) {
    const int si = pa, fi = pb;
    const bool se = I.rule_se != 0;
    const bool dij = se ? (c == si && fi >= fj) : (fi + c >= fj + si);
    const bool dji = se ? (c == sj && fj >= fi) : (fj + c >= fi + sj);
    return (dij && (!dji || i < j)) ? 1 : 0;
  }
  return (c == sj && (c != pa || i < j)) ? 1 : 0;
}

// Sum of the tests over the occupied slots of a table of S packed words,
// read by lanes li, li + STRIDE, ...: four slots per lane at a time, their
// partners' loads issued together (an empty slot loads the victim's own
// entry, which is cached, and counts nothing; in the vertex phase only
// slots that can count load).
template <bool VERTEX, int STRIDE>
__device__ __forceinline__ int scan_table(const KInst& I, const unsigned* t, int S, int li, int cb, int sj, int fj,
                                          int j) {
  const unsigned cm = (1u << cb) - 1;
  int v = 0;
  for (int h0 = 0; h0 < S; h0 += 4 * STRIDE) {
    unsigned wd[4];
    int pi[4], pa[4], pb[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int h = h0 + u * STRIDE + li;
      wd[u] = h < S ? t[h] : kEmpty;
      pi[u] = wd[u] != kEmpty ? (int)(wd[u] >> cb) : j;
    }
    if (!VERTEX) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        pa[u] = I.esz[pi[u]];
        pb[u] = I.fw[pi[u]];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (wd[u] != kEmpty) v += pair_verdict<VERTEX>(I, pi[u], (int)(wd[u] & cm), pa[u], pb[u], sj, fj, j);
    } else {
      // MD counts a partner only if its count equals d_j (it lies on every
      // alive hyperedge of v_j): only those load the partner's degree, so a
      // wave whose slots hold none skips the round trip
      bool cand[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) cand[u] = wd[u] != kEmpty && (int)(wd[u] & cm) == sj;
#pragma unroll
      for (int u = 0; u < 4; ++u) pa[u] = cand[u] ? I.vdeg[pi[u]] : 0;
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (cand[u]) v += pair_verdict<VERTEX>(I, pi[u], sj, pa[u], 0, sj, fj, j);
    }
  }
  return v;
}

// Slack keys (edge phase under DP): a table word holds (partner << 8 |
// slack) above the count bits, the slack byte as the term loop loaded it
// (min(|e_i| - f(e_i), 254)), when the partner ids leave room for it.  Then
// D_ij (count >= f_j + slack_i) needs no load: a partner with a lower id
// that satisfies it deletes e_j outright.  Only the partners whose slack
// byte is capped (254: not exact) or that satisfy D_ij with a higher id (the
// tie break asks D_ji, which needs f_i) take their size and demand from
// memory, in a second pass that runs only if the first found no deleter.
__device__ __forceinline__ bool packs_slack(int nid, int cb) { return ((uint64_t)nid << (cb + 8)) < (1ull << 32); }

// First pass over a slack-key table (slots li, li + STRIDE, ...): *del
// counts the partners that delete e_j without a load, *need those that
// need one.
template <int STRIDE>
__device__ __forceinline__ void slack_scan(const unsigned* t, int S, int li, int cb, int fj, int j, int* del,
                                           int* need) {
  const unsigned cm = (1u << cb) - 1;
  int d = 0, n = 0;
  for (int h = li; h < S; h += STRIDE) {
    const unsigned wd = t[h];
    if (wd == kEmpty) continue;
    const unsigned key = wd >> cb;
    const int i = (int)(key >> 8), sl = (int)(key & 255u), c = (int)(wd & cm);
    if (sl >= 254) n += 1;
    else if (c >= fj + sl) {
      if (i < j) d += 1;
      else n += 1;
    }
  }
  *del = d;
  *need = n;
}

// Second pass: the exact test of the partners slack_scan could not decide.
template <int STRIDE>
__device__ __forceinline__ int slack_rest(const KInst& I, const unsigned* t, int S, int li, int cb, int sj, int fj,
                                          int j) {
  const unsigned cm = (1u << cb) - 1;
  int v = 0;
  for (int h = li; h < S; h += STRIDE) {
    const unsigned wd = t[h];
    if (wd == kEmpty) continue;
    const unsigned key = wd >> cb;
    const int i = (int)(key >> 8), sl = (int)(key & 255u), c = (int)(wd & cm);
    if (sl >= 254 || (c >= fj + sl && i > j)) v += pair_verdict<false>(I, i, c, I.esz[i], I.fw[i], sj, fj, j);
  }
  return v;
}

// A tile's victims go four ways.  In the edge phase, those with at most 16
// outer elements and kGMaxP product terms are counted four per wave, 16
// lanes each, in tables of up to kWHash / 4 slots; of the others, those
// with at most 32 outer elements and kG2MaxP terms two per wave, 32 lanes
// each, in tables of up to kWHash / 2 slots.  A group victim with P terms
// uses the smallest power of two >= 4P/3 within its region: P stays below
// the region's size, so the table never fills.  Either way one wave keeps
// the dependent loads of several victims in flight.  The rest go to a
// list: those with at most kWHash / 2 terms one per wave (each wave's table
// of kWHash slots), then the others with the whole block and the four
// tables joined (4 kWHash slots, split over passes by partner hash when the
// terms exceed half of them).  A victim whose table does not pack or still
// overflows, or every victim when force_range is set, is counted over dense
// ranges of partner ids, which cannot overflow.  Two table sizes: the small
// one leaves room for more workgroups per CU (batches of small instances),
// the big one takes victims with twice the terms in groups (sets whose
// victims have many terms); the host chooses.
template <bool BIG>
struct SpTables {
  static constexpr int kWHash = BIG ? 2048 : 1024;   // slots of a wave's table
  static constexpr int kGMaxP = BIG ? 320 : 192;     // terms of a 16-lane group victim
  static constexpr int kG2MaxP = BIG ? 736 : 368;    // terms of a 32-lane group victim
  // a group victim has at most that many distinct partners, so its table
  // never fills and never leaves the group's region
  static_assert(kGMaxP < kWHash / 4 && kG2MaxP < kWHash / 2, "group tables must hold every partner");
};

// One sweep of groups of GL lanes (64 / GL victims per wave) over `count`
// victims: rows first, first + 1, ... (list == nullptr) or the rows list[k].
// A victim the groups do not take (vertex phase, more than GL outer
// elements or MAXP terms, a table that does not pack, force_range) goes to
// out[] (*nout counts); an isolated vertex goes nowhere: the compaction
// deletes it.  wtab: this wave's kWHash table slots; w_start / w_pref: its
// 64 entries of each.
template <bool VERTEX, int GL, int SLOTS, int MAXP>
__device__ void sp_groups(const KInst& I, int first, int count, const int* list, int* out, int* nout,
                          unsigned* wtab, int32_t* w_start, int* w_pref, int force_range, bool r1,
                          unsigned long long* pairs_seen) {
  constexpr int G = 64 / GL;
  const int w = threadIdx.x >> 6, lane = lane_id();
  const int q = lane / GL, gl = lane & (GL - 1);
  const int nid = VERTEX ? I.n : I.m;
  unsigned* gt = wtab + q * SLOTS;
  int32_t* g_start = w_start + q * GL;
  int* g_pref = w_pref + q * GL;
  for (int k0 = w * G; k0 < count; k0 += 4 * G) {
    const int k = k0 + q;
    const bool have = k < count;
    int r = 0, j = 0, sj = 0, fj = 0;
    int oa = 0, ob = 0;
    if (have) {
      r = list ? list[k] : first + k;
      j = I.rid[r];
      sj = I.rs[r];
      fj = I.rf[r];
      outer_range<VERTEX>(I, j, &oa, &ob);
    }
    const bool mine = have && !(VERTEX && sj == 0);
    const int K = mine ? (int)(ob - oa) : 0;
    bool grp = !VERTEX && mine && K <= GL && !force_range;
    const int cls = r1 ? slack_class(min(max(sj - fj, 0), 254)) : -1;
    int ia = 0, ib = 0;
    if (grp && gl < K && !outer_elem<VERTEX>(I, oa + gl, &ia, &ib, cls)) ia = ib = 0;
    int P;
    const int pre = group_exscan<GL>(grp && gl < K ? (int)(ib - ia) : 0, &P);
    const int cb = count_bits(sj);
    if (grp && (P > MAXP || !packs(nid, cb))) grp = false;
    const bool slk = !VERTEX && !I.rule_se && packs_slack(nid, cb);
    if (mine && !grp && gl == 0) out[atomicAdd(nout, 1)] = r;
    const int S = grp ? min(SLOTS, max(32, pow2_at_least((4 * P + 2) / 3))) : 0;
    for (int h = gl; h < S; h += GL) gt[h] = kEmpty;
    g_start[gl] = (int32_t)ia;
    g_pref[gl] = pre;
    wave_sync();
    // capped slacks keep the test exact: min(a, 254) > min(b, 254) implies a > b
    const int slack_cap = (VERTEX || I.rule_se) ? 254 : min(sj - fj, 254);
    // Under DP a victim with f_j = 1 and s_j >= 2 is deleted by any partner
    // e_i of slack 0 (|e_i| = f_i) it shares a vertex with: then X_ij >= 1
    // = f_j + s_i - f_i, so D_ij, and D_ji (f_j + X_ij >= f_i + s_j, with
    // X_ij <= s_i = f_i) would need s_j <= 1, so the tie break deletes e_j
    // whatever the ids.  Such a victim stops at the first term step that
    // meets one (no further terms, no verdict).
    const bool probe = !VERTEX && !I.rule_se && fj == 1 && sj >= 2;
    int never = 0;   // a table of >= 4P/3 slots never fills
    int visited;
    const bool found = group_terms<VERTEX, GL>(I, j, K, grp ? P : 0, g_start, g_pref, slack_cap, probe,
                                               &visited, [&](int partner, int st) {
      hash_insert(gt, S, cb, 1, 0, slk ? (partner << 8) | st : partner, &never);
    });
    if (grp && gl == 0) *pairs_seen += (unsigned long long)visited;
    wave_sync();
    // a: deleters (slack keys) or the exact test sum; b: partners left for
    // the second pass
    int a = found ? 1 : 0, b = 0;
    if (!found) {
      if (slk) slack_scan<GL>(gt, S, gl, cb, fj, j, &a, &b);
      else a = scan_table<VERTEX, GL>(I, gt, S, gl, cb, sj, fj, j);
    }
    a = group_sum<GL>(a);
    b = group_sum<GL>(b);
    int rest = 0;
    if (slk && a == 0 && b > 0) rest = slack_rest<GL>(I, gt, S, gl, cb, sj, fj, j);
    const int v = a + group_sum<GL>(rest);
    if (grp && gl == 0) {
      if (!VERTEX) { if (v) I.kill[r] = 1; }
      else I.cnt[r] = v;
    }
    wave_sync();
  }
}

template <bool VERTEX, bool BIG>
__device__ void sp_count_tile(const KInst& I, int tile, int force_range) {
  constexpr int kWHash = SpTables<BIG>::kWHash;
  constexpr int kGMaxP = SpTables<BIG>::kGMaxP;
  constexpr int kG2MaxP = SpTables<BIG>::kG2MaxP;
  __shared__ unsigned tab[4 * kWHash];
  __shared__ int32_t s_start[256];
  __shared__ int s_pref[256];
  __shared__ int sh[5];
  __shared__ int s_over[5];
  __shared__ int s_heavy[kTile], s_heavyP[kTile];
  __shared__ int s_wl[kTile], s_wl2[kTile], s_ord[kTile];
  __shared__ int s_nheavy, s_nwl, s_nwl2, s_verdict, s_nfront, s_nback;
  if (inst_idle(I.ctr) || !is_sparse(I)) return;
  const int rows = VERTEX ? I.ctr[C_NA] : I.ctr[C_MA];
  if (tile * kTile >= rows) return;
  const int tid = threadIdx.x, w = tid >> 6, lane = lane_id();
  const int nid = VERTEX ? I.n : I.m;   // partner ids
  if (tid == 0) { s_nheavy = 0; s_nwl = 0; s_nwl2 = 0; s_nfront = 0; s_nback = 0; }
  __syncthreads();
  unsigned long long pairs_seen = 0;
  const int rend = min(rows, (tile + 1) * kTile);
  // round 1 of the edge phase: lists in slack-class order (k_prep_slack)
  const bool r1 = !VERTEX && I.ctr[C_ROUND] == 1;
  // verdict on one partner i with count c: DP / SE any, MD a count
  auto judge = [&](int i, int c, int sj, int fj, int j) -> int {
    return pair_verdict<VERTEX>(I, i, c, VERTEX ? I.vdeg[i] : I.esz[i], VERTEX ? 0 : I.fw[i], sj, fj, j);
  };
  // ---- edge phase: groups of 16 lanes over the tile, then 32 lanes over
  // what they left; the vertex phase takes every row one per wave
  const int* wl = nullptr;
  int nwl = rend - tile * kTile;
  if (!VERTEX) {
    // a wave runs its groups in lockstep: the victims the slack-0 probe can
    // stop early (DP, f_j = 1, s_j >= 2; see sp_groups) go first, the others
    // after them, so that waves mostly hold victims of one kind
    if (tid < nwl) {
      const int r = tile * kTile + tid;
      if (!I.rule_se && I.rf[r] == 1 && I.rs[r] >= 2) s_ord[atomicAdd(&s_nfront, 1)] = r;
      else s_ord[nwl - 1 - atomicAdd(&s_nback, 1)] = r;
    }
    __syncthreads();
    sp_groups<VERTEX, 16, kWHash / 4, kGMaxP>(I, 0, nwl, s_ord, s_wl, &s_nwl, tab + w * kWHash, s_start + w * 64,
                                              s_pref + w * 64, force_range, r1, &pairs_seen);
    __syncthreads();
    wl = s_wl;
    nwl = s_nwl;
  }
  if (!VERTEX && !force_range && nwl > 0) {
    sp_groups<VERTEX, 32, kWHash / 2, kG2MaxP>(I, 0, nwl, s_wl, s_wl2, &s_nwl2, tab + w * kWHash,
                                               s_start + w * 64, s_pref + w * 64, force_range, r1, &pairs_seen);
    __syncthreads();
    wl = s_wl2;
    nwl = s_nwl2;
  }
  // ---- the victims the groups left (edge phase) or every row (vertex
  // phase), one per wave
  unsigned* ht = tab + w * kWHash;
  int32_t* w_start = s_start + w * 64;
  int* w_pref = s_pref + w * 64;
  for (int k = w; k < nwl; k += 4) {
    const int r = wl ? wl[k] : tile * kTile + k;
    const int j = I.rid[r];
    const int sj = I.rs[r], fj = I.rf[r];
    // an isolated vertex needs no count: the compaction deletes it
    if (VERTEX && sj == 0) continue;
    int oa, ob;
    outer_range<VERTEX>(I, j, &oa, &ob);
    const int cls = r1 ? slack_class(min(max(sj - fj, 0), 254)) : -1;
    // an outer list of at most 64 elements is read once: its inner starts
    // and lengths stay in the lanes for the count
    const bool one = ob - oa <= 64;
    const int K = one ? (int)(ob - oa) : 0;
    int P = 0, pre = 0;
    int ia1 = 0;
    if (one) {
      int ib = 0;
      if (lane < K && !outer_elem<VERTEX>(I, oa + lane, &ia1, &ib, cls)) ia1 = ib = 0;
      pre = wave_exscan((int)(ib - ia1), &P);
    } else {
      for (int p = oa + lane; p < ob; p += 64) {
        int ia, ib;
        if (outer_elem<VERTEX>(I, p, &ia, &ib, cls)) P += (int)(ib - ia);
      }
      P = wave_sum(P);
    }
    if (lane == 0) pairs_seen += (unsigned long long)P;
    if (P > kWHash / 2) {
      if (lane == 0) {
        const int q = atomicAdd(&s_nheavy, 1);
        s_heavy[q] = r;
        s_heavyP[q] = P;
      }
      continue;
    }
    const int cb = count_bits(sj);
    int verdict = 0;
    bool overflow = force_range != 0 || !packs(nid, cb);
    if (!overflow) {
      const int S = max(64, pow2_at_least(2 * P));
      for (int h = lane; h < S; h += 64) ht[h] = kEmpty;
      if (lane == 0) s_over[w] = 0;
      if (one) {
        w_start[lane] = (int32_t)ia1;
        w_pref[lane] = pre;
      }
      wave_sync();
      auto ins = [&](int partner) { hash_insert(ht, S, cb, 1, 0, partner, &s_over[w]); };
      // capped slacks keep the test exact: min(a, 254) > min(b, 254) implies a > b
      const int slack_cap = (VERTEX || I.rule_se) ? 254 : min(sj - fj, 254);
      const bool slk = one && !VERTEX && !I.rule_se && packs_slack(nid, cb);
      if (one)
        wave_terms_one<VERTEX>(I, j, K, P, w_start, w_pref, slack_cap, [&](int partner, int st) {
          hash_insert(ht, S, cb, 1, 0, slk ? (partner << 8) | st : partner, &s_over[w]);
        });
      else
        wave_for_each_term<VERTEX>(I, j, w_start, w_pref, cls, ins);
      wave_sync();
      if (s_over[w]) {
        overflow = true;
      } else if (slk) {
        int a, b;
        slack_scan<64>(ht, S, lane, cb, fj, j, &a, &b);
        a = wave_sum(a);
        b = wave_sum(b);
        verdict = a;
        if (a == 0 && b > 0) verdict = wave_sum(slack_rest<64>(I, ht, S, lane, cb, sj, fj, j));
      } else {
        verdict = wave_sum(scan_table<VERTEX, 64>(I, ht, S, lane, cb, sj, fj, j));
      }
      wave_sync();
    }
    if (overflow) {
      verdict = 0;
      int* hv = reinterpret_cast<int*>(ht);
      for (int lo = 0; lo < nid; lo += kWHash) {
        for (int h = lane; h < kWHash; h += 64) hv[h] = 0;
        wave_sync();
        wave_for_each_term<VERTEX>(I, j, w_start, w_pref, cls, [&](int partner) {
          if (partner >= lo && partner < lo + kWHash) atomicAdd(&hv[partner - lo], 1);
        });
        wave_sync();
        int v = 0;
        for (int h = lane; h < kWHash; h += 64)
          if (hv[h] > 0 && lo + h < nid) v += judge(lo + h, hv[h], sj, fj, j);
        verdict += wave_sum(v);
        wave_sync();
      }
    }
    if (lane == 0) {
      if (!VERTEX) { if (verdict) I.kill[r] = 1; }
      else I.cnt[r] = verdict;
    }
  }
  // each lane holds the terms of the victims it led (a group's first lane,
  // a wave's lane 0)
  if (pairs_seen) gadd(reinterpret_cast<GLOBAL unsigned long long*>(&I.ctr[C_PAIRS_SUM]), pairs_seen);
  __syncthreads();
  // ---- heavy victims, the whole block each
  constexpr int BS = 4 * kWHash;
  const int nheavy = s_nheavy;
  for (int q = 0; q < nheavy; ++q) {
    const int r = s_heavy[q];
    const int j = I.rid[r];
    const int sj = I.rs[r], fj = I.rf[r];
    const int P = s_heavyP[q];
    const int cls = r1 ? slack_class(min(max(sj - fj, 0), 254)) : -1;
    const int passes = max(1, (P + BS / 2 - 1) / (BS / 2));
    const int S = passes > 1 ? BS : max(256, pow2_at_least(2 * P));
    const int cb = count_bits(sj);
    const unsigned cm = (1u << cb) - 1;
    if (tid == 0) s_verdict = 0;
    bool overflow = force_range != 0 || !packs(nid, cb);
    for (int pass = 0; pass < passes && !overflow; ++pass) {
      for (int h = tid; h < S; h += blockDim.x) tab[h] = kEmpty;
      if (tid == 0) s_over[4] = 0;
      __syncthreads();
      block_for_each_term<VERTEX>(I, j, s_start, s_pref, sh, cls, [&](int partner) {
        hash_insert(tab, S, cb, passes, pass, partner, &s_over[4]);
      });
      if (s_over[4]) { overflow = true; break; }
      for (int h = tid; h < S; h += blockDim.x) {
        const unsigned wd = tab[h];
        if (wd != kEmpty && judge((int)(wd >> cb), (int)(wd & cm), sj, fj, j)) atomicAdd(&s_verdict, 1);
      }
      __syncthreads();
      if (!VERTEX && s_verdict) break;
    }
    if (overflow) {
      int* hv = reinterpret_cast<int*>(tab);
      if (tid == 0) s_verdict = 0;
      __syncthreads();
      for (int lo = 0; lo < nid; lo += BS) {
        for (int h = tid; h < BS; h += blockDim.x) hv[h] = 0;
        __syncthreads();
        block_for_each_term<VERTEX>(I, j, s_start, s_pref, sh, cls, [&](int partner) {
          if (partner >= lo && partner < lo + BS) atomicAdd(&hv[partner - lo], 1);
        });
        for (int h = tid; h < BS; h += blockDim.x)
          if (hv[h] > 0 && lo + h < nid && judge(lo + h, hv[h], sj, fj, j)) atomicAdd(&s_verdict, 1);
        __syncthreads();
      }
    }
    if (tid == 0) {
      if (!VERTEX) { if (s_verdict) I.kill[r] = 1; }
      else I.cnt[r] = s_verdict;
    }
    __syncthreads();
  }
}

// Over the phase's alive sparse tiles (prefix `ap`), one per workgroup when
// the grid covers them all; the waves of a workgroup share nothing but the
// tile, so none waits for another.  In a set the tiles of one member go to
// one XCD (xcd_remap), whose L2 then holds that member's lists for all of
// them.  Bounded to six waves per SIMD (80 VGPRs, a few spilled): the
// counting is latency-bound, and the sixth wave hides more of it than the
// spills cost.
template <bool VERTEX, bool BIG>
__global__ __launch_bounds__(256, 6) void k_sp_count(const DInst* __restrict__ insts, int ninst, const int32_t* ap, int force_range) {
  const int32_t* pf = ap;   // read where it is: the prefix is small and cached
  const int total = pf[ninst];
  if ((int)blockIdx.x >= total) return;
  for (int w = ninst > 1 && gridDim.x >= (unsigned)total ? xcd_remap(blockIdx.x, total) : (int)blockIdx.x;
       w < total; w += gridDim.x) {
    const int x = unit_owner(pf, ninst, w);
    const KInst I = kview(insts[x]);
    sp_count_tile<VERTEX, BIG>(I, w - pf[x], force_range);
  }
}

// ------------------------------------------------------------- compaction
// One pass per phase, one block of kBlock rows each: the deletion decision,
// the survivors' stable positions and the scatter.  In the vertex phase the
// block first takes the MD decision: delete v_j iff C_j >= the largest demand
// over E(v_j) (an isolated vertex has largest demand 0 and is always
// deleted).  In FE mode (instances whose FE pass fired this round) the kill
// flags come from the FE pass (k_fe_apply, k_fe_vkill).
//
// Positions come from a decoupled look-back scan: every block publishes its
// survivor count in its status word, and its inclusive prefix once known;
// a block sums its predecessors' words back to the nearest inclusive one,
// 64 at a time.  Blocks take tickets in launch order, so every block a
// block waits for already holds a ticket, runs, and never waits for a later
// one: the waits end.  Status words carry an epoch (4 per round, one per
// compaction launch) so that words of earlier launches read as not ready;
// the prepare step zeroes them.  The instance's last block writes the new
// alive count, the number deleted and advances the compaction count, whose
// parity names the current compact list: every block of the instance has
// read both before it, since they publish after reading them.
constexpr uint64_t kStAgg = 1, kStInc = 2;

// An instance's counters as a round's last kernel sees them.
struct RoundState {
  int done, err, killed_e, killed_v, round, ma, na;
};
__device__ int end_round(const KInst& I, int* v);
__device__ int end_round_from(const KInst& I, const RoundState& st, int* v);
__device__ void publish_active(int32_t* gctr, int32_t* hflag, int active);

// The counters a compaction block needs, read together (no branch between
// the loads; a set of one reads them before taking its first ticket).
struct CompactState {
  RoundState st;
  int fe_fired, ncomp;
};
template <bool VERTEX>
__device__ __forceinline__ CompactState compact_state(const KInst& I) {
  const GLOBAL int32_t* c = I.ctr;
  CompactState s;
  s.st.done = c[C_DONE];
  s.st.err = c[C_ERR];
  s.st.killed_e = c[C_KILLED_E];
  s.st.killed_v = c[C_KILLED_V];
  s.st.round = c[C_ROUND];
  s.st.ma = c[C_MA];
  s.st.na = c[C_NA];
  s.fe_fired = c[C_FE_FIRED];
  s.ncomp = c[VERTEX ? C_NCOMP_V : C_NCOMP_E];
  return s;
}


template <bool VERTEX, bool FE>
__device__ void compact_block(const DInst* __restrict__ insts, const int32_t* bp, int ninst, int g, int phase,
                              int32_t* gctr, int32_t* hflag, int32_t* ap, int fuse_end, bool have_st,
                              CompactState st_in) {
  __shared__ int sh[17];
  __shared__ int s_excl;
  const int x = unit_owner(bp, ninst, g);
  const KInst I = kview(insts[x]);
  const CompactState cs = have_st ? st_in : compact_state<VERTEX>(I);
  if (cs.st.done | cs.st.err) {
    // a set of one whose instance is already done (rejected input): the
    // round still ends, with no instance active
    if (VERTEX && !FE && fuse_end && g == 0 && threadIdx.x == 0) {
      gctr[G_TICKET] = 0;
      publish_active(gctr, hflag, 0);
    }
    return;
  }
  if (FE && !cs.fe_fired) return;
  const int rows = VERTEX ? cs.st.na : cs.st.ma;
  const int blk = g - bp[x];
  const int nb = max(1, (rows + kBlock - 1) / kBlock);
  if (blk >= nb) return;
  const int ncomp = cs.ncomp;
  const int cur = ncomp & 1, nxt = cur ^ 1;
  const int round = cs.st.round;
  const uint64_t epoch = (uint64_t)((round * 4 + phase) & 0x3fffffff) << 34;
  const int r = blk * kBlock + threadIdx.x;
  int alive = 0, id = 0;
  if (r < rows) {
    if (VERTEX && !FE) {
      // loaded together: no short circuit between them
      const int rs_ = I.rs[r], cnt_ = I.cnt[r], rf_ = I.rf[r];
      const int k = (rs_ == 0) | (cnt_ >= rf_);
      I.kill[r] = (uint8_t)k;
      alive = !k;
    } else {
      alive = !I.kill[r];   // DP flags, or FE flags (k_fe_apply / k_fe_vkill)
    }
    id = VERTEX ? vrow_list(I, cur)[r] : erow_list(I, cur)[r];
  }
  int tot;
  const int pre = block_exscan(alive, sh, &tot);
  if (threadIdx.x == 0) {
    st_store(&I.bstat[blk], epoch | ((blk == 0 ? kStInc : kStAgg) << 32) | (uint32_t)tot);
    s_excl = 0;
  }
  if (blk > 0 && threadIdx.x < 64) {
    const int lane = threadIdx.x;
    int excl = 0;
    int top = blk - 1;
    long long spins = 0;
    for (;;) {
      const int q = top - lane;
      const uint64_t w = q >= 0 ? st_load(&I.bstat[q]) : 0;
      const bool ready = q >= 0 && (w >> 34) == (epoch >> 34);
      const bool inc = ready && ((w >> 32) & 3) == kStInc;
      const unsigned long long incm = __ballot(inc);
      // lanes up to the nearest inclusive word (all valid lanes if none)
      const int upto = incm ? __ffsll((long long)incm) - 1 : 63;
      const bool need = lane <= upto && q >= 0;
      if (__ballot(need && !ready)) {
        if (++spins > kSpinMax) {
          if (lane == 0) set_err(I.ctr, E_STALL);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
        continue;
      }
      int v = need ? (int)(uint32_t)w : 0;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
      excl += v;
      if (incm || top - 63 <= 0) break;
      top -= 64;
    }
    if (lane == 0) {
      s_excl = excl;
      st_store(&I.bstat[blk], epoch | (kStInc << 32) | (uint32_t)(excl + tot));
    }
  }
  __syncthreads();
  const int base = s_excl;
  if (blk == nb - 1 && threadIdx.x == 0) {
    const int total = base + tot;
    I.ctr[VERTEX ? C_NA : C_MA] = total;
    I.ctr[VERTEX ? C_NCOMP_V : C_NCOMP_E] = ncomp + 1;
    if (rows - total) {
      gadd(&I.ctr[VERTEX ? C_KILLED_V : C_KILLED_E], rows - total);
      if (FE && VERTEX) gadd(&I.ctr[C_NFORCED], rows - total);
    }
    if (VERTEX && !FE && fuse_end) {
      // a set of one instance without FE: this block ends the round (the
      // edge compaction resets this launch's ticket), from the counts it
      // already holds: the round's last writer of C_KILLED_V and C_NA is
      // this block
      RoundState st = cs.st;
      st.killed_v += rows - total;
      st.na = total;
      int v[AP_N];
      const int active = end_round_from(I, st, v);
#pragma unroll
      for (int k = 0; k < AP_N; ++k) { ap[k * 2] = 0; ap[k * 2 + 1] = v[k]; }
      gctr[G_TICKET] = 0;
      publish_active(gctr, hflag, active);
    }
  }
  if (r < rows) {
    const int pos = base + pre;
    if (VERTEX) {
      if (alive) { vrow_list(I, nxt)[pos] = id; I.vcol[id] = pos; }
      else { I.death_v[id] = round; I.vcol[id] = -1; }
    } else {
      if (alive) { erow_list(I, nxt)[pos] = id; I.ecol[id] = pos; }
      else { I.death_e[id] = round; I.ecol[id] = -1; I.eslk[id] = 255; }
    }
  }
}

// Persistent: workgroups take compaction blocks (prefix `bp` over the
// instances) by ticket until none is left; a workgroup finishes its block,
// look-back included, before taking the next ticket.
template <bool VERTEX, bool FE>
__global__ __launch_bounds__(kBlock) void k_compact(const DInst* __restrict__ insts, int ninst, const int32_t* bp, int32_t* gctr,
                                                   int slot, int phase, int32_t* hflag, int32_t* ap,
                                                   int fuse_end) {
  __shared__ int32_t s_pf[kPrefLds];
  __shared__ int s_tk;
  const int32_t* pf = cache_prefix(bp, ninst, s_pf);
  const int total = pf[ninst];
  // a set of one: the instance's counters load with the first ticket
  CompactState st1 = {};
  if (ninst == 1) st1 = compact_state<VERTEX>(kview(insts[0]));
  for (;;) {
    if (threadIdx.x == 0) s_tk = atomicAdd(&gctr[slot], 1);
    __syncthreads();
    const int g = s_tk;
    if (!FE && fuse_end && g == 0 && threadIdx.x == 0) {
      if (!VERTEX) {
        // the previous round's vertex compaction has finished: reset its
        // ticket for this round
        gctr[G_TICKET + 1] = 0;
      } else if (total == 0) {
        // nothing alive (a round queued after the fixpoint): the round
        // still ends, with no instance active
        gctr[G_TICKET] = 0;
        publish_active(gctr, hflag, 0);
      }
    }
    if (g >= total) break;
    compact_block<VERTEX, FE>(insts, pf, ninst, g, phase, gctr, hflag, ap, fuse_end, ninst == 1, st1);
    __syncthreads();
  }
}

// ------------------------------------------------------------ FE pass
// Vertex rows of an instance whose FE pass fired: deleted iff forced.
__global__ void k_fe_vkill(const DInst* __restrict__ insts, int ninst, const int32_t* bp) {
  const int x = unit_owner(bp, ninst, blockIdx.x);
  const KInst I = kview(insts[x]);
  if (!I.rule_fe || inst_idle(I.ctr) || !I.ctr[C_FE_FIRED]) return;
  const int r = (blockIdx.x - bp[x]) * kBlock + threadIdx.x;
  if (r >= I.ctr[C_NA]) return;
  I.kill[r] = I.forced[vrow_list(I, I.ctr[C_NCOMP_V] & 1)[r]] ? 1 : 0;
}

// Full-edge rule (Section 3.1), for instances that apply it, in a round in
// which DP and MD deleted nothing: every alive hyperedge whose alive size
// equals its current demand forces its alive vertices into the solution.
// Forcing removes a vertex and one unit of demand from every hyperedge
// containing it, so |e| - f(e) is unchanged and one pass is exhaustive.
__global__ void k_fe_mark(const DInst* __restrict__ insts, int ninst, const int32_t* bp) {
  const int x = unit_owner(bp, ninst, blockIdx.x);
  const KInst I = kview(insts[x]);
  if (!I.rule_fe || inst_idle(I.ctr) || I.ctr[C_KILLED_E] || I.ctr[C_KILLED_V]) return;
  const int rows = I.ctr[C_MA];
  const int r = (blockIdx.x - bp[x]) * kBlock + threadIdx.x;
  if (r >= rows) return;
  const int e = erow_list(I, I.ctr[C_NCOMP_E] & 1)[r];
  int sz = 0;
  for (int64_t p = I.eptr[e], q = I.eptr[e + 1]; p < q; ++p) sz += I.vcol[I.evtx[p]] >= 0;
  if (sz != I.fw[e]) return;
  for (int64_t p = I.eptr[e], q = I.eptr[e + 1]; p < q; ++p) {
    const int v = I.evtx[p];
    if (I.vcol[v] >= 0) I.forced[v] = 1;
  }
  I.ctr[C_FE_FIRED] = 1;
}

// Demand update: every alive hyperedge loses one unit per forced alive
// vertex; it is deleted when its demand reaches 0 (the full ones included).
__global__ void k_fe_apply(const DInst* __restrict__ insts, int ninst, const int32_t* bp) {
  const int x = unit_owner(bp, ninst, blockIdx.x);
  const KInst I = kview(insts[x]);
  if (!I.rule_fe || inst_idle(I.ctr) || !I.ctr[C_FE_FIRED]) return;
  const int rows = I.ctr[C_MA];
  const int r = (blockIdx.x - bp[x]) * kBlock + threadIdx.x;
  if (r >= rows) return;
  const int e = erow_list(I, I.ctr[C_NCOMP_E] & 1)[r];
  int t = 0;
  for (int64_t p = I.eptr[e], q = I.eptr[e + 1]; p < q; ++p) {
    const int v = I.evtx[p];
    if (I.vcol[v] >= 0 && I.forced[v]) ++t;
  }
  const int f = I.fw[e] - t;
  I.fw[e] = f;
  I.kill[r] = f <= 0 ? 1 : 0;
}

// ------------------------------------------------------------------ phases
static const int32_t* alive_prefix(const LaunchCtx& c, int k) { return c.ap + (size_t)k * (c.ninst + 1); }

template <bool VERTEX>
static void launch_rows_sparse_t(const LaunchCtx& c) {
  const int nb = VERTEX ? c.n_vblocks : c.n_eblocks;
  if (c.has_sparse && nb)
    hipLaunchKernelGGL(k_sp_rows<VERTEX>, dim3(std::min(nb, 2 * c.cus)), dim3(kBlock), 0, c.stream, c.insts,
                       c.ninst, alive_prefix(c, VERTEX ? AP_VB : AP_EB));
}

template <bool VERTEX>
static void launch_rows_dense_t(const LaunchCtx& c) {
  const int ntiles = VERTEX ? c.n_vtiles : c.n_etiles;
  if (!c.has_dense || !ntiles) return;
  const dim3 grid(std::min(ntiles, 2 * c.cus));
  const int32_t* ap = alive_prefix(c, VERTEX ? AP_VTD : AP_ETD);
  if (c.variant == 2)
    hipLaunchKernelGGL((k_rows_encode<VERTEX, true>), grid, dim3(kRowsThreads), 0, c.stream, c.insts, c.ninst, ap,
                       c.count_work);
  else
    hipLaunchKernelGGL((k_rows_encode<VERTEX, false>), grid, dim3(kRowsThreads), 0, c.stream, c.insts, c.ninst, ap,
                       c.count_work);
}

template <bool VERTEX, bool SE>
static void launch_int8(const LaunchCtx& c, const int32_t* pp) {
  if (c.gemm_lds == 2)
    hipLaunchKernelGGL((k_gemm_async<VERTEX, SE>), dim3(c.gemm_grid), dim3(kPairThreads), 0, c.stream, c.insts,
                       c.ninst, pp, c.count_work);
  else if (c.gemm_lds)
    hipLaunchKernelGGL((k_gemm_lds<VERTEX, SE>), dim3(c.gemm_grid), dim3(kPairThreads), 0, c.stream, c.insts,
                       c.ninst, pp, c.count_work);
  else
    hipLaunchKernelGGL((k_gemm<VERTEX, SE>), dim3(c.gemm_grid), dim3(kPairThreads), 0, c.stream, c.insts, c.ninst,
                       pp, c.count_work);
}

template <bool VERTEX>
static void launch_sparse_count(const LaunchCtx& c) {
  if (c.has_sparse) {
    // one workgroup per tile: tiles differ widely in cost (hyperedge sizes
    // and degrees vary between and within instances), and the hardware
    // scheduler then balances them, where a persistent grid with a fixed
    // stride leaves some workgroups with the expensive ones
    const int ntiles = VERTEX ? c.n_vtiles : c.n_etiles;
    if (ntiles && c.sparse_big)
      hipLaunchKernelGGL((k_sp_count<VERTEX, true>), dim3(ntiles), dim3(256), 0, c.stream, c.insts,
                         c.ninst, alive_prefix(c, VERTEX ? AP_VTS : AP_ETS), c.sparse_force_range);
    else if (ntiles)
      hipLaunchKernelGGL((k_sp_count<VERTEX, false>), dim3(ntiles), dim3(256), 0, c.stream, c.insts,
                         c.ninst, alive_prefix(c, VERTEX ? AP_VTS : AP_ETS), c.sparse_force_range);
  }
}

template <bool VERTEX>
static void launch_dense_contraction(const LaunchCtx& c) {
  if (!c.has_dense) return;
  const int32_t* pp = alive_prefix(c, VERTEX ? AP_VP : AP_EP);
  if (c.variant == 2)
    hipLaunchKernelGGL(k_gemm_bits<VERTEX>, dim3(c.gemm_grid), dim3(kPairThreads), 0, c.stream, c.insts, c.ninst, pp,
                       c.count_work);
  else if (!VERTEX && c.rule_se)
    launch_int8<VERTEX, true>(c, pp);
  else
    launch_int8<VERTEX, false>(c, pp);
}

template <bool VERTEX>
static void launch_phase_post(const LaunchCtx& c) {
  // always launched: every active instance has at least one block (a set of
  // one ends its round there)
  const int nb = std::max(1, VERTEX ? c.n_vblocks : c.n_eblocks);
  hipLaunchKernelGGL((k_compact<VERTEX, false>), dim3(std::min(nb, 2 * c.cus)), dim3(kBlock), 0, c.stream, c.insts,
                     c.ninst, alive_prefix(c, VERTEX ? AP_VB : AP_EB), c.gctr, G_TICKET + (VERTEX ? 1 : 0),
                     VERTEX ? 1 : 0, c.hflag, c.ap, c.fuse_end);
}

void launch_rows(const LaunchCtx& c, bool vertex) {
  launch_rows_sparse(c, vertex);
  launch_rows_dense(c, vertex);
}
void launch_rows_sparse(const LaunchCtx& c, bool vertex) {
  if (!c.ninst) return;
  if (vertex) launch_rows_sparse_t<true>(c); else launch_rows_sparse_t<false>(c);
}
void launch_rows_dense(const LaunchCtx& c, bool vertex) {
  if (!c.ninst) return;
  if (vertex) launch_rows_dense_t<true>(c); else launch_rows_dense_t<false>(c);
}
void launch_contraction(const LaunchCtx& c, bool vertex) {
  launch_contraction_sparse(c, vertex);
  launch_contraction_dense(c, vertex);
}
void launch_contraction_sparse(const LaunchCtx& c, bool vertex) {
  if (!c.ninst) return;
  if (vertex) launch_sparse_count<true>(c); else launch_sparse_count<false>(c);
}
void launch_contraction_dense(const LaunchCtx& c, bool vertex) {
  if (!c.ninst) return;
  if (vertex) launch_dense_contraction<true>(c); else launch_dense_contraction<false>(c);
}
void launch_compact(const LaunchCtx& c, bool vertex) {
  if (!c.ninst) return;
  if (vertex) launch_phase_post<true>(c); else launch_phase_post<false>(c);
}

void launch_fe(const LaunchCtx& c) {
  if (!c.ninst || !c.has_fe) return;
  if (c.n_eblocks) {
    hipLaunchKernelGGL(k_fe_mark, dim3(c.n_eblocks), dim3(kBlock), 0, c.stream, c.insts, c.ninst, c.ebp);
    hipLaunchKernelGGL(k_fe_apply, dim3(c.n_eblocks), dim3(kBlock), 0, c.stream, c.insts, c.ninst, c.ebp);
    hipLaunchKernelGGL((k_compact<false, true>), dim3(std::min(c.n_eblocks, 2 * c.cus)), dim3(kBlock), 0, c.stream,
                       c.insts, c.ninst, c.ebp, c.gctr, G_TICKET + 2, 2, c.hflag, c.ap, 0);
  }
  if (c.n_vblocks) {
    hipLaunchKernelGGL(k_fe_vkill, dim3(c.n_vblocks), dim3(kBlock), 0, c.stream, c.insts, c.ninst, c.vbp);
    hipLaunchKernelGGL((k_compact<true, true>), dim3(std::min(c.n_vblocks, 2 * c.cus)), dim3(kBlock), 0, c.stream,
                       c.insts, c.ninst, c.vbp, c.gctr, G_TICKET + 3, 3, c.hflag, c.ap, 0);
  }
}

// Bounded busy wait on the device clock (profiling only): keeps the queue
// busy while the host enqueues a round, so that event timestamps bracket
// kernels that run back to back.  Always exits after `ticks`.
__global__ void k_delay(long long ticks) {
  const long long t0 = wall_clock64();
  while (wall_clock64() - t0 < ticks) {}
}

void launch_delay(hipStream_t stream, long long ticks) {
  hipLaunchKernelGGL(k_delay, dim3(1), dim3(1), 0, stream, ticks);
}

// -------------------------------------------------------------- round end
// One block.  Fixpoint test of Algorithm 3 per instance: an iteration that
// deletes nothing ends it; `rounds` counts the iterations that deleted
// something.  Instances still active move to the next iteration with their
// per-phase counters cleared; G_ANY receives the number still active and the
// compaction tickets restart at 0.
// End of a round for one instance (Algorithm 3's loop test): an instance
// whose round deleted nothing is done (its round count excludes this round);
// otherwise its counters are reset for the next round and v[] receives the
// next round's work units.  Returns 1 if the instance stays active.
__device__ int end_round_from(const KInst& I, const RoundState& st, int* v) {
  GLOBAL int32_t* ctr = I.ctr;
#pragma unroll
  for (int k = 0; k < AP_N; ++k) v[k] = 0;
  ctr[C_FE_FIRED] = 0;
  if (st.done || st.err) return 0;
  if (st.killed_e == 0 && st.killed_v == 0) {
    ctr[C_DONE] = 1;
    ctr[C_ROUNDS] = st.round - 1;
    return 0;
  }
  ctr[C_ROUNDS] = st.round;
  ctr[C_ROUND] = st.round + 1;
  ctr[C_KILLED_E] = 0;
  ctr[C_KILLED_V] = 0;
  const int re = st.ma, rv = st.na;
  const bool sp = is_sparse(I);
  const int te = (re + kTile - 1) / kTile, tv = (rv + kTile - 1) / kTile;
  v[AP_ETD] = sp ? 0 : te;
  v[AP_VTD] = sp ? 0 : tv;
  v[AP_ETS] = sp ? te : 0;
  v[AP_VTS] = sp ? tv : 0;
  // at least one compaction block per active instance: it advances the
  // compaction count and, for a set of one, ends the round
  v[AP_EB] = max(1, (re + kBlock - 1) / kBlock);
  v[AP_VB] = max(1, (rv + kBlock - 1) / kBlock);
  // contraction candidates (a set's total is checked to fit on the host)
  v[AP_EP] = sp ? 0 : (int)min<int64_t>((int64_t)te * (te + 1) / 2, INT32_MAX);
  v[AP_VP] = sp ? 0 : (int)min<int64_t>((int64_t)tv * (tv + 1) / 2, INT32_MAX);
  return 1;
}

__device__ int end_round(const KInst& I, int* v) {
  const GLOBAL int32_t* c = I.ctr;
  RoundState st;
  st.done = c[C_DONE];
  st.err = c[C_ERR];
  st.killed_e = c[C_KILLED_E];
  st.killed_v = c[C_KILLED_V];
  st.round = c[C_ROUND];
  st.ma = c[C_MA];
  st.na = c[C_NA];
  return end_round_from(I, st, v);
}

// Publishes the number of active instances: G_ANY, and the host-mapped slot
// of this round end (sequence number mod kFlagSlots): the count, then the
// sequence number with release order, so a host that sees the number sees
// the count.
__device__ void publish_active(int32_t* gctr, int32_t* hflag, int active) {
  gctr[G_ANY] = active;
  const int seq = gctr[G_RSEQ] + 1;
  gctr[G_RSEQ] = seq;
  if (hflag) {
    int32_t* s = hflag + 2 * (seq % kFlagSlots);
    __hip_atomic_store(s + 1, active, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(s, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

__global__ void k_round_end(const DInst* __restrict__ insts, int ninst, int32_t* gctr, int32_t* hflag, int32_t* ap) {
  __shared__ int sh[5];
  int carry[AP_N];
#pragma unroll
  for (int k = 0; k < AP_N; ++k) carry[k] = 0;
  int active_tot = 0;
  for (int base = 0; base < ninst; base += blockDim.x) {
    const int x = base + threadIdx.x;
    int v[AP_N];
#pragma unroll
    for (int k = 0; k < AP_N; ++k) v[k] = 0;
    const int active = x < ninst ? end_round(kview(insts[x]), v) : 0;
    int tot;
    block_exscan(active, sh, &tot);
    active_tot += tot;
#pragma unroll
    for (int k = 0; k < AP_N; ++k) {
      const int pre = block_exscan(v[k], sh, &tot);
      if (x < ninst) ap[k * (ninst + 1) + x] = carry[k] + pre;
      carry[k] += tot;
    }
  }
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < AP_N; ++k) ap[k * (ninst + 1) + ninst] = carry[k];
    for (int k = 0; k < 4; ++k) gctr[G_TICKET + k] = 0;
    publish_active(gctr, hflag, active_tot);
  }
}

void launch_round_end(const LaunchCtx& c) {
  if (!c.ninst || c.fuse_end) return;
  hipLaunchKernelGGL(k_round_end, dim3(1), dim3(256), 0, c.stream, c.insts, c.ninst, c.gctr, c.hflag, c.ap);
}

// ------------------------------------------------------------------ widen
// kWidenBlocks workgroups per instance stride over its three arrays.
__global__ __launch_bounds__(256) void k_widen(const WidenJob* __restrict__ jobs) {
  const WidenJob J = jobs[blockIdx.x / kWidenBlocks];
  if (J.m <= 0) return;
  const int64_t t = (int64_t)(blockIdx.x % kWidenBlocks) * blockDim.x + threadIdx.x;
  const int64_t step = (int64_t)kWidenBlocks * blockDim.x;
  for (int64_t i = t; i <= J.m; i += step) J.dptr[i] = J.sptr[i];
  if (J.vtx16) {
    const uint16_t* sv = static_cast<const uint16_t*>(J.svtx);
    for (int64_t i = t; i < J.nnz; i += step) J.dvtx[i] = sv[i];
  } else {
    const int32_t* sv = static_cast<const int32_t*>(J.svtx);
    for (int64_t i = t; i < J.nnz; i += step) J.dvtx[i] = sv[i];
  }
  for (int64_t i = t; i < J.m; i += step) J.ddem[i] = J.sdem[i];
}

void launch_widen(hipStream_t stream, const WidenJob* jobs, int count) {
  if (count > 0)
    hipLaunchKernelGGL(k_widen, dim3((unsigned)count * kWidenBlocks), dim3(256), 0, stream, jobs);
}

// ------------------------------------------------------------------ gather
// One workgroup per instance writes its results where GatherLayout puts
// them (the caller's layout: arrays concatenated over the instances) and
// counts its kept hyperedges and vertices.
__global__ __launch_bounds__(256) void k_gather(const DInst* __restrict__ insts, const int64_t* ooff, int32_t* out,
                                                int ninst, GatherLayout g) {
  __shared__ int s_kept[2];
  const int x = blockIdx.x;
  const KInst I = kview(insts[x]);
  const int64_t mo = ooff[x], no = ooff[ninst + 1 + x];
  if (threadIdx.x < 2) s_kept[threadIdx.x] = 0;
  for (int i = threadIdx.x; i < kCtr; i += blockDim.x) out[g.ctr + (int64_t)x * kCtr + i] = I.ctr[i];
  __syncthreads();
  int km = 0, kn = 0;
  char* ob = reinterpret_cast<char*>(out);
  // one array element: int32, or uint16 when the layout is narrow
  auto put = [&](int64_t byte0, int64_t i, int v) {
    if (g.narrow) reinterpret_cast<uint16_t*>(ob + byte0)[i] = (uint16_t)v;
    else reinterpret_cast<int32_t*>(ob + byte0)[i] = v;
  };
  for (int i = threadIdx.x; i < I.m; i += blockDim.x) {
    const int d = I.death_e[i];
    put(g.de_b, mo + i, d);
    put(g.dem_b, mo + i, d ? 0 : I.fw[i]);
    km += d == 0;
  }
  uint8_t* fo = reinterpret_cast<uint8_t*>(ob + g.forced_b) + no;
  for (int i = threadIdx.x; i < I.n; i += blockDim.x) {
    const int d = I.death_v[i];
    put(g.dv_b, no + i, d);
    fo[i] = I.forced[i];
    kn += d == 0;
  }
  km = wave_sum(km);
  kn = wave_sum(kn);
  if (lane_id() == 0) {
    atomicAdd(&s_kept[0], km);
    atomicAdd(&s_kept[1], kn);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    out[g.kept + x] = s_kept[0];
    out[g.kept + ninst + x] = s_kept[1];
  }
}

void launch_gather(const LaunchCtx& c, const GatherLayout& g) {
  if (!c.ninst) return;
  hipLaunchKernelGGL(k_gather, dim3(c.ninst), dim3(256), 0, c.stream, c.insts, c.ooff, c.out, c.ninst, g);
}

// Sum over an instance's hyperedges of (last member - first member + 1), for
// the per-instance contraction choice of device-resident batches; one thread
// per hyperedge (prefix `ebp` over the instances' blocks of kBlock).
// Malformed hyperedges are skipped: the prepare step reports them.
__global__ __launch_bounds__(kBlock) void k_span(const DInst* __restrict__ insts, int ninst, const int32_t* ebp,
                                                 unsigned long long* spans) {
  __shared__ unsigned long long s_sum[kBlock / 64];
  const int x = unit_owner(ebp, ninst, blockIdx.x);
  const KInst I = kview(insts[x]);
  const int e = (blockIdx.x - ebp[x]) * kBlock + threadIdx.x;
  unsigned long long v = 0;
  if (e < I.m) {
    const int64_t a = I.eptr[e], b = I.eptr[e + 1];
    if (a >= 0 && b > a && b <= I.nnz) {
      const int lo = I.evtx[a], hi = I.evtx[b - 1];
      if (lo >= 0 && hi < I.n && hi >= lo) v = (unsigned long long)(hi - lo + 1);
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if (lane_id() == 0) s_sum[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int w = 0; w < kBlock / 64; ++w) t += s_sum[w];
    if (t) atomicAdd(&spans[x], t);
  }
}

void launch_span(const LaunchCtx& c, unsigned long long* spans) {
  if (!c.ninst || !c.n_eblocks) return;
  hipLaunchKernelGGL(k_span, dim3(c.n_eblocks), dim3(kBlock), 0, c.stream, c.insts, c.ninst, c.ebp, spans);
}

// Counters only: out + x * kCtr.
__global__ void k_gather_ctr(const DInst* __restrict__ insts, int ninst, int32_t* out) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ninst * kCtr) return;
  out[g] = insts[g / kCtr].ctr[g % kCtr];
}

void launch_gather_ctr(const LaunchCtx& c) {
  if (!c.ninst) return;
  hipLaunchKernelGGL(k_gather_ctr, dim3((c.ninst * kCtr + 255) / 256), dim3(256), 0, c.stream, c.insts,
                     c.ninst, c.out);
}

}  // namespace mhsk
