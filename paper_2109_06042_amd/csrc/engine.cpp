// engine.cpp -- host side of the round loop: workspace layout, set tables,
// hipGraph capture of one round, fixpoint loop, result readback.
#include "engine.h"
#include <atomic>
#include "host.h"

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>

namespace mhsk {

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

InstLayout inst_layout(int32_t n, int32_t m, int64_t nnz, bool stage_input, bool stage_compact) {
  InstLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o = align_up(o + std::max<size_t>(bytes, 16), 256);
    return r;
  };
  const size_t N = (size_t)n, M = (size_t)m, Z = (size_t)nnz;
  const size_t R = std::max(N, M);
  const size_t T = (R + kTile - 1) / kTile;
  const size_t B = (R + kBlock - 1) / kBlock;
  // results first: counters and death rounds are read back together
  L.off_ctr = take(kCtr * 4);
  L.off_death_e = take(M * 4);
  L.off_death_v = take(N * 4);
  L.off_forced = take(N);
  L.off_fw = take(M * 4);
  L.staged = stage_input;
  if (stage_input) {
    L.off_in_ptr = take((M + 1) * 8);
    L.off_in_vtx = take(Z * 4);
    L.off_in_dem = take(M * 4);
    if (stage_compact && m > 0) L.off_in_cmp = take(compact_layout(n, m, nnz).bytes);
  }
  L.off_vptr = take((N + 1) * 4);
  L.off_vedg = take(Z * 4);
  L.off_vend = take(N * 4);
  L.off_erow0 = take(M * 4);
  L.off_erow1 = take(M * 4);
  L.off_vrow0 = take(N * 4);
  L.off_vrow1 = take(N * 4);
  L.off_ecol = take(M * 4);
  L.off_vcol = take(N * 4);
  L.off_rs = take(R * 4);
  L.off_rf = take(R * 4);
  L.off_rid = take(R * 4);
  L.off_cnt = take(N * 4);
  L.off_kill = take(R);
  L.off_esz = take(M * 4);
  L.off_vdeg = take(N * 4);
  L.off_eslk = take(M);
  L.off_tkl = take(T * 4);
  L.off_tkh = take(T * 4);
  L.off_toff = take(T * 8);
  L.off_bstat = take(B * 8);
  const size_t te = (M + kTile - 1) / kTile, ce = (N + kChunk - 1) / kChunk;
  const size_t tv = (N + kTile - 1) / kTile, cv = (M + kChunk - 1) / kChunk;
  L.blob_cap = (int64_t)(std::max(te * ce, tv * cv) * (size_t)kChunkBytes);
  // the LDS prepare keeps its workgroups' offsets there before the first
  // round: 2 n ints per workgroup
  if (n <= kLocalN && m > 0) {
    const size_t G = (size_t)std::max<int64_t>(1, (nnz + kLocalChunk - 1) / kLocalChunk);
    L.blob_cap = std::max<int64_t>(L.blob_cap, (int64_t)(2 * N * G * 4));
  }
  // the sparse variant's round-1 class ends: kSlackClasses ints per vertex
  L.blob_cap = std::max<int64_t>(L.blob_cap, (int64_t)(N * kSlackClasses * 4));
  L.off_blob = take((size_t)L.blob_cap);
  L.bytes = o;
  return L;
}

size_t set_control_bytes(int32_t ninst) {
  const size_t X = (size_t)std::max(ninst, 1);
  size_t o = 0;
  o += align_up(X * sizeof(DInst), 256);
  o += 7 * align_up((X + 1) * 4, 256);
  o += align_up(AP_N * (X + 1) * 4, 256);
  o += align_up(G_N * 4, 256);
  o += align_up(2 * (X + 1) * 8, 256);
  o += align_up(X * kCtr * 4, 256);   // counter gather area
  return o;
}

DInst make_dinst(const HostInst& h) {
  DInst d;
  std::memset(&d, 0, sizeof(d));
  const InstLayout& L = h.L;
  char* s = h.slice;
  d.n = h.n;
  d.m = h.m;
  d.nnz = h.nnz;
  d.eptr = h.ptr;
  d.evtx = h.vtx;
  d.dem = h.dem;
  d.vptr = (int32_t*)(s + L.off_vptr);
  d.vedg = (int32_t*)(s + L.off_vedg);
  d.vend = (int32_t*)(s + L.off_vend);
  d.death_e = (int32_t*)(s + L.off_death_e);
  d.death_v = (int32_t*)(s + L.off_death_v);
  d.erow[0] = (int32_t*)(s + L.off_erow0);
  d.erow[1] = (int32_t*)(s + L.off_erow1);
  d.vrow[0] = (int32_t*)(s + L.off_vrow0);
  d.vrow[1] = (int32_t*)(s + L.off_vrow1);
  d.ecol = (int32_t*)(s + L.off_ecol);
  d.vcol = (int32_t*)(s + L.off_vcol);
  d.rs = (int32_t*)(s + L.off_rs);
  d.rf = (int32_t*)(s + L.off_rf);
  d.rid = (int32_t*)(s + L.off_rid);
  d.cnt = (int32_t*)(s + L.off_cnt);
  d.kill = (uint8_t*)(s + L.off_kill);
  d.esz = (int32_t*)(s + L.off_esz);
  d.vdeg = (int32_t*)(s + L.off_vdeg);
  d.eslk = (uint8_t*)(s + L.off_eslk);
  d.tkl = (int32_t*)(s + L.off_tkl);
  d.tkh = (int32_t*)(s + L.off_tkh);
  d.toff = (int64_t*)(s + L.off_toff);
  d.bstat = (uint64_t*)(s + L.off_bstat);
  d.blob = (int8_t*)(s + L.off_blob);
  d.blob_cap = L.blob_cap;
  d.ctr = (int32_t*)(s + L.off_ctr);
  d.fw = (int32_t*)(s + L.off_fw);
  d.forced = (uint8_t*)(s + L.off_forced);
  d.variant = h.variant;
  d.rule_se = h.rule_se;
  d.rule_fe = h.rule_fe;
  return d;
}

// ------------------------------------------------------------------ pinned
// Thread-local pinned staging buffer for device-to-host readback.
void* pinned_buffer(size_t bytes) {
  thread_local void* buf = nullptr;
  thread_local size_t cap = 0;
  if (bytes > cap) {
    if (buf) (void)hipHostFree(buf);
    buf = nullptr;
    size_t want = std::max(bytes, (size_t)1 << 20);
    if (hipHostMalloc(&buf, want, hipHostMallocDefault) != hipSuccess) { buf = nullptr; cap = 0; return nullptr; }
    cap = want;
  }
  return buf;
}

// Thread-local pinned staging buffer for host-to-device uploads (kept apart
// from the readback buffer: both are live within one call).
void* pinned_upload(size_t bytes) {
  thread_local void* buf = nullptr;
  thread_local size_t cap = 0;
  if (bytes > cap) {
    if (buf) (void)hipHostFree(buf);
    buf = nullptr;
    cap = 0;
    size_t want = std::max(bytes, (size_t)1 << 20);
    if (hipHostMalloc(&buf, want, hipHostMallocDefault) != hipSuccess) { buf = nullptr; return nullptr; }
    cap = want;
  }
  return buf;
}

// Thread-local pinned, host-mapped and coherent slots for the per-round
// "still active" counts, which the round-end kernel stores directly; kept
// apart from pinned_buffer, which may be reallocated.  *dev receives the
// device-side address.
int32_t* pinned_flags(int32_t** dev) {
  thread_local int32_t* buf = nullptr;
  thread_local int32_t* dbuf = nullptr;
  if (!buf) {
    void* p = nullptr;
    if (hipHostMalloc(&p, 256, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) return nullptr;
    void* d = nullptr;
    if (hipHostGetDevicePointer(&d, p, 0) != hipSuccess) {
      (void)hipHostFree(p);
      return nullptr;
    }
    buf = (int32_t*)p;
    dbuf = (int32_t*)d;
  }
  *dev = dbuf;
  return buf;
}

int device_cu_count() {
  // cached per device (a process may switch devices between calls)
  thread_local int last_dev = -1, last_cu = 256;
  int dev = 0, cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (dev == last_dev) return last_cu;
  if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0) cu = 256;
  last_dev = dev;
  last_cu = cu;
  return cu;
}

// ---------------------------------------------------------------------- Set
int Set::build(const std::vector<HostInst>& insts, char* control, size_t control_bytes,
               hipStream_t stream) {
  members = insts;
  const int32_t X = (int32_t)insts.size();
  if (control_bytes < set_control_bytes(X)) return set_error(MHS_ENOSPC, "control region too small");
  ctx = LaunchCtx();
  ctx.stream = stream;
  ctx.ninst = X;
  char* o = control;
  auto take = [&](size_t bytes) { char* r = o; o += align_up(std::max<size_t>(bytes, 16), 256); return r; };
  const size_t Xs = (size_t)std::max(X, 1);
  ctx.insts = (DInst*)take(Xs * sizeof(DInst));
  ctx.etp = (int32_t*)take((Xs + 1) * 4);
  ctx.vtp = (int32_t*)take((Xs + 1) * 4);
  ctx.ebp = (int32_t*)take((Xs + 1) * 4);
  ctx.vbp = (int32_t*)take((Xs + 1) * 4);
  ctx.lpb = (int32_t*)take((Xs + 1) * 4);
  ctx.gbp = (int32_t*)take((Xs + 1) * 4);
  ctx.ap = (int32_t*)take(AP_N * (Xs + 1) * 4);
  ctx.gctr = (int32_t*)take(G_N * 4);
  ctx.ooff = (int64_t*)take(2 * (Xs + 1) * 8);
  ctr_area = (int32_t*)take(Xs * kCtr * 4);

  h_dinst.resize(X);
  h_pref.assign((6 + AP_N) * (size_t)(X + 1), 0);
  h_ooff.resize(Xs);
  int32_t* etp = h_pref.data();
  int32_t* vtp = etp + (X + 1);
  int32_t* ebp = vtp + (X + 1);
  int32_t* vbp = ebp + (X + 1);
  int32_t* lpb = vbp + (X + 1);
  int32_t* gbp = lpb + (X + 1);
  int32_t* ap = gbp + (X + 1);   // AP_N arrays of X + 1
  max_n = max_m = 0;
  int32_t ctx_max_local_n = 0;
  int64_t pairs_e = 0, pairs_v = 0;   // contraction candidates, numbered in int32 across a set
  for (int32_t x = 0; x < X; ++x) {
    const HostInst& h = insts[x];
    h_dinst[x] = make_dinst(h);
    const bool lds = X > 1 && h.n <= kLocalN && h.m > 0;
    h_dinst[x].prep_lds = lds ? 1 : 0;
    lpb[x + 1] = lpb[x] + (lds ? (int32_t)std::max<int64_t>(1, (h.nnz + kLocalChunk - 1) / kLocalChunk) : 0);
    gbp[x + 1] = gbp[x] + (lds ? 0 : (h.m + kBlock - 1) / kBlock);
    if (lds) ctx_max_local_n = std::max(ctx_max_local_n, h.n);
    etp[x + 1] = etp[x] + (h.m + kTile - 1) / kTile;
    vtp[x + 1] = vtp[x] + (h.n + kTile - 1) / kTile;
    ebp[x + 1] = ebp[x] + (h.m + kBlock - 1) / kBlock;
    vbp[x + 1] = vbp[x] + (h.n + kBlock - 1) / kBlock;
    const bool sp = h.variant == 3;
    const int32_t te = (h.m + kTile - 1) / kTile, tv = (h.n + kTile - 1) / kTile;
    int32_t* a = ap;
    a[AP_ETD * (X + 1) + x + 1] = a[AP_ETD * (X + 1) + x] + (sp ? 0 : te);
    a[AP_VTD * (X + 1) + x + 1] = a[AP_VTD * (X + 1) + x] + (sp ? 0 : tv);
    a[AP_ETS * (X + 1) + x + 1] = a[AP_ETS * (X + 1) + x] + (sp ? te : 0);
    a[AP_VTS * (X + 1) + x + 1] = a[AP_VTS * (X + 1) + x] + (sp ? tv : 0);
    a[AP_EB * (X + 1) + x + 1] = a[AP_EB * (X + 1) + x] + std::max(1, (h.m + kBlock - 1) / kBlock);
    a[AP_VB * (X + 1) + x + 1] = a[AP_VB * (X + 1) + x] + std::max(1, (h.n + kBlock - 1) / kBlock);
    const int64_t pe = sp ? 0 : (int64_t)te * (te + 1) / 2, pv = sp ? 0 : (int64_t)tv * (tv + 1) / 2;
    pairs_e += pe;
    pairs_v += pv;
    a[AP_EP * (X + 1) + x + 1] = (int32_t)std::min<int64_t>(a[AP_EP * (X + 1) + x] + pe, INT32_MAX);
    a[AP_VP * (X + 1) + x + 1] = (int32_t)std::min<int64_t>(a[AP_VP * (X + 1) + x] + pv, INT32_MAX);
    h_ooff[x] = 0;
    max_n = std::max(max_n, h.n);
    max_m = std::max(max_m, h.m);
  }
  if (X > 1 && std::max(pairs_e, pairs_v) > INT32_MAX)
    return set_error(MHS_EINVAL, "a set's dense tile pairs exceed 2^31 per phase; split it or use the sparse variant");
  ctx.n_etiles = etp[X];
  ctx.n_vtiles = vtp[X];
  ctx.n_eblocks = ebp[X];
  ctx.n_vblocks = vbp[X];
  ctx.n_lblocks = lpb[X];
  ctx.n_gblocks = gbp[X];
  // the global-atomic prepare gives each hyperedge 64 lanes instead of 8
  // when those members' hyperedges have 32 entries or more on average
  {
    int64_t gm = 0, gz = 0;
    for (int32_t x = 0; x < X; ++x)
      if (!h_dinst[x].prep_lds) { gm += insts[x].m; gz += insts[x].nnz; }
    ctx.prep_long = (gm > 0 && gz >= 32 * gm) ? 1 : 0;
  }
  ctx.max_local_n = ctx_max_local_n;
  ctx.cus = device_cu_count();
  ctx.gemm_grid = ctx.cus * per_cu;
  ctx.variant = variant;
  ctx.has_dense = 0;
  ctx.has_sparse = 0;
  ctx.has_fe = 0;
  for (const HostInst& h : insts) {
    // a hyperedge's product terms are about nnz^2 / (n m) on average (the sum
    // of its vertices' degrees): one sparse instance above 256 takes the big
    // tables; sets keep the small ones, whose extra resident workgroups
    // measured faster on a mixed batch (its few members with many terms per
    // victim are counted one victim per wave or per workgroup either way)
    if (X == 1 && h.variant == 3 && h.n > 0 && h.m > 0 && (double)h.nnz * h.nnz > 256.0 * h.n * h.m)
      ctx.sparse_big = 1;
    if (h.variant == 3) ctx.has_sparse = 1;
    else ctx.has_dense = 1;
    if (h.rule_fe) ctx.has_fe = 1;
    if (h.rule_se) ctx.rule_se = 1;
  }
  // test knob: exercise the sparse variant's overflow path on every victim
  const char* fr = std::getenv("MHSK_SPARSE_FORCE_RANGE");
  ctx.sparse_force_range = (fr && fr[0] == '1') ? 1 : 0;
  // int8 contraction kernel: LDS-staged through registers (default), direct
  // fragment loads, or asynchronous global-to-LDS copies
  const char* gk = std::getenv("MHSK_GEMM");
  ctx.gemm_lds = 1;
  if (gk && std::strcmp(gk, "direct") == 0) ctx.gemm_lds = 0;
  if (gk && std::strcmp(gk, "async") == 0) ctx.gemm_lds = 2;
  // a staging the caller asked for (MHS_GEMM_SCHED) overrides the default
  if (gemm_sched == 0) ctx.gemm_lds = 1;
  if (gemm_sched == 1) ctx.gemm_lds = 0;
  if (gemm_sched == 2) ctx.gemm_lds = 2;
  ctx.fuse_end = (X == 1 && !ctx.has_fe) ? 1 : 0;
  ctx.count_work = profile ? 1 : 0;
  const char* rk = std::getenv("MHSK_ROUNDS_PER_LAUNCH");
  if (rk && rk[0] >= '1' && rk[0] <= '0' + kMaxRoundsPerLaunch && !rk[1]) rounds_per_launch = rk[0] - '0';
  // One upload of the whole table region (instance table, prefix arrays and
  // global counters, contiguous in the control block).  Global counters
  // start at zero in every new set: a set may be built over instances that
  // were prepared elsewhere (the server prepares newly admitted requests in
  // a set of their own), so nothing else clears them.
  const size_t image = (size_t)((char*)(ctx.gctr + G_N) - control);
  h_image.assign(image, 0);
  auto put = [&](const void* dst, const void* src, size_t bytes) {
    if (bytes) std::memcpy(h_image.data() + ((const char*)dst - control), src, bytes);
  };
  put(ctx.insts, h_dinst.data(), (size_t)X * sizeof(DInst));
  put(ctx.etp, etp, (size_t)(X + 1) * 4);
  put(ctx.vtp, vtp, (size_t)(X + 1) * 4);
  put(ctx.ebp, ebp, (size_t)(X + 1) * 4);
  put(ctx.vbp, vbp, (size_t)(X + 1) * 4);
  put(ctx.lpb, lpb, (size_t)(X + 1) * 4);
  put(ctx.gbp, gbp, (size_t)(X + 1) * 4);
  put(ctx.ap, ap, (size_t)AP_N * (X + 1) * 4);
  const void* src = h_image.data();
  if (stage && stage_bytes >= image) {
    std::memcpy(stage, h_image.data(), image);
    src = stage;
  }
  if (hipMemcpyAsync(control, src, image, hipMemcpyHostToDevice, stream) != hipSuccess)
    return set_error(MHS_EDEVICE, "table upload failed");
  return MHS_OK;
}

namespace {
// A second stream for the dense branch of a phase, with its fork and join
// events, per host thread and device (created on first use and kept, at the
// default priority).
struct AuxStream {
  int dev = -1;
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
thread_local AuxStream g_aux;
AuxStream* aux_stream() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  if (g_aux.s && g_aux.dev == dev) return &g_aux;
  AuxStream a;
  if (hipStreamCreateWithFlags(&a.s, hipStreamNonBlocking) != hipSuccess) return nullptr;
  if (hipEventCreateWithFlags(&a.fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&a.join, hipEventDisableTiming) != hipSuccess) {
    if (a.fork) (void)hipEventDestroy(a.fork);
    (void)hipStreamDestroy(a.s);
    return nullptr;
  }
  a.dev = dev;
  g_aux = a;   // a stream of another device, if any, is left as it is
  return &g_aux;
}
}  // namespace

// Sets with sparse and dense members run each phase's two branches
// concurrently: the sparse rows and counts on the set's stream, the dense
// rows and contraction on the auxiliary one (they touch disjoint members and
// only read the shared tables); the compaction waits for both.  Profiled
// runs keep them in order, for their per-step events.
bool Set::split_branches() const { return ctx.has_sparse && ctx.has_dense && !profile && ctx.ninst > 1; }

void Set::launch_round_direct() {
  // profiling: a bounded device-side delay lets the host enqueue the whole
  // round first, then one event per step boundary
  if (profile) {
    int rate_khz = 0, dev = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || rate_khz <= 0)
      rate_khz = 100000;
    launch_delay(ctx.stream, (long long)rate_khz / 5);   // 200 us
  }
  auto mark = [&]() { if (profile) (void)hipEventRecord(ev_pool.get(ev_used++), ctx.stream); };
  mark();
  AuxStream* aux = split_branches() ? aux_stream() : nullptr;
  for (int v = 0; v < 2; ++v) {
    if (aux) {
      LaunchCtx cb = ctx;
      cb.stream = aux->s;
      (void)hipEventRecord(aux->fork, ctx.stream);
      (void)hipStreamWaitEvent(aux->s, aux->fork, 0);
      // the dense branch is queued first: its rows kernel takes whole
      // workgroups of 1024 threads, which find no room once the sparse
      // count's many small workgroups hold the compute units
      launch_rows_dense(cb, v == 1);
      launch_contraction_dense(cb, v == 1);
      launch_rows_sparse(ctx, v == 1);
      launch_contraction_sparse(ctx, v == 1);
      (void)hipEventRecord(aux->join, aux->s);
      (void)hipStreamWaitEvent(ctx.stream, aux->join, 0);
    } else {
      launch_rows(ctx, v == 1);
      mark();
      launch_contraction_sparse(ctx, v == 1);
      mark();
      launch_contraction_dense(ctx, v == 1);
      mark();
    }
    launch_compact(ctx, v == 1);
    mark();
  }
  launch_fe(ctx);
  launch_round_end(ctx);
  mark();
}

// Instantiated round graphs, keyed by every kernel argument of a round.
// Kernel arguments are device pointers into the caller's workspace plus
// grid sizes, so two calls with the same workspace and instance shapes share
// one graph; the instance data itself is read from device memory.
namespace {
struct GraphKey {
  DInst* insts;
  int32_t* etp;
  int32_t* vtp;
  int32_t* ebp;
  int32_t* vbp;
  int32_t* gctr;
  int32_t* hflag;
  int32_t* ap;
  int32_t ninst, n_etiles, n_vtiles, n_eblocks, n_vblocks, gemm_grid, variant, force_range, gemm_lds, has_dense, has_sparse, has_fe,
      rule_se, cus, fuse_end, count_work, sparse_big, rounds;
  bool operator==(const GraphKey& o) const { return std::memcmp(this, &o, sizeof(GraphKey)) == 0; }
};
GraphKey key_of(const LaunchCtx& c) {
  GraphKey k;
  std::memset(&k, 0, sizeof(k));
  k.insts = c.insts; k.etp = c.etp; k.vtp = c.vtp; k.ebp = c.ebp; k.vbp = c.vbp;
  k.gctr = c.gctr; k.hflag = c.hflag; k.ap = c.ap;
  k.ninst = c.ninst; k.n_etiles = c.n_etiles; k.n_vtiles = c.n_vtiles;
  k.n_eblocks = c.n_eblocks; k.n_vblocks = c.n_vblocks; k.gemm_grid = c.gemm_grid;
  k.variant = c.variant;
  k.force_range = c.sparse_force_range;
  k.gemm_lds = c.gemm_lds;
  k.has_dense = c.has_dense;
  k.has_sparse = c.has_sparse;
  k.has_fe = c.has_fe;
  k.rule_se = c.rule_se;
  k.cus = c.cus;
  k.count_work = c.count_work;
  k.fuse_end = c.fuse_end;
  k.sparse_big = c.sparse_big;
  return k;
}
struct GraphCache {
  struct Entry { GraphKey key; hipGraphExec_t exec; uint64_t used; };
  std::vector<Entry> entries;
  uint64_t clock = 0;
  hipGraphExec_t find(const GraphKey& k) {
    for (Entry& e : entries) if (e.key == k) { e.used = ++clock; return e.exec; }
    return nullptr;
  }
  void put(const GraphKey& k, hipGraphExec_t g) {
    if (entries.size() >= 8) {
      size_t old = 0;
      for (size_t i = 1; i < entries.size(); ++i) if (entries[i].used < entries[old].used) old = i;
      (void)hipGraphExecDestroy(entries[old].exec);
      entries.erase(entries.begin() + old);
    }
    entries.push_back({k, g, ++clock});
  }
};
thread_local GraphCache g_graphs;
}  // namespace

int Set::launch_rounds(bool use_graph, int k) {
  // the legacy default stream cannot be captured: launch directly there
  if (!use_graph || profile || ctx.stream == nullptr) {
    for (int i = 0; i < k; ++i) launch_round_direct();
    return hipGetLastError() == hipSuccess ? MHS_OK : set_error(MHS_EDEVICE, "kernel launch failed");
  }
  // the auxiliary stream exists before a capture begins
  if (split_branches() && !aux_stream()) return set_error(MHS_EDEVICE, "auxiliary stream creation failed");
  GraphKey key = key_of(ctx);
  key.rounds = k;
  hipGraphExec_t exec = g_graphs.find(key);
  if (!exec) {
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(ctx.stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return set_error(MHS_EDEVICE, "stream capture failed");
    for (int i = 0; i < k; ++i) launch_round_direct();
    if (hipStreamEndCapture(ctx.stream, &g) != hipSuccess || !g) return set_error(MHS_EDEVICE, "end capture failed");
    hipError_t e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return set_error(MHS_EDEVICE, "graph instantiate failed");
    g_graphs.put(key, exec);
  }
  if (hipGraphLaunch(exec, ctx.stream) != hipSuccess) return set_error(MHS_EDEVICE, "graph launch failed");
  return MHS_OK;
}

Set::~Set() {}

// Fixpoint loop of Algorithm 3 with the host one launch behind the device:
// launch u+1 (k rounds; one graph when graphs are used) is queued before the
// host waits for the last round of launch u, so the device never idles on
// the host.  Rounds queued after the last productive one find every instance
// done and do no work.  Round r's end stores (r, active count) into
// host-mapped slot r mod kFlagSlots, which the host polls: no event or copy
// is queued between rounds.  A stream that went idle (or failed) without
// publishing the round is an error.
int Set::run_to_fixpoint(bool use_graph, int64_t max_iter, int32_t* iters) {
  int32_t* dslot = nullptr;
  volatile int32_t* slot = pinned_flags(&dslot);
  if (!slot) return set_error(MHS_EDEVICE, "pinned allocation failed");
  // The prepare step zeroed G_RSEQ, so round r (from 1) publishes sequence
  // number r; at most 2k consecutive rounds are in flight while the host
  // reads one of them.  A write still due from an earlier call's last
  // queued rounds carries a number this call has not reached or has already
  // passed.
  for (int i = 0; i < 2 * kFlagSlots; ++i) slot[i] = 0;
  ctx.hflag = dslot;
  const bool speculate = !profile;
  const int k = (use_graph && !profile) ? std::max(1, std::min(rounds_per_launch, kMaxRoundsPerLaunch)) : 1;
  auto wait_round = [&](int64_t r, int* active) -> int {
    volatile int32_t* s = slot + 2 * (r % kFlagSlots);
    for (uint64_t spin = 1;; ++spin) {
      if (s[0] == (int32_t)r) {
        std::atomic_thread_fence(std::memory_order_acquire);
        *active = s[1];
        return MHS_OK;
      }
      if ((spin & 255) == 0) {
        const hipError_t q = hipStreamQuery(ctx.stream);
        if (q == hipSuccess && s[0] != (int32_t)r) {
          std::string seen;
          for (int i = 0; i < kFlagSlots; ++i) seen += " " + std::to_string(slot[2 * i]);
          return set_error(MHS_EDEVICE, "round " + std::to_string(r) + " ended without its result (slots hold rounds" +
                                            seen + ")");
        }
        if (q != hipSuccess && q != hipErrorNotReady) return set_error(MHS_EDEVICE, "round failed");
      }
    }
  };
  int64_t queued = 0;   // rounds queued so far
  auto enqueue = [&]() -> int {
    if (queued + k > max_iter + 2 * k) return set_error(MHS_EDEVICE, "iteration bound exceeded");
    queued += k;
    return launch_rounds(use_graph, k);
  };
  int rc = enqueue();
  if (rc) return rc;
  int64_t r = k;        // the round waited for: the last of the oldest unread launch
  for (;;) {
    if (speculate) {
      rc = enqueue();
      if (rc) return rc;
    }
    int any = 0;
    rc = wait_round(r, &any);
    if (rc) return rc;
    if (!any) break;
    r += k;
    if (!speculate) {
      rc = enqueue();
      if (rc) return rc;
    }
  }
  *iters = (int32_t)r;
  return MHS_OK;
}

int Set::read_any(int* any) {
  int32_t* p = (int32_t*)pinned_buffer(64);
  if (!p) return set_error(MHS_EDEVICE, "pinned allocation failed");
  if (hipMemcpyAsync(p, ctx.gctr + G_ANY, 4, hipMemcpyDeviceToHost, ctx.stream) != hipSuccess ||
      hipStreamSynchronize(ctx.stream) != hipSuccess)
    return set_error(MHS_EDEVICE, "readback failed");
  *any = p[0];
  return MHS_OK;
}

// Counters of every member (one gather kernel, one copy).
int Set::read_counters(std::vector<int32_t>& out) {
  const int32_t X = ctx.ninst;
  out.assign((size_t)X * kCtr, 0);
  if (!X) return MHS_OK;
  LaunchCtx c = ctx;
  c.out = ctr_area;
  launch_gather_ctr(c);
  int32_t* p = (int32_t*)pinned_buffer((size_t)X * kCtr * 4);
  if (!p) return set_error(MHS_EDEVICE, "pinned allocation failed");
  if (hipMemcpyAsync(p, ctr_area, (size_t)X * kCtr * 4, hipMemcpyDeviceToHost, ctx.stream) != hipSuccess ||
      hipStreamSynchronize(ctx.stream) != hipSuccess)
    return set_error(MHS_EDEVICE, "counter readback failed");
  std::memcpy(out.data(), p, (size_t)X * kCtr * 4);
  return MHS_OK;
}

int Set::enqueue_counters(int32_t* dst) {
  const int32_t X = ctx.ninst;
  if (!X) return MHS_OK;
  LaunchCtx c = ctx;
  c.out = ctr_area;
  launch_gather_ctr(c);
  if (hipMemcpyAsync(dst, ctr_area, (size_t)X * kCtr * 4, hipMemcpyDeviceToHost, ctx.stream) != hipSuccess)
    return set_error(MHS_EDEVICE, "counter readback failed");
  return MHS_OK;
}

// Copy one member's counters and death rounds (contiguous at its slice start).
int Set::read_member(int32_t x, std::vector<int32_t>& ctr, std::vector<int32_t>& de,
                     std::vector<int32_t>& dv, std::vector<uint8_t>* forced, std::vector<int32_t>* fw) {
  const HostInst& h = members[x];
  const size_t bytes = h.L.off_fw + (size_t)h.m * 4;
  char* p = (char*)pinned_buffer(bytes);
  if (!p) return set_error(MHS_EDEVICE, "pinned allocation failed");
  if (hipMemcpyAsync(p, h.slice, bytes, hipMemcpyDeviceToHost, ctx.stream) != hipSuccess ||
      hipStreamSynchronize(ctx.stream) != hipSuccess)
    return set_error(MHS_EDEVICE, "result readback failed");
  ctr.assign((int32_t*)(p + h.L.off_ctr), (int32_t*)(p + h.L.off_ctr) + kCtr);
  de.assign((int32_t*)(p + h.L.off_death_e), (int32_t*)(p + h.L.off_death_e) + h.m);
  dv.assign((int32_t*)(p + h.L.off_death_v), (int32_t*)(p + h.L.off_death_v) + h.n);
  if (forced) forced->assign((uint8_t*)(p + h.L.off_forced), (uint8_t*)(p + h.L.off_forced) + h.n);
  if (fw) fw->assign((int32_t*)(p + h.L.off_fw), (int32_t*)(p + h.L.off_fw) + h.m);
  return MHS_OK;
}

// Events collected during a profiled run -> time per step.  Per round the
// marks are: start | rows_E | sparse_E | dense_E | compact_E | rows_V
// | sparse_V | dense_V | compact_V | round_end.
void Set::collect_profile(double* step_ms) {
  for (int k = 0; k < kSteps; ++k) step_ms[k] = 0.0;
  const int per_round = 10;
  for (int base = 0; base + per_round <= ev_used; base += per_round) {
    float d[per_round - 1];
    for (int i = 0; i + 1 < per_round; ++i) {
      d[i] = 0.f;
      (void)hipEventElapsedTime(&d[i], ev_pool.get(base + i), ev_pool.get(base + i + 1));
    }
    step_ms[STEP_ROWS] += d[0] + d[4];
    step_ms[STEP_SPARSE_E] += d[1];
    step_ms[STEP_GEMM_E] += d[2];
    step_ms[STEP_SPARSE_V] += d[5];
    step_ms[STEP_GEMM_V] += d[6];
    step_ms[STEP_COMPACT] += d[3] + d[7];
    step_ms[STEP_ROUND_END] += d[8];
  }
  ev_used = 0;
}

hipEvent_t EventPool::get(int i) {
  while ((int)ev.size() <= i) {
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    ev.push_back(e);
  }
  return ev[i];
}

EventPool::~EventPool() {
  for (hipEvent_t e : ev) if (e) (void)hipEventDestroy(e);
}

}  // namespace mhsk
