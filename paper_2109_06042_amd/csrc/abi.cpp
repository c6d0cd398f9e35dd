// abi.cpp -- the C ABI (include/mhsk.h): argument checks, host validation,
// workspace carving, the fixpoint loop, result objects.
#include "host.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <cstring>
#include <map>
#include <atomic>
#include <functional>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

using namespace mhsk;

struct mhs_result {
  int32_t n = 0, m = 0;
  int64_t k = 0;
  int32_t rounds = 0;
  int32_t n_forced = 0;
  std::vector<int32_t> death_e, death_v;
  std::vector<int32_t> demand;      // demands at the end (0 for deleted hyperedges)
  std::vector<uint8_t> forced;      // forced into the solution (full-edge rule)
  mhs_stats stats;
  int32_t status = 0;               // MHS_OK, or why the server could not finish the request
  std::string error;                // message of a failed request
};

namespace mhsk {

thread_local std::string g_err;

int set_error(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// A pool of host threads (up to 15 besides the caller, started on first
// use) that runs parallel_for's items; the caller works on its own job too
// and returns when every item has run.  Jobs from several threads may be
// queued at once.
namespace {
class Pool {
 public:
  static Pool& get() {
    static Pool p;
    return p;
  }
  int threads() const { return (int)th_.size() + 1; }
  void run(int32_t count, const std::function<void(int32_t)>& f) {
    Job job;
    job.f = &f;
    job.count = count;
    {
      std::lock_guard<std::mutex> g(mu_);
      q_.push_back(&job);
    }
    cv_.notify_all();
    job.work();
    {
      // no worker takes the job from here on; wait for those that did
      std::lock_guard<std::mutex> g(mu_);
      for (auto it = q_.begin(); it != q_.end(); ++it)
        if (*it == &job) { q_.erase(it); break; }
    }
    while (job.done.load(std::memory_order_acquire) < count || job.users.load(std::memory_order_acquire) > 0)
      std::this_thread::yield();
  }
  ~Pool() {
    {
      std::lock_guard<std::mutex> g(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    for (std::thread& t : th_) t.join();
  }

 private:
  struct Job {
    const std::function<void(int32_t)>* f = nullptr;
    int32_t count = 0;
    std::atomic<int32_t> next{0}, done{0}, users{0};
    void work() {
      for (;;) {
        const int32_t i = next.fetch_add(1);
        if (i >= count) break;
        (*f)(i);
        done.fetch_add(1, std::memory_order_release);
      }
    }
  };
  Pool() {
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int T = (int)std::min<unsigned>(16u, hw);
    for (int t = 1; t < T; ++t) th_.emplace_back([this] { loop(); });
  }
  void loop() {
    for (;;) {
      Job* j = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return stop_ || !q_.empty(); });
        if (stop_) return;
        j = q_.front();
        j->users.fetch_add(1);
        // a job whose items are all taken leaves the queue
        if (j->next.load() >= j->count) q_.pop_front();
      }
      j->work();
      j->users.fetch_sub(1, std::memory_order_release);
    }
  }
  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<Job*> q_;
  std::vector<std::thread> th_;
  bool stop_ = false;
};
}  // namespace

// Runs f(0..count-1) on the pool's threads (inline for small counts).
void parallel_for(int32_t count, const std::function<void(int32_t)>& f) {
  if (count < 4 || Pool::get().threads() < 2) {
    for (int32_t i = 0; i < count; ++i) f(i);
    return;
  }
  Pool::get().run(count, f);
}

// Sizes and pointers of a host instance (reads edge_ptr[0] and edge_ptr[m]
// only); *nnz_out receives edge_ptr[m].
int validate_shape(const mhs_instance* in, int64_t* nnz_out, std::string* why) {
  const int32_t n = in->n, m = in->m;
  if (n < 0 || m < 0) { *why = "negative n or m"; return E_PTR; }
  if (m == 0) { *nnz_out = 0; return 0; }
  if (!in->edge_ptr || !in->demand) { *why = "NULL edge_ptr or demand"; return E_PTR; }
  if (in->edge_ptr[0] != 0) { *why = "edge_ptr[0] != 0"; return E_PTR; }
  const int64_t nnz = in->edge_ptr[m];
  if (nnz < 0 || nnz >= ((int64_t)1 << 31)) { *why = "nnz out of range"; return E_PTR; }
  if (nnz > 0 && !in->edge_vtx) { *why = "NULL edge_vtx"; return E_PTR; }
  *nnz_out = nnz;
  return 0;
}

// Every hyperedge of an instance that passed validate_shape: pointers,
// vertex ids, order and demands.
static int validate_body(const mhs_instance* in, int64_t nnz, std::string* why) {
  const int32_t n = in->n, m = in->m;
  for (int32_t e = 0; e < m; ++e) {
    const int64_t a = in->edge_ptr[e], b = in->edge_ptr[e + 1];
    if (b < a || b > nnz) { *why = "edge_ptr not nondecreasing at hyperedge " + std::to_string(e); return E_PTR; }
    if (b == a) { *why = "empty hyperedge " + std::to_string(e); return E_EMPTY; }
    for (int64_t p = a; p < b; ++p) {
      const int32_t v = in->edge_vtx[p];
      if (v < 0 || v >= n) { *why = "vertex id out of range in hyperedge " + std::to_string(e); return E_RANGE; }
      if (p > a && v <= in->edge_vtx[p - 1]) {
        *why = "hyperedge " + std::to_string(e) + " not strictly increasing";
        return E_ORDER;
      }
    }
    const int32_t d = in->demand[e];
    if (d < 1 || (int64_t)d > b - a) { *why = "demand of hyperedge " + std::to_string(e) + " outside [1, |e|]"; return E_DEMAND; }
  }
  return 0;
}

static int validate_host(const mhs_instance* in, int64_t* nnz_out, std::string* why) {
  int64_t nnz = 0;
  if (int c = validate_shape(in, &nnz, why)) return c;
  if (int c = validate_body(in, nnz, why)) return c;
  *nnz_out = nnz;
  return 0;
}

int variant_of(uint32_t flags) {
  const uint32_t v = flags & MHS_VARIANT_MASK;
  return v == MHS_VARIANT_BITSET ? 2 : v == MHS_VARIANT_SPARSE ? 3 : 1;
}

// Per-instance contraction variant.  Explicit variants apply to every
// instance; HYBRID (and AUTO without a tuned class) takes dense MFMA tiles
// for instances whose hyperedges are local in vertex id (mean span below 5%
// of n: the tiles are banded and most tile pairs are skipped) and sparse
// counting otherwise.  Device-resident inputs are not inspected on the
// host: they take int8.
// The rule above, given the sum over hyperedges of (last id - first id + 1).
int variant_with_span(uint32_t flags, const mhs_instance* in, double span) {
  // dense tiles encode counts below 2^29 in their epilogue: larger instances
  // (far beyond any dense blob that fits a device) count sparsely
  if (std::max(in->n, in->m) >= (1 << 29)) return 3;
  const uint32_t v = flags & MHS_VARIANT_MASK;
  if (v != MHS_VARIANT_AUTO && v != MHS_VARIANT_HYBRID) return variant_of(flags);
  if ((flags & MHS_INPUT_DEVICE) || in->m == 0 || in->n == 0 || !in->edge_ptr || !in->edge_vtx) return 1;
  return span / ((double)in->m * in->n) > 0.05 ? 3 : 1;
}

static bool variant_needs_span(uint32_t flags, const mhs_instance* in) {
  const uint32_t v = flags & MHS_VARIANT_MASK;
  return std::max(in->n, in->m) < (1 << 29) && (v == MHS_VARIANT_AUTO || v == MHS_VARIANT_HYBRID) &&
         !(flags & MHS_INPUT_DEVICE) && in->m > 0 && in->n > 0 && in->edge_ptr && in->edge_vtx;
}

int instance_variant(uint32_t flags, const mhs_instance* in) {
  double span = 0;
  if (variant_needs_span(flags, in))
    for (int32_t e = 0; e < in->m; ++e) {
      const int64_t a = in->edge_ptr[e], b = in->edge_ptr[e + 1];
      if (b > a) span += (double)(in->edge_vtx[b - 1] - in->edge_vtx[a] + 1);
    }
  return variant_with_span(flags, in, span);
}

int gemm_sched_of(uint32_t flags) {
  return (int)((flags & MHS_GEMM_SCHED_MASK) >> 20) - 1;
}

int grid_per_cu(uint32_t flags) {
  const uint32_t g = (flags & MHS_GRID_MASK) >> 24;
  return g ? (1 << (g - 1)) : 4;
}

// ------------------------------------------------------------- autotuning
// Size class of a set of instances: log2 of the mean hyperedge count, mean
// hyperedge size and vertex count, rounded.
typedef std::tuple<int, int, int> SizeClass;

static SizeClass size_class(const mhs_instance* insts, int32_t count, bool device) {
  double m = 0, n = 0, z = 0;
  for (int32_t i = 0; i < count; ++i) {
    m += insts[i].m;
    n += insts[i].n;
    // device instances: the nnz they carry (their edge_ptr is not readable here)
    if (insts[i].m > 0 && device) z += (double)std::max<int64_t>(insts[i].nnz, 0);
    else if (insts[i].m > 0 && insts[i].edge_ptr) z += (double)insts[i].edge_ptr[insts[i].m];
  }
  auto l2 = [](double v) { return v > 0 ? (int)std::lround(std::log2(v)) : -1; };
  return SizeClass(l2(m / std::max(count, 1)), l2(m > 0 ? z / m : 0), l2(n / std::max(count, 1)));
}

static std::mutex g_tune_mu;
static std::map<SizeClass, uint32_t> g_tuned;

// MHS_VARIANT_AUTO: the tuned variant and grid of the class, else the default.
static uint32_t resolve_auto(uint32_t flags, const mhs_instance* insts, int32_t count) {
  if ((flags & MHS_VARIANT_MASK) != MHS_VARIANT_AUTO) return flags;
  const SizeClass c = size_class(insts, count, (flags & MHS_INPUT_DEVICE) != 0);
  std::lock_guard<std::mutex> g(g_tune_mu);
  auto it = g_tuned.find(c);
  if (it == g_tuned.end()) return flags;
  return (flags & ~(MHS_VARIANT_MASK | MHS_GRID_MASK | MHS_GEMM_SCHED_MASK)) | it->second;
}

static const char* err_name(int code) {
  switch (code) {
    case E_PTR: return "malformed edge_ptr";
    case E_RANGE: return "vertex id out of range";
    case E_ORDER: return "hyperedge not strictly increasing";
    case E_EMPTY: return "empty hyperedge";
    case E_DEMAND: return "demand outside [1, |e|]";
    case E_CAPACITY: return "internal capacity exceeded";
    case E_STALL: return "internal: compaction look-back did not complete";
    default: return "invalid instance";
  }
}

static int check_flags(uint32_t flags) {
  const uint32_t v = flags & MHS_VARIANT_MASK;
  if (v > MHS_VARIANT_HYBRID) return set_error(MHS_EINVAL, "unknown contraction variant");
  const uint32_t known = MHS_VARIANT_MASK | MHS_TRACE_ROUNDS | MHS_INPUT_DEVICE | MHS_NO_GRAPH | MHS_GRAPH |
                         MHS_PROFILE | MHS_GRID_MASK | MHS_GEMM_SCHED_MASK | MHS_RULE_SE | MHS_RULE_FE;
  if (flags & ~known) return set_error(MHS_EINVAL, "unknown flag bits");
  if ((flags & MHS_GRAPH) && (flags & MHS_NO_GRAPH)) return set_error(MHS_EINVAL, "MHS_GRAPH with MHS_NO_GRAPH");
  if (((flags & MHS_GRID_MASK) >> 24) > 5) return set_error(MHS_EINVAL, "grid exponent above 4");
  return MHS_OK;
}

// nnz of an instance (host or device edge_ptr) plus host validation.
static int instance_nnz(const mhs_instance* in, uint32_t flags, int64_t* nnz, hipStream_t stream) {
  if (!in) return set_error(MHS_EINVAL, "NULL instance");
  if (in->n < 0 || in->m < 0) return set_error(MHS_EINVAL, "negative n or m");
  if (!(flags & MHS_INPUT_DEVICE)) {
    std::string why;
    if (validate_host(in, nnz, &why)) return set_error(MHS_EINVAL, why);
    return MHS_OK;
  }
  if (in->m == 0) { *nnz = 0; return MHS_OK; }
  if (!in->edge_ptr || !in->edge_vtx || !in->demand) return set_error(MHS_EINVAL, "NULL device array");
  if (in->nnz > 0) {
    // the device-side validation checks edge_ptr against this value
    if (in->nnz >= ((int64_t)1 << 31)) return set_error(MHS_EINVAL, "nnz out of range");
    *nnz = in->nnz;
    return MHS_OK;
  }
  int64_t* p = (int64_t*)pinned_buffer(64);
  if (!p) return set_error(MHS_EDEVICE, "pinned allocation failed");
  if (hipMemcpyAsync(p, in->edge_ptr + in->m, 8, hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return set_error(MHS_EDEVICE, "cannot read edge_ptr[m] from device");
  *nnz = p[0];
  if (*nnz < 0 || *nnz >= ((int64_t)1 << 31)) return set_error(MHS_EINVAL, "nnz out of range");
  return MHS_OK;
}

// Stage a host instance into its slice (or point at the caller's device arrays).
static int bind_input(HostInst& h, const mhs_instance* in, uint32_t flags, hipStream_t stream) {
  if (flags & MHS_INPUT_DEVICE) {
    h.ptr = in->edge_ptr;
    h.vtx = in->edge_vtx;
    h.dem = in->demand;
    return MHS_OK;
  }
  int64_t* dptr = (int64_t*)(h.slice + h.L.off_in_ptr);
  int32_t* dvtx = (int32_t*)(h.slice + h.L.off_in_vtx);
  int32_t* ddem = (int32_t*)(h.slice + h.L.off_in_dem);
  hipError_t e = hipSuccess;
  if (h.m > 0) {
    e = hipMemcpyAsync(dptr, in->edge_ptr, (size_t)(h.m + 1) * 8, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && h.nnz > 0)
      e = hipMemcpyAsync(dvtx, in->edge_vtx, (size_t)h.nnz * 4, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(ddem, in->demand, (size_t)h.m * 4, hipMemcpyHostToDevice, stream);
  }
  if (e != hipSuccess) return set_error(MHS_EDEVICE, "input upload failed");
  h.ptr = dptr;
  h.vtx = dvtx;
  h.dem = ddem;
  return MHS_OK;
}

// Fixpoint loop of Algorithm 3 over a built set.  Returns the number of
// iterations executed in *iters.
static int run_rounds(Set& S, uint32_t flags, int32_t* iters) {
  launch_prepare(S.ctx);
  if (hipGetLastError() != hipSuccess) return set_error(MHS_EDEVICE, "prepare launch failed");
  int64_t max_iter = 2;
  for (const HostInst& h : S.members) max_iter = std::max<int64_t>(max_iter, (int64_t)std::min(h.n, h.m) + 2);
  // graph replay by request, else for sets of several instances only
  const bool graph = (flags & MHS_GRAPH) || (!(flags & MHS_NO_GRAPH) && S.ctx.ninst > 1);
  return S.run_to_fixpoint(graph, max_iter, iters);
}

// Work counters of one instance from its counter words.
static void stats_from_counters(const int32_t* ctr, mhs_stats* st) {
  std::memset(st, 0, sizeof(*st));
  auto c64 = [&](int i) { long long v; std::memcpy(&v, &ctr[i], 8); return (double)v; };
  const double per_chunk = 2.0 * kTile * kTile * kChunk;   // MFMA ops per item chunk
  st->iterations = ctr[C_ROUND];
  st->edge_issued_ops = c64(C_CHUNKS_SUM_E) * per_chunk;
  st->vertex_issued_ops = c64(C_CHUNKS_SUM_V) * per_chunk;
  st->issued_ops = st->edge_issued_ops + st->vertex_issued_ops;
  st->blob_bytes = c64(C_BLOB_SUM);
  st->terms = c64(C_PAIRS_SUM);
  st->encode_bytes = 37.0 * c64(C_ROWS_SUM) + 8.0 * c64(C_ENTRIES_SUM) + c64(C_BLOB_SUM);
}

static mhs_result* make_result(const HostInst& h, const std::vector<int32_t>& ctr,
                               std::vector<int32_t>&& de, std::vector<int32_t>&& dv,
                               std::vector<int32_t>&& fw, std::vector<uint8_t>&& forced) {
  mhs_result* r = new mhs_result();
  r->n = h.n;
  r->m = h.m;
  r->k = h.k;
  r->rounds = ctr[C_ROUNDS];
  r->n_forced = ctr[C_NFORCED];
  r->death_e = std::move(de);
  r->death_v = std::move(dv);
  r->demand = std::move(fw);
  r->forced = std::move(forced);
  r->demand.resize(h.m, 0);
  r->forced.resize(h.n, 0);
  for (int32_t e = 0; e < h.m; ++e)
    if (r->death_e[e]) r->demand[e] = 0;
  stats_from_counters(ctr.data(), &r->stats);
  return r;
}

static void fill_profile(Set& S, mhs_stats* st) {
  double step[Set::kSteps];
  S.collect_profile(step);
  st->rows_ms = step[Set::STEP_ROWS];
  st->edge_sparse_ms = step[Set::STEP_SPARSE_E];
  st->vertex_sparse_ms = step[Set::STEP_SPARSE_V];
  st->sparse_ms = st->edge_sparse_ms + st->vertex_sparse_ms;
  st->edge_gemm_ms = step[Set::STEP_GEMM_E] + st->edge_sparse_ms;
  st->vertex_gemm_ms = step[Set::STEP_GEMM_V] + st->vertex_sparse_ms;
  st->gemm_ms = st->edge_gemm_ms + st->vertex_gemm_ms;
  st->compact_ms = step[Set::STEP_COMPACT];
  st->round_end_ms = step[Set::STEP_ROUND_END];
}

// A request the server could not reduce: the device reported error `code`
// (C_ERR) for it.
mhs_result* make_failed_result(const HostInst& h, int code) {
  mhs_result* r = new mhs_result();
  r->n = h.n;
  r->m = h.m;
  r->k = h.k;
  r->status = code == E_CAPACITY ? MHS_ENOSPC : code == E_STALL ? MHS_EDEVICE : MHS_EINVAL;
  r->error = err_name(code);
  std::memset(&r->stats, 0, sizeof(r->stats));
  return r;
}

mhs_result* make_result_public(const HostInst& h, const std::vector<int32_t>& ctr, std::vector<int32_t>&& de,
                               std::vector<int32_t>&& dv, std::vector<int32_t>&& fw,
                               std::vector<uint8_t>&& forced) {
  return make_result(h, ctr, std::move(de), std::move(dv), std::move(fw), std::move(forced));
}

int validate_host_public(const mhs_instance* in, int64_t* nnz, std::string* why) {
  if (!in) { *why = "NULL instance"; return E_PTR; }
  return validate_host(in, nnz, why);
}

// mhs_run over a workspace without any allocation (no pinned staging, no
// host-mapped round slots, no events, no graphs): rounds are launched one at
// a time and the active count is read into host memory after each, and the
// results are copied straight into the caller's arrays.  `ws` is device
// memory of ws_bytes bytes.
int run_without_allocation(const mhs_instance* inst, uint32_t flags, char* ws, size_t ws_bytes,
                           hipStream_t stream, mhs_summary* sum, int32_t* death_e, int32_t* death_v) {
  if (!inst || !sum) return set_error(MHS_EINVAL, "NULL instance or summary");
  int rc = check_flags(flags);
  if (rc) return rc;
  if (flags & (MHS_PROFILE | MHS_GRAPH)) return set_error(MHS_EINVAL, "MHS_PROFILE and MHS_GRAPH need allocations");
  flags = resolve_auto(flags, inst, 1);
  if (inst->n < 0 || inst->m < 0) return set_error(MHS_EINVAL, "negative n or m");
  if ((inst->m > 0 && !death_e) || (inst->n > 0 && !death_v)) return set_error(MHS_EINVAL, "NULL output array");
  int64_t nnz = 0;
  if (!(flags & MHS_INPUT_DEVICE)) {
    std::string why;
    if (validate_host(inst, &nnz, &why)) return set_error(MHS_EINVAL, why);
  } else if (inst->m > 0) {
    if (!inst->edge_ptr || !inst->edge_vtx || !inst->demand) return set_error(MHS_EINVAL, "NULL device array");
    nnz = inst->nnz;
    if (nnz <= 0) {
      int64_t v = -1;
      if (hipMemcpyAsync(&v, inst->edge_ptr + inst->m, 8, hipMemcpyDeviceToHost, stream) != hipSuccess ||
          hipStreamSynchronize(stream) != hipSuccess)
        return set_error(MHS_EDEVICE, "cannot read edge_ptr[m] from device");
      nnz = v;
    }
    if (nnz < 0 || nnz >= ((int64_t)1 << 31)) return set_error(MHS_EINVAL, "nnz out of range");
  }
  HostInst h;
  h.n = inst->n;
  h.m = inst->m;
  h.nnz = nnz;
  h.k = inst->k;
  h.L = inst_layout(h.n, h.m, nnz, !(flags & MHS_INPUT_DEVICE));
  h.variant = instance_variant(flags, inst);
  h.rule_se = (flags & MHS_RULE_SE) ? 1 : 0;
  h.rule_fe = (flags & MHS_RULE_FE) ? 1 : 0;
  const size_t ctrl = set_control_bytes(1);
  if (ws_bytes < ctrl + h.L.bytes)
    return set_error(MHS_ENOSPC, "instance needs " + std::to_string(ctrl + h.L.bytes) +
                                     " bytes of scratch, the static scratch holds " + std::to_string(ws_bytes));
  h.slice = ws + ctrl;
  rc = bind_input(h, inst, flags, stream);
  if (rc) return rc;
  Set S;
  S.variant = variant_of(flags);
  S.per_cu = grid_per_cu(flags);
  S.gemm_sched = gemm_sched_of(flags);
  rc = S.build({h}, ws, ctrl, stream);
  if (rc) return rc;
  launch_prepare(S.ctx);
  if (hipGetLastError() != hipSuccess) return set_error(MHS_EDEVICE, "prepare launch failed");
  const int64_t max_iter = std::max<int64_t>(2, (int64_t)std::min(h.n, h.m) + 2);
  for (int64_t it = 1;; ++it) {
    if (it > max_iter) return set_error(MHS_EDEVICE, "iteration bound exceeded");
    rc = S.launch_round(false);
    if (rc) return rc;
    int32_t any = -1;
    if (hipMemcpyAsync(&any, S.ctx.gctr + G_ANY, 4, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
      return set_error(MHS_EDEVICE, "round failed");
    if (any == 0) break;
  }
  int32_t ctr[kCtr];
  hipError_t e = hipMemcpyAsync(ctr, h.slice + h.L.off_ctr, sizeof(ctr), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess && h.m > 0)
    e = hipMemcpyAsync(death_e, h.slice + h.L.off_death_e, (size_t)h.m * 4, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess && h.n > 0)
    e = hipMemcpyAsync(death_v, h.slice + h.L.off_death_v, (size_t)h.n * 4, hipMemcpyDeviceToHost, stream);
  if (e != hipSuccess || hipStreamSynchronize(stream) != hipSuccess)
    return set_error(MHS_EDEVICE, "result readback failed");
  if (ctr[C_ERR]) return set_error(ctr[C_ERR] == E_CAPACITY ? MHS_ENOSPC : MHS_EINVAL, err_name(ctr[C_ERR]));
  sum->n_kept = (int32_t)std::count(death_v, death_v + h.n, 0);
  sum->m_kept = (int32_t)std::count(death_e, death_e + h.m, 0);
  sum->n_forced = ctr[C_NFORCED];
  sum->rounds = ctr[C_ROUNDS];
  sum->k_out = h.k - ctr[C_NFORCED];
  return MHS_OK;
}

CompactLayout compact_layout(int32_t n, int32_t m, int64_t nnz) {
  CompactLayout c;
  c.v16 = n <= 65536;
  if (m <= 0) return c;
  size_t o = 0;
  auto take = [&](size_t b) { const size_t r = o; o = align_up(o + b, 256); return r; };
  c.ptr = take(((size_t)m + 1) * 4);
  c.vtx = take((size_t)nnz * (c.v16 ? 2 : 4));
  c.dem = take((size_t)m * 4);
  c.bytes = o;
  return c;
}

// One pass over an instance that passed validate_shape: the checks of
// validate_body (same order, same messages), the sum of hyperedge spans the
// variant rule needs, and the compact image written to b.
// pack_compact over hyperedges [e0, e1): 0 or the error of its first bad
// hyperedge; *span receives the range's span sum.
static int pack_range(const mhs_instance* in, int64_t nnz, const CompactLayout& C, char* b, int32_t e0,
                      int32_t e1, int64_t* span, std::string* why) {
  const int32_t n = in->n;
  int32_t* cp = (int32_t*)(b + C.ptr);
  int32_t* cd = (int32_t*)(b + C.dem);
  uint16_t* cv16 = C.v16 ? (uint16_t*)(b + C.vtx) : nullptr;
  int32_t* cv32 = C.v16 ? nullptr : (int32_t*)(b + C.vtx);
  int64_t sp = 0;
  for (int32_t e = e0; e < e1; ++e) {
    const int64_t a = in->edge_ptr[e], z = in->edge_ptr[e + 1];
    if (z < a || z > nnz) { *why = "edge_ptr not nondecreasing at hyperedge " + std::to_string(e); return E_PTR; }
    if (z == a) { *why = "empty hyperedge " + std::to_string(e); return E_EMPTY; }
    cp[e + 1] = (int32_t)z;   // nnz < 2^31
    int32_t prev = -1;
    for (int64_t p = a; p < z; ++p) {
      const int32_t v = in->edge_vtx[p];
      if (v < 0 || v >= n) { *why = "vertex id out of range in hyperedge " + std::to_string(e); return E_RANGE; }
      if (p > a && v <= prev) { *why = "hyperedge " + std::to_string(e) + " not strictly increasing"; return E_ORDER; }
      prev = v;
      if (cv16) cv16[p] = (uint16_t)v;   // 0 <= v < n <= 65536
      else cv32[p] = v;
    }
    sp += prev - in->edge_vtx[a] + 1;
    const int32_t d = in->demand[e];
    if (d < 1 || (int64_t)d > z - a) { *why = "demand of hyperedge " + std::to_string(e) + " outside [1, |e|]"; return E_DEMAND; }
    cd[e] = d;
  }
  *span = sp;
  return 0;
}

// One pass over an instance that passed validate_shape: the checks of
// validate_body (same order, same messages: the first bad hyperedge is
// reported), the sum of hyperedge spans the variant rule needs (exact: an
// integer sum), and the compact image written to b.  Large instances are
// split into ranges of hyperedges packed on the pool's threads.
int pack_compact(const mhs_instance* in, int64_t nnz, const CompactLayout& C, char* b, double* span,
                 std::string* why) {
  const int32_t m = in->m;
  *span = 0;
  if (m == 0) return 0;
  ((int32_t*)(b + C.ptr))[0] = 0;
  constexpr int64_t kRange = 1 << 17;   // incidences per range
  const int32_t R = (int32_t)std::min<int64_t>(std::max<int64_t>(1, nnz / kRange), std::min(m, 64));
  if (R == 1) {
    int64_t sp = 0;
    const int rc = pack_range(in, nnz, C, b, 0, m, &sp, why);
    *span = (double)sp;
    return rc;
  }
  std::vector<int> code(R, 0);
  std::vector<int64_t> sp(R, 0);
  std::vector<std::string> msg(R);
  parallel_for(R, [&](int32_t r) {
    const int32_t e0 = (int32_t)((int64_t)m * r / R), e1 = (int32_t)((int64_t)m * (r + 1) / R);
    code[r] = pack_range(in, nnz, C, b, e0, e1, &sp[r], &msg[r]);
  });
  int64_t tot = 0;
  for (int32_t r = 0; r < R; ++r) {
    if (code[r]) {
      *why = msg[r];
      return code[r];
    }
    tot += sp[r];
  }
  *span = (double)tot;
  return 0;
}

}  // namespace mhsk

// ======================================================================= ABI
extern "C" {

const char* mhs_last_error(void) { return g_err.c_str(); }
#ifndef MHSK_SOURCE_SHA
#define MHSK_SOURCE_SHA "unknown"
#endif
// The build stamps the hash of the sources it compiled (csrc and the public
// header), so a caller can tell whether a library matches the tree it ships in.
const char* mhs_version(void) { return "mhsk 0.2 (gfx950, int8 MFMA) src=" MHSK_SOURCE_SHA; }

size_t mhs_workspace_bytes(int32_t n, int32_t m, int64_t nnz, uint32_t flags) {
  if (n < 0 || m < 0 || nnz < 0) return 0;
  return set_control_bytes(1) + inst_layout(n, m, nnz, !(flags & MHS_INPUT_DEVICE)).bytes;
}

int mhs_run(const mhs_instance* inst, uint32_t flags, void* d_ws, size_t ws_bytes, void* hip_stream,
            mhs_result** out) {
  auto t0 = std::chrono::steady_clock::now();
  if (!out) return set_error(MHS_EINVAL, "NULL out");
  *out = nullptr;
  int rc = check_flags(flags);
  if (rc) return rc;
  if (inst) flags = resolve_auto(flags, inst, 1);
  hipStream_t stream = (hipStream_t)hip_stream;
  int64_t nnz = 0;
  rc = instance_nnz(inst, flags, &nnz, stream);
  if (rc) return rc;
  if (!d_ws || ((uintptr_t)d_ws & 255)) return set_error(MHS_EINVAL, "workspace NULL or not 256-byte aligned");
  HostInst h;
  h.n = inst->n;
  h.m = inst->m;
  h.nnz = nnz;
  h.k = inst->k;
  h.L = inst_layout(h.n, h.m, nnz, !(flags & MHS_INPUT_DEVICE));
  h.variant = instance_variant(flags, inst);
  h.rule_se = (flags & MHS_RULE_SE) ? 1 : 0;
  h.rule_fe = (flags & MHS_RULE_FE) ? 1 : 0;
  const size_t ctrl = set_control_bytes(1);
  if (ws_bytes < ctrl + h.L.bytes) return set_error(MHS_ENOSPC, "workspace smaller than mhs_workspace_bytes");
  h.slice = (char*)d_ws + ctrl;
  rc = bind_input(h, inst, flags, stream);
  if (rc) return rc;
  Set S;
  S.profile = (flags & MHS_PROFILE) != 0;
  S.variant = variant_of(flags);
  S.per_cu = grid_per_cu(flags);
  S.gemm_sched = gemm_sched_of(flags);
  rc = S.build({h}, (char*)d_ws, ctrl, stream);
  if (rc) return rc;
  int32_t iters = 0;
  rc = run_rounds(S, flags, &iters);
  if (rc) return rc;
  std::vector<int32_t> ctr, de, dv, fw;
  std::vector<uint8_t> forced;
  rc = S.read_member(0, ctr, de, dv, &forced, &fw);
  if (rc) return rc;
  if (ctr[C_ERR]) return set_error(ctr[C_ERR] == E_CAPACITY ? MHS_ENOSPC : MHS_EINVAL, err_name(ctr[C_ERR]));
  mhs_result* r = make_result(h, ctr, std::move(de), std::move(dv), std::move(fw), std::move(forced));
  if (S.profile) fill_profile(S, &r->stats);
  r->stats.gemm_launches = 2 * iters;
  r->stats.total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = r;
  return MHS_OK;
}

// Bytes of an instance's staged input (edge_ptr, edge_vtx, demand as the
// staging part of its layout places them).
static size_t staged_span(int32_t n, int32_t m, int64_t nnz) {
  if (m <= 0) return 0;
  const InstLayout L = inst_layout(n, m, nnz, true);
  return L.off_in_dem + (size_t)m * 4 - L.off_in_ptr;
}

size_t mhs_batch_workspace_bytes(const mhs_instance* insts, int32_t count, uint32_t flags) {
  if (count < 0 || (count > 0 && !insts)) return 0;
  const bool dev = (flags & MHS_INPUT_DEVICE) != 0;
  size_t total = set_control_bytes(count);
  size_t out_words = 0;
  for (int32_t i = 0; i < count; ++i) {
    const mhs_instance& in = insts[i];
    if (in.n < 0 || in.m < 0) return 0;
    int64_t nnz = 0;
    if (in.m > 0) {
      nnz = dev ? in.nnz : (in.edge_ptr ? in.edge_ptr[in.m] : 0);
      if (dev && nnz <= 0) return 0;   // device batches carry every instance's nnz
    }
    // the instance's slice; host inputs add their input as the kernels read
    // it and their compact upload
    total += inst_layout(in.n, in.m, nnz, false).bytes;
    if (!dev) total += align_up(staged_span(in.n, in.m, nnz), 256) + compact_layout(in.n, in.m, nnz).bytes;
    out_words += kCtr + 2 + 2 * ((size_t)in.n + (size_t)in.m);   // counters, kept counts, arrays
  }
  const size_t tail = dev ? align_up((size_t)count * 8, 256) : align_up((size_t)count * sizeof(WidenJob), 256);
  return total + align_up(out_words * 4, 256) + tail;
}

// The part of a batched run after the inputs are in place: the set, the
// rounds to the fixpoint, one gather of every result, the readback in
// chunks, the result objects or the caller's arrays.  `out` is the device
// area for the gathered results (out_words words).
// Events of one chunked readback (created per call: a few microseconds).
struct EventSet {
  std::vector<hipEvent_t> ev;
  explicit EventSet(int k) : ev(k, nullptr) {
    for (hipEvent_t& e : ev)
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) e = nullptr;
  }
  ~EventSet() {
    for (hipEvent_t e : ev)
      if (e) hipEventDestroy(e);
  }
  EventSet(const EventSet&) = delete;
  EventSet& operator=(const EventSet&) = delete;
  bool ok() const {
    for (hipEvent_t e : ev)
      if (!e) return false;
    return true;
  }
  hipEvent_t operator[](int k) const { return ev[k]; }
};
constexpr int32_t kReadbackChunks = 8;   // chunks of a batch's result readback

// Caller arrays a batch's results are written into (mhs_run_batch_into);
// any may be NULL.
struct BatchArrays {
  mhs_summary* sums;
  mhs_stats* stats;
  int32_t* death_e;
  int32_t* death_v;
  int32_t* demand;
  uint8_t* forced;
};

static int finish_batch(std::vector<HostInst>& hs, uint32_t flags, void* d_ws, size_t ctrl, char* out,
                        size_t out_words, hipStream_t stream, mhs_result** outs,
                        std::chrono::steady_clock::time_point t0, const BatchArrays* arr = nullptr) {
  const int32_t count = (int32_t)hs.size();
  Set S;
  S.profile = (flags & MHS_PROFILE) != 0;
  S.variant = variant_of(flags);
  S.per_cu = grid_per_cu(flags);
  S.gemm_sched = gemm_sched_of(flags);
  int rc = S.build(hs, (char*)d_ws, ctrl, stream);
  if (rc) return rc;
  int32_t iters = 0;
  rc = run_rounds(S, flags, &iters);
  if (rc) return rc;
  // One gather kernel writes the results in the caller's layout (every
  // member's counters and kept counts first, then death_e, death_v, the
  // final demands and the forced flags, each concatenated over the members),
  // then the readback: the counters first, checked for errors before
  // anything is exported, then the arrays in chunks of members, each chunk
  // exported on the host threads (contiguous copies) while the next one is
  // on its way.
  std::vector<int64_t> off(2 * ((size_t)count + 1), 0);   // [m prefix | n prefix]
  int64_t* moff = off.data();
  int64_t* noff = off.data() + count + 1;
  for (int32_t i = 0; i < count; ++i) {
    moff[i + 1] = moff[i] + hs[i].m;
    noff[i + 1] = noff[i] + hs[i].n;
  }
  const int64_t M = moff[count], N = noff[count];
  int32_t max_n = 0;
  for (const HostInst& h : hs) max_n = std::max(max_n, h.n);
  // a death round is at most the rounds run, a final demand at most its
  // hyperedge's size (validated), which is at most n: below 2^16 both travel
  // as 16-bit values, half the bytes over the bus
  const bool narrow = iters < 65535 && max_n < 65536;
  const int64_t es = narrow ? 2 : 4;
  GatherLayout G;
  G.ctr = 0;
  G.kept = (int64_t)count * kCtr;
  G.de_b = (G.kept + 2 * (int64_t)count) * 4;
  G.dv_b = G.de_b + M * es;
  G.dem_b = G.dv_b + N * es;
  G.forced_b = G.dem_b + M * es;
  G.narrow = narrow ? 1 : 0;
  if ((size_t)(G.forced_b + N) > out_words * 4) return set_error(MHS_EINVAL, "result area too small");
  LaunchCtx c = S.ctx;
  c.out = (int32_t*)out;
  if (hipMemcpyAsync(c.ooff, off.data(), off.size() * 8, hipMemcpyHostToDevice, stream) != hipSuccess)
    return set_error(MHS_EDEVICE, "offset upload failed");
  launch_gather(c, G);
  int32_t* p = (int32_t*)pinned_buffer(out_words * 4);
  if (!p) return set_error(MHS_EDEVICE, "pinned allocation failed");
  const uint8_t* pb = reinterpret_cast<const uint8_t*>(p);
  const int32_t C = std::max(1, std::min(count, kReadbackChunks));
  std::vector<int32_t> cb(C + 1, count);   // chunk k: members [cb[k], cb[k+1]), about equal in entries
  cb[0] = 0;
  for (int32_t k = 1, i = 0; k < C; ++k) {
    const int64_t target = (M + N) * k / C;
    while (i < count && moff[i] + noff[i] < target) ++i;
    cb[k] = i;
  }
  EventSet ev(C + 1);
  if (!ev.ok()) return set_error(MHS_EDEVICE, "event creation failed");
  auto d2h = [&](int64_t byte0, int64_t bytes) {
    return bytes <= 0 || hipMemcpyAsync((char*)p + byte0, (char*)c.out + byte0, (size_t)bytes,
                                        hipMemcpyDeviceToHost, stream) == hipSuccess;
  };
  bool queued = d2h(0, G.de_b) && hipEventRecord(ev[0], stream) == hipSuccess;
  for (int32_t k = 0; queued && k < C; ++k) {
    const int64_t ma = moff[cb[k]], mb = moff[cb[k + 1]], na = noff[cb[k]], nb = noff[cb[k + 1]];
    queued = d2h(G.de_b + ma * es, (mb - ma) * es) && d2h(G.dv_b + na * es, (nb - na) * es) &&
             d2h(G.dem_b + ma * es, (mb - ma) * es) && d2h(G.forced_b + na, nb - na) &&
             hipEventRecord(ev[k + 1], stream) == hipSuccess;
  }
  if (!queued || hipEventSynchronize(ev[0]) != hipSuccess) {
    hipStreamSynchronize(stream);
    return set_error(MHS_EDEVICE, "result readback failed");
  }
  for (int32_t i = 0; i < count; ++i) {
    const int32_t err = p[(size_t)i * kCtr + C_ERR];
    if (err) {
      hipStreamSynchronize(stream);   // the copies still write into the pinned buffer
      return set_error(err == E_CAPACITY ? MHS_ENOSPC : MHS_EINVAL,
                       "instance " + std::to_string(i) + ": " + err_name(err));
    }
  }
  mhs_stats prof;
  std::memset(&prof, 0, sizeof(prof));
  if (S.profile) fill_profile(S, &prof);
  auto set_prof = [&](mhs_stats& st) {
    st.edge_gemm_ms = prof.edge_gemm_ms;
    st.vertex_gemm_ms = prof.vertex_gemm_ms;
    st.gemm_ms = prof.gemm_ms;
    st.rows_ms = prof.rows_ms;
    st.compact_ms = prof.compact_ms;
    st.round_end_ms = prof.round_end_ms;
    st.sparse_ms = prof.sparse_ms;
    st.edge_sparse_ms = prof.edge_sparse_ms;
    st.vertex_sparse_ms = prof.vertex_sparse_ms;
  };
  // elements [i0, i0 + len) of the array at byte offset byte0, as int32
  auto widened = [&](int64_t byte0, int64_t i0, int64_t len) {
    if (narrow) {
      const uint16_t* a = reinterpret_cast<const uint16_t*>(pb + byte0) + i0;
      return std::vector<int32_t>(a, a + len);
    }
    const int32_t* a = reinterpret_cast<const int32_t*>(pb + byte0) + i0;
    return std::vector<int32_t>(a, a + len);
  };
  // member i's summary and stats (caller arrays), or its result object
  auto export_one = [&](int32_t i) {
    const HostInst& h = hs[i];
    const int32_t* ctr = p + (size_t)i * kCtr;
    if (!arr) {
      const uint8_t* fo = pb + G.forced_b + noff[i];
      mhs_result* r = make_result(h, std::vector<int32_t>(ctr, ctr + kCtr), widened(G.de_b, moff[i], h.m),
                                  widened(G.dv_b, noff[i], h.n), widened(G.dem_b, moff[i], h.m),
                                  std::vector<uint8_t>(fo, fo + h.n));
      r->stats.gemm_launches = 2 * iters;
      if (i == 0 && S.profile) set_prof(r->stats);   // set-wide timings are reported on the first result
      outs[i] = r;
      return;
    }
    if (arr->sums) {
      mhs_summary& sm = arr->sums[i];
      sm.m_kept = p[G.kept + i];
      sm.n_kept = p[G.kept + count + i];
      sm.n_forced = ctr[C_NFORCED];
      sm.rounds = ctr[C_ROUNDS];
      sm.k_out = h.k - ctr[C_NFORCED];
    }
    if (arr->stats) {
      mhs_stats& st = arr->stats[i];
      stats_from_counters(ctr, &st);
      st.gemm_launches = 2 * iters;
      if (i == 0 && S.profile) set_prof(st);
    }
  };
  // a chunk's arrays into the caller's: contiguous ranges, split in pieces
  // of 2^18 elements over the host threads (16-bit values widened)
  auto export_arrays = [&](int32_t k) {
    const int64_t ma = moff[cb[k]], mb = moff[cb[k + 1]], na = noff[cb[k]], nb = noff[cb[k + 1]];
    struct Piece { void* dst; const uint8_t* src; int64_t n; int kind; };   // kind: 0 bytes, 1 int32, 2 uint16
    std::vector<Piece> pieces;
    auto add = [&](void* dst, int es_dst, const uint8_t* src, int kind, int64_t n) {
      if (!dst) return;
      const int es_src = kind == 2 ? 2 : es_dst;
      for (int64_t o = 0; o < n; o += (int64_t)1 << 18)
        pieces.push_back({(char*)dst + o * es_dst, src + o * es_src, std::min<int64_t>((int64_t)1 << 18, n - o), kind});
    };
    const int ak = narrow ? 2 : 1;
    add(arr->death_e ? arr->death_e + ma : nullptr, 4, pb + G.de_b + ma * es, ak, mb - ma);
    add(arr->death_v ? arr->death_v + na : nullptr, 4, pb + G.dv_b + na * es, ak, nb - na);
    add(arr->demand ? arr->demand + ma : nullptr, 4, pb + G.dem_b + ma * es, ak, mb - ma);
    add(arr->forced ? arr->forced + na : nullptr, 1, pb + G.forced_b + na, 0, nb - na);
    parallel_for((int32_t)pieces.size(), [&](int32_t t) {
      const Piece& q = pieces[t];
      if (q.kind == 2) {
        const uint16_t* a = reinterpret_cast<const uint16_t*>(q.src);
        int32_t* d = static_cast<int32_t*>(q.dst);
        for (int64_t i = 0; i < q.n; ++i) d[i] = a[i];
      } else {
        std::memcpy(q.dst, q.src, (size_t)q.n * (q.kind == 1 ? 4 : 1));
      }
    });
  };
  for (int32_t k = 0; k < C; ++k) {
    if (hipEventSynchronize(ev[k + 1]) != hipSuccess) {
      hipStreamSynchronize(stream);
      if (!arr)
        for (int32_t i = 0; i < cb[k]; ++i) { mhs_result_free(outs[i]); outs[i] = nullptr; }
      return set_error(MHS_EDEVICE, "result readback failed");
    }
    if (arr) {
      export_arrays(k);
      for (int32_t i = cb[k]; i < cb[k + 1]; ++i) export_one(i);
    } else {
      parallel_for(cb[k + 1] - cb[k], [&](int32_t t) { export_one(cb[k] + t); });
    }
  }
  const double total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  for (int32_t i = 0; i < count; ++i) {
    if (!arr) outs[i]->stats.total_ms = total_ms;
    else if (arr->stats) arr->stats[i].total_ms = total_ms;
  }
  return MHS_OK;
}


// Batches of device-resident instances: the arrays are read in place (the
// prepare step validates them), every instance gives its nnz, and the
// hybrid rule's span sums are computed on the device (one small kernel and
// one copy) before the set is built.
static int run_batch_device(const mhs_instance* insts, int32_t count, uint32_t flags, void* d_ws, size_t ws_bytes,
                            void* hip_stream, mhs_result** outs, std::chrono::steady_clock::time_point t0,
                            const BatchArrays* arr) {
  if (!d_ws || ((uintptr_t)d_ws & 255)) return set_error(MHS_EINVAL, "workspace NULL or not 256-byte aligned");
  hipStream_t stream = (hipStream_t)hip_stream;
  const size_t ctrl = set_control_bytes(count);
  std::vector<HostInst> hs(count);
  size_t off = ctrl, out_words = 0;
  for (int32_t i = 0; i < count; ++i) {
    const mhs_instance& in = insts[i];
    const std::string at = "instance " + std::to_string(i) + ": ";
    if (in.n < 0 || in.m < 0) return set_error(MHS_EINVAL, at + "negative n or m");
    if (in.m > 0) {
      if (!in.edge_ptr || !in.edge_vtx || !in.demand) return set_error(MHS_EINVAL, at + "NULL device array");
      if (in.nnz <= 0) return set_error(MHS_EINVAL, at + "device batches need the nnz of every instance");
      if (in.nnz >= ((int64_t)1 << 31)) return set_error(MHS_EINVAL, at + "nnz out of range");
    }
    HostInst& h = hs[i];
    h.n = in.n;
    h.m = in.m;
    h.nnz = in.m > 0 ? in.nnz : 0;
    h.k = in.k;
    h.L = inst_layout(h.n, h.m, h.nnz, false);
    h.ptr = in.edge_ptr;
    h.vtx = in.edge_vtx;
    h.dem = in.demand;
    h.rule_se = (flags & MHS_RULE_SE) ? 1 : 0;
    h.rule_fe = (flags & MHS_RULE_FE) ? 1 : 0;
    h.slice = (char*)d_ws + off;
    off += h.L.bytes;
    out_words += kCtr + 2 + 2 * ((size_t)h.n + (size_t)h.m);   // counters, kept counts, arrays
  }
  const size_t out_bytes = align_up(out_words * 4, 256);
  unsigned long long* spans = (unsigned long long*)((char*)d_ws + off + out_bytes);
  if (ws_bytes < off + out_bytes + align_up((size_t)count * 8, 256))
    return set_error(MHS_ENOSPC, "workspace smaller than mhs_batch_workspace_bytes");
  // the per-instance contraction: explicit variants apply to all; the
  // hybrid rule needs every instance's span sum
  const uint32_t host_rule = flags & ~MHS_INPUT_DEVICE;
  bool need_span = false;
  for (int32_t i = 0; i < count; ++i) {
    hs[i].variant = variant_with_span(host_rule, &insts[i], 0.0);
    const uint32_t v = flags & MHS_VARIANT_MASK;
    if ((v == MHS_VARIANT_AUTO || v == MHS_VARIANT_HYBRID) && std::max(hs[i].n, hs[i].m) < (1 << 29) &&
        hs[i].m > 0 && hs[i].n > 0)
      need_span = true;
  }
  if (need_span) {
    Set probe;
    int rc = probe.build(hs, (char*)d_ws, ctrl, stream);
    if (rc) return rc;
    if (hipMemsetAsync(spans, 0, (size_t)count * 8, stream) != hipSuccess)
      return set_error(MHS_EDEVICE, "span clear failed");
    launch_span(probe.ctx, spans);
    unsigned long long* p = (unsigned long long*)pinned_buffer((size_t)count * 8);
    if (!p) return set_error(MHS_EDEVICE, "pinned allocation failed");
    if (hipMemcpyAsync(p, spans, (size_t)count * 8, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
      return set_error(MHS_EDEVICE, "span readback failed");
    for (int32_t i = 0; i < count; ++i) {
      mhs_instance probe_in = insts[i];
      hs[i].variant = variant_with_span(host_rule, &probe_in, (double)p[i]);
    }
  }
  return finish_batch(hs, flags, d_ws, ctrl, (char*)d_ws + off, out_words, stream, outs, t0, arr);
}

static int run_batch(const mhs_instance* insts, int32_t count, uint32_t flags, void* d_ws, size_t ws_bytes,
                     void* hip_stream, mhs_result** outs, const BatchArrays* arr);

int mhs_run_batch(const mhs_instance* insts, int32_t count, uint32_t flags, void* d_ws, size_t ws_bytes,
                  void* hip_stream, mhs_result** outs) {
  if (count < 0 || (count > 0 && !outs)) return set_error(MHS_EINVAL, "bad batch arguments");
  for (int32_t i = 0; i < count; ++i) outs[i] = nullptr;
  return run_batch(insts, count, flags, d_ws, ws_bytes, hip_stream, outs, nullptr);
}

int mhs_run_batch_into(const mhs_instance* insts, int32_t count, uint32_t flags, void* d_ws, size_t ws_bytes,
                       void* hip_stream, mhs_summary* sums, mhs_stats* stats, int32_t* death_e, int32_t* death_v,
                       int32_t* demand, uint8_t* forced) {
  const BatchArrays arr = {sums, stats, death_e, death_v, demand, forced};
  return run_batch(insts, count, flags, d_ws, ws_bytes, hip_stream, nullptr, &arr);
}

static int run_batch(const mhs_instance* insts, int32_t count, uint32_t flags, void* d_ws, size_t ws_bytes,
                     void* hip_stream, mhs_result** outs, const BatchArrays* arr) {
  auto t0 = std::chrono::steady_clock::now();
  if (count < 0 || (count > 0 && !insts)) return set_error(MHS_EINVAL, "bad batch arguments");
  int rc = check_flags(flags);
  if (rc) return rc;
  if (count == 0) return MHS_OK;
  flags = resolve_auto(flags, insts, count);
  if (flags & MHS_INPUT_DEVICE) return run_batch_device(insts, count, flags, d_ws, ws_bytes, hip_stream, outs, t0, arr);
  if (!d_ws || ((uintptr_t)d_ws & 255)) return set_error(MHS_EINVAL, "workspace NULL or not 256-byte aligned");
  hipStream_t stream = (hipStream_t)hip_stream;
  const size_t ctrl = set_control_bytes(count);
  std::vector<HostInst> hs(count);
  std::vector<std::string> why(count);
  // shapes and layouts first (edge_ptr[0] and edge_ptr[m] of each instance);
  // the error reported is that of the first bad instance, as a full
  // validation in index order finds it
  for (int32_t i = 0; i < count; ++i) {
    int64_t nnz = 0;
    if (validate_shape(&insts[i], &nnz, &why[i])) {
      for (int32_t k = 0; k < i; ++k)
        if (validate_body(&insts[k], hs[k].nnz, &why[k]))
          return set_error(MHS_EINVAL, "instance " + std::to_string(k) + ": " + why[k]);
      return set_error(MHS_EINVAL, "instance " + std::to_string(i) + ": " + why[i]);
    }
    HostInst& h = hs[i];
    h.n = insts[i].n;
    h.m = insts[i].m;
    h.nnz = nnz;
    h.k = insts[i].k;
    h.L = inst_layout(h.n, h.m, nnz, false);
    h.rule_se = (flags & MHS_RULE_SE) ? 1 : 0;
    h.rule_fe = (flags & MHS_RULE_FE) ? 1 : 0;
  }
  // workspace: control block | every instance's input as the kernels read
  // it (edge_ptr int64, edge_vtx int32, demand) | the instances' slices |
  // results | the upload: widening jobs, then every instance's compact input
  std::vector<size_t> soff(count + 1, 0), coff(count + 1, 0);
  std::vector<InstLayout> SL(count);
  std::vector<CompactLayout> CL(count);
  coff[0] = align_up((size_t)count * sizeof(WidenJob), 256);
  for (int32_t i = 0; i < count; ++i) {
    SL[i] = inst_layout(hs[i].n, hs[i].m, hs[i].nnz, true);   // where the staging part puts each array
    soff[i + 1] = soff[i] + align_up(staged_span(hs[i].n, hs[i].m, hs[i].nnz), 256);
    CL[i] = compact_layout(hs[i].n, hs[i].m, hs[i].nnz);
    coff[i + 1] = coff[i] + CL[i].bytes;
  }
  char* const stage = (char*)d_ws + ctrl;
  size_t off = ctrl + soff[count], out_words = 0;
  for (int32_t i = 0; i < count; ++i) {
    hs[i].slice = (char*)d_ws + off;
    off += hs[i].L.bytes;
    out_words += kCtr + 2 + 2 * ((size_t)hs[i].n + (size_t)hs[i].m);   // counters, kept counts, arrays
  }
  const size_t out_bytes = align_up(out_words * 4, 256);
  char* const up = (char*)d_ws + off + out_bytes;
  if (ws_bytes < off + out_bytes + coff[count])
    return set_error(MHS_ENOSPC, "workspace smaller than mhs_batch_workspace_bytes");
  char* img = (char*)pinned_upload(coff[count]);
  if (!img) return set_error(MHS_EDEVICE, "pinned allocation failed");
  WidenJob* jobs = reinterpret_cast<WidenJob*>(img);
  // one pass over each instance's arrays, in parallel: validation, variant
  // choice, and the narrowing copy into the pinned image while they are
  // still cached; in chunks of instances, each uploaded while the next one
  // is packed
  std::vector<uint8_t> bad(count, 0);
  auto pack = [&](int32_t i) {
    HostInst& h = hs[i];
    const CompactLayout& C = CL[i];
    const InstLayout& L = SL[i];
    double span = 0;
    if (pack_compact(&insts[i], h.nnz, C, img + coff[i], &span, &why[i])) { bad[i] = 1; return; }
    h.variant = variant_with_span(flags, &insts[i], span);
    char* const w = stage + soff[i];   // device: wide arrays
    char* const c = up + coff[i];      // device: compact arrays
    WidenJob J;
    std::memset(&J, 0, sizeof(J));
    J.m = h.m;
    J.nnz = h.nnz;
    J.vtx16 = C.v16 ? 1 : 0;
    if (h.m > 0) {
      J.sptr = (const int32_t*)(c + C.ptr);
      J.svtx = c + C.vtx;
      J.sdem = (const int32_t*)(c + C.dem);
      J.dptr = (int64_t*)w;
      J.dvtx = (int32_t*)(w + (L.off_in_vtx - L.off_in_ptr));
      J.ddem = (int32_t*)(w + (L.off_in_dem - L.off_in_ptr));
    }
    jobs[i] = J;
  };
  // the worker that packs a chunk's last instance uploads the chunk
  const int32_t chunks = std::min<int32_t>(8, count);
  auto chunk_lo = [&](int32_t k) { return (int32_t)((int64_t)count * k / chunks); };
  std::vector<std::atomic<int32_t>> left(chunks);
  for (int32_t k = 0; k < chunks; ++k) left[k] = chunk_lo(k + 1) - chunk_lo(k);
  std::atomic<bool> copy_failed(false);
  parallel_for(count, [&](int32_t i) {
    pack(i);
    int32_t kk = 0;   // chunk of i
    while (kk + 1 < chunks && i >= chunk_lo(kk + 1)) ++kk;
    if (left[kk].fetch_sub(1) == 1) {
      const size_t a = coff[chunk_lo(kk)], e = coff[chunk_lo(kk + 1)];
      if (e > a && hipMemcpyAsync(up + a, img + a, e - a, hipMemcpyHostToDevice, stream) != hipSuccess)
        copy_failed = true;
    }
  });
  // the widening jobs, written by every chunk, go last
  if (hipMemcpyAsync(up, img, coff[0], hipMemcpyHostToDevice, stream) != hipSuccess) copy_failed = true;
  int32_t first_bad = -1;
  for (int32_t i = 0; i < count && first_bad < 0; ++i)
    if (bad[i]) first_bad = i;
  if (first_bad >= 0 || copy_failed) {
    // no copy may still read the pinned image or write the workspace
    // once this call returns
    hipStreamSynchronize(stream);
    if (first_bad >= 0)
      return set_error(MHS_EINVAL, "instance " + std::to_string(first_bad) + ": " + why[first_bad]);
    return set_error(MHS_EDEVICE, "input upload failed");
  }
  for (int32_t i = 0; i < count; ++i) {
    HostInst& h = hs[i];
    const InstLayout& L = SL[i];
    char* b = stage + soff[i];
    h.ptr = (const int64_t*)b;
    h.vtx = (const int32_t*)(b + (L.off_in_vtx - L.off_in_ptr));
    h.dem = (const int32_t*)(b + (L.off_in_dem - L.off_in_ptr));
  }
  launch_widen(stream, reinterpret_cast<const WidenJob*>(up), count);
  return finish_batch(hs, flags, d_ws, ctrl, (char*)d_ws + off, out_words, stream, outs, t0, arr);
}

int mhs_tune(const mhs_instance* insts, int32_t count, uint32_t flags, void* d_ws, size_t ws_bytes,
             void* hip_stream, mhs_tune_report* report) {
  if (!report || count < 1 || !insts) return set_error(MHS_EINVAL, "bad tune arguments");
  if (flags & ~(uint32_t)(MHS_NO_GRAPH | MHS_GRAPH | MHS_RULE_SE | MHS_RULE_FE | MHS_INPUT_DEVICE))
    return set_error(MHS_EINVAL, "tune takes MHS_NO_GRAPH, MHS_GRAPH, MHS_RULE_SE, MHS_RULE_FE, MHS_INPUT_DEVICE");
  std::memset(report, 0, sizeof(*report));
  std::vector<mhs_result*> outs(count, nullptr), ref(count, nullptr);
  auto release = [&](std::vector<mhs_result*>& v) { for (auto*& r : v) { delete r; r = nullptr; } };
  // a candidate's time: the best of three runs after one that warms up
  // (graph capture); one run alone left the choice among close candidates
  // to noise
  auto timed = [&](uint32_t f, double* ms) -> int {
    int rc = MHS_OK;
    *ms = 1e300;
    for (int rep = 0; rep < 4 && rc == MHS_OK; ++rep) {
      release(outs);
      auto t0 = std::chrono::steady_clock::now();
      rc = mhs_run_batch(insts, count, f, d_ws, ws_bytes, hip_stream, outs.data());
      const double t = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      if (rep > 0) *ms = std::min(*ms, t);
    }
    return rc;
  };
  const uint32_t base = flags & (MHS_NO_GRAPH | MHS_GRAPH | MHS_RULE_SE | MHS_RULE_FE | MHS_INPUT_DEVICE);
  double best = 1e300, dflt = 0;
  uint32_t best_flags = MHS_VARIANT_INT8;
  int rc = timed(base | MHS_VARIANT_INT8, &dflt);
  if (rc) { release(outs); return rc; }
  ref.swap(outs);
  int cand = 0;
  std::vector<uint32_t> cands;
  for (uint32_t v : {MHS_VARIANT_INT8, MHS_VARIANT_BITSET, MHS_VARIANT_HYBRID})
    for (int g = 0; g < (v == MHS_VARIANT_BITSET ? 1 : 3); ++g)
      for (int k = 0; k <= 4; ++k)
        cands.push_back(v | MHS_GRID_LOG2(k) | (v == MHS_VARIANT_BITSET ? 0u : MHS_GEMM_SCHED(g)));
  cands.push_back(MHS_VARIANT_SPARSE | MHS_GRID_LOG2(2));   // no persistent grid
  for (const uint32_t f : cands) {
    {
      double ms = 0;
      rc = timed(base | f, &ms);
      if (rc) { release(outs); release(ref); return rc; }
      ++cand;
      for (int32_t i = 0; i < count; ++i)
        if (outs[i]->rounds != ref[i]->rounds || outs[i]->death_e != ref[i]->death_e ||
            outs[i]->death_v != ref[i]->death_v) {
          release(outs);
          release(ref);
          return set_error(MHS_EDEVICE, "autotuner candidates disagree");
        }
      if (ms < best) { best = ms; best_flags = f; }
    }
  }
  release(outs);
  release(ref);
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tuned[size_class(insts, count, (flags & MHS_INPUT_DEVICE) != 0)] = best_flags;
  }
  report->best_flags = best_flags;
  report->candidates = cand;
  report->best_ms = best;
  report->default_ms = dflt;
  return MHS_OK;
}

void mhs_tune_reset(void) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tuned.clear();
}

// A failed result reports its status (and message) from every accessor.
static int failed(const mhs_result* r) { return r->status ? set_error(r->status, r->error) : MHS_OK; }

int mhs_result_status(const mhs_result* r) {
  if (!r) return set_error(MHS_EINVAL, "NULL result");
  return failed(r);
}

int mhs_result_summary(const mhs_result* r, mhs_summary* s) {
  if (!r || !s) return set_error(MHS_EINVAL, "NULL argument");
  if (int rc = failed(r)) return rc;
  s->n_kept = (int32_t)std::count(r->death_v.begin(), r->death_v.end(), 0);
  s->m_kept = (int32_t)std::count(r->death_e.begin(), r->death_e.end(), 0);
  s->n_forced = r->n_forced;
  s->rounds = r->rounds;
  s->k_out = r->k - r->n_forced;
  return MHS_OK;
}

int mhs_result_stats(const mhs_result* r, mhs_stats* s) {
  if (!r || !s) return set_error(MHS_EINVAL, "NULL argument");
  if (int rc = failed(r)) return rc;
  *s = r->stats;
  return MHS_OK;
}

int mhs_result_copy(const mhs_result* r, int32_t* kept_v, int32_t* kept_e, int32_t* forced_v) {
  if (!r) return set_error(MHS_EINVAL, "NULL result");
  if (int rc = failed(r)) return rc;
  if (forced_v) {
    int32_t k = 0;
    for (int32_t v = 0; v < r->n; ++v) if (r->forced[v]) forced_v[k++] = v;
  }
  if (kept_v) {
    int32_t k = 0;
    for (int32_t v = 0; v < r->n; ++v) if (r->death_v[v] == 0) kept_v[k++] = v;
  }
  if (kept_e) {
    int32_t k = 0;
    for (int32_t e = 0; e < r->m; ++e) if (r->death_e[e] == 0) kept_e[k++] = e;
  }
  return MHS_OK;
}

int mhs_result_deaths(const mhs_result* r, int32_t* death_e, int32_t* death_v) {
  if (!r) return set_error(MHS_EINVAL, "NULL result");
  if (int rc = failed(r)) return rc;
  if (death_e && r->m) std::memcpy(death_e, r->death_e.data(), (size_t)r->m * 4);
  if (death_v && r->n) std::memcpy(death_v, r->death_v.data(), (size_t)r->n * 4);
  return MHS_OK;
}

int mhs_result_demands(const mhs_result* r, int32_t* demand) {
  if (!r) return set_error(MHS_EINVAL, "NULL result");
  if (int rc = failed(r)) return rc;
  if (demand && r->m) std::memcpy(demand, r->demand.data(), (size_t)r->m * 4);
  return MHS_OK;
}

int mhs_result_forced(const mhs_result* r, uint8_t* forced) {
  if (!r) return set_error(MHS_EINVAL, "NULL result");
  if (int rc = failed(r)) return rc;
  if (forced && r->n) std::memcpy(forced, r->forced.data(), (size_t)r->n);
  return MHS_OK;
}

int mhs_result_round(const mhs_result* r, int32_t round, int32_t* n_del_e, int32_t* del_e,
                     int32_t* n_del_v, int32_t* del_v) {
  if (!r) return set_error(MHS_EINVAL, "NULL result");
  if (int rc = failed(r)) return rc;
  if (round < 1 || round > r->rounds) return set_error(MHS_EINVAL, "round out of range");
  int32_t ke = 0, kv = 0;
  for (int32_t e = 0; e < r->m; ++e)
    if (r->death_e[e] == round) { if (del_e) del_e[ke] = e; ++ke; }
  for (int32_t v = 0; v < r->n; ++v)
    if (r->death_v[v] == round) { if (del_v) del_v[kv] = v; ++kv; }
  if (n_del_e) *n_del_e = ke;
  if (n_del_v) *n_del_v = kv;
  return MHS_OK;
}

void mhs_result_free(mhs_result* r) { delete r; }

int mhs_results_take(mhs_result** rs, int32_t count, mhs_summary* sums, mhs_stats* stats, int32_t* death_e,
                     int32_t* death_v, int32_t* demand, uint8_t* forced) {
  if (count < 0 || (count > 0 && !rs)) return set_error(MHS_EINVAL, "bad arguments");
  std::vector<size_t> mo(count + 1, 0), no(count + 1, 0);
  for (int32_t i = 0; i < count; ++i) {
    if (!rs[i]) return set_error(MHS_EINVAL, "NULL result " + std::to_string(i));
    if (rs[i]->status)
      return set_error(rs[i]->status, "result " + std::to_string(i) + " failed: " + rs[i]->error);
    mo[i + 1] = mo[i] + (size_t)rs[i]->m;
    no[i + 1] = no[i] + (size_t)rs[i]->n;
  }
  parallel_for(count, [&](int32_t i) {
    const mhs_result* r = rs[i];
    if (sums) mhs_result_summary(r, &sums[i]);
    if (stats) stats[i] = r->stats;
    if (death_e && r->m) std::memcpy(death_e + mo[i], r->death_e.data(), (size_t)r->m * 4);
    if (demand && r->m) std::memcpy(demand + mo[i], r->demand.data(), (size_t)r->m * 4);
    if (death_v && r->n) std::memcpy(death_v + no[i], r->death_v.data(), (size_t)r->n * 4);
    if (forced && r->n) std::memcpy(forced + no[i], r->forced.data(), (size_t)r->n);
    delete r;
    rs[i] = nullptr;
  });
  return MHS_OK;
}

}  // extern "C"
