// server.cpp -- continuous batching over a caller-provided device arena.
//
// Requests are validated and copied at submit and queued on the host.  The
// server advances in steps.  A step is the GPU work one poll queues on the
// stream, in this order:
//   1. retirement: the members found finished when the last step was
//      harvested are read back (counters, deletion rounds, forced flags,
//      demands) into pinned memory, and their arena ranges and slots are
//      freed at once (stream order keeps those copies ahead of any later
//      write to the ranges);
//   2. admission: queued requests in arrival order while a slot and arena
//      space are free (first fit over a free list, never overcommitting):
//      their compact copies (32-bit offsets, 16-bit vertex ids when they
//      fit) cross the bus from one pinned image, are widened on the device
//      and prepared together;
//   3. one round of Algorithm 3 over every resident instance in shared
//      launches, then every member's counters into pinned memory;
//   4. an event.
// At most two steps are in flight: a poll queues the next step before the
// counters of the previous one are read, and never waits for the device.  A
// step whose event has passed is harvested: the results read back in it are
// built on the host threads and queued for return, and the members whose
// counters say done (or failed) are retired by the next step.  Each instance
// keeps its own round counter, so its result does not depend on what else
// is resident.
#include "host.h"

#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

using namespace mhsk;

struct mhs_result;  // defined in abi.cpp
namespace mhsk {
mhs_result* make_result_public(const HostInst& h, const std::vector<int32_t>& ctr, std::vector<int32_t>&& de,
                               std::vector<int32_t>&& dv, std::vector<int32_t>&& fw,
                               std::vector<uint8_t>&& forced);
mhs_result* make_failed_result(const HostInst& h, int code);
int validate_host_public(const mhs_instance* in, int64_t* nnz, std::string* why);
}  // namespace mhsk

namespace {

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Request {
  uint64_t id = 0;
  int32_t n = 0, m = 0;
  int64_t nnz = 0, k = 0;
  // the host copy, compact (compact_layout: 32-bit offsets, vertex ids as
  // uint16 when n <= 65536), written while it is validated; widened when it
  // is uploaded
  std::unique_ptr<char[]> img;
  CompactLayout C;
  size_t footprint = 0;
  int variant = 1;
};

struct Resident {
  uint64_t id = 0;
  uint64_t uid = 0;      // unique per admission (request ids may repeat)
  HostInst h;
  size_t off = 0, size = 0;
  bool retiring = false; // finished: the next step retires it
  int err = 0;           // device error code (C_ERR) of a failed request
};

// A member retired in a step: where its result lands in the step's readback.
struct Retired {
  uint64_t id = 0;
  HostInst h;
  size_t off = 0;
};

// Pinned host buffer that grows on demand (only while no copy uses it).
struct Pinned {
  char* p = nullptr;
  size_t cap = 0;
  char* get(size_t bytes) {
    if (bytes > cap) {
      if (p) (void)hipHostFree(p);
      p = nullptr;
      cap = 0;
      const size_t want = std::max(bytes + bytes / 4, (size_t)1 << 16);
      if (hipHostMalloc((void**)&p, want, hipHostMallocDefault) != hipSuccess) { p = nullptr; return nullptr; }
      cap = want;
    }
    return p;
  }
  ~Pinned() { if (p) (void)hipHostFree(p); }
};

struct Step {
  hipEvent_t ev = nullptr;
  bool busy = false;
  std::vector<uint64_t> uids;      // members of the step's round, in set order
  std::vector<Retired> retired;    // read back in this step
  Pinned ctr, rb, up, tab;         // counters, readback, upload image, set tables
};

// First-fit allocator over [0, size) of the arena's instance region.
class FreeList {
 public:
  void reset(size_t size) { free_.clear(); if (size) free_[0] = size; used_ = 0; }
  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t noff = it->first + bytes;
        free_.erase(it);
        if (rest) free_[noff] = rest;
        used_ += bytes;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }

 private:
  std::map<size_t, size_t> free_;
  size_t used_ = 0;
};

}  // namespace

struct mhs_server {
  char* arena = nullptr;
  size_t arena_bytes = 0;
  int32_t max_slots = 0;
  uint32_t flags = 0;
  hipStream_t stream = nullptr;
  char* ctrl_set = nullptr;      // control block of the resident set
  char* ctrl_new = nullptr;      // control block of the newly admitted subset
  size_t ctrl_bytes = 0;
  WidenJob* jobs = nullptr;      // device: widening jobs of an admission (max_slots)
  size_t jobs_bytes = 0;
  char* pool = nullptr;          // instance slices
  size_t pool_bytes = 0;
  FreeList fl;
  std::mutex qmu;                // guards queue (submit may run on another thread)
  std::deque<Request> queue;
  std::vector<Resident> res;
  std::deque<std::pair<uint64_t, mhs_result*>> finished;
  Set set;
  bool dirty = true;             // the resident set changed: rebuild its tables
  Step steps[2];
  int next_step = 0;             // slot of the next step to queue
  int inflight = 0;              // steps queued and not yet harvested
  uint64_t next_uid = 1;
  int64_t fail_id = -1;          // test hook: this request's upload is corrupted
};

namespace {

bool queue_empty(mhs_server* s) {
  std::lock_guard<std::mutex> g(s->qmu);
  return s->queue.empty();
}

bool has_work(mhs_server* s) { return !s->res.empty() || !queue_empty(s); }

// Harvest the steps whose event has passed, oldest first (with `wait`, the
// oldest one is waited for).
int harvest(mhs_server* s, bool wait) {
  while (s->inflight > 0) {
    Step& st = s->steps[(s->next_step + 2 - s->inflight) % 2];
    const hipError_t q = wait ? hipEventSynchronize(st.ev) : hipEventQuery(st.ev);
    if (q == hipErrorNotReady) return MHS_OK;
    if (q != hipSuccess) return set_error(MHS_EDEVICE, "server step failed on the device");
    wait = false;
    // results read back in this step, built on the host threads
    std::vector<mhs_result*> made(st.retired.size(), nullptr);
    parallel_for((int32_t)st.retired.size(), [&](int32_t k) {
      const HostInst& h = st.retired[k].h;
      const char* b = st.rb.p + st.retired[k].off;
      const int32_t* c = (const int32_t*)(b + h.L.off_ctr);
      std::vector<int32_t> ctr(c, c + kCtr);
      const int32_t* de = (const int32_t*)(b + h.L.off_death_e);
      const int32_t* dv = (const int32_t*)(b + h.L.off_death_v);
      const uint8_t* fo = (const uint8_t*)(b + h.L.off_forced);
      const int32_t* fw = (const int32_t*)(b + h.L.off_fw);
      made[k] = make_result_public(h, ctr, std::vector<int32_t>(de, de + h.m), std::vector<int32_t>(dv, dv + h.n),
                                   std::vector<int32_t>(fw, fw + h.m), std::vector<uint8_t>(fo, fo + h.n));
    });
    for (size_t k = 0; k < made.size(); ++k) s->finished.emplace_back(st.retired[k].id, made[k]);
    st.retired.clear();
    // members that reached their fixpoint (or failed) in this step's round
    if (!st.uids.empty()) {
      std::unordered_map<uint64_t, size_t> at;
      for (size_t x = 0; x < s->res.size(); ++x) at[s->res[x].uid] = x;
      const int32_t* ctr = (const int32_t*)st.ctr.p;
      for (size_t i = 0; i < st.uids.size(); ++i) {
        auto it = at.find(st.uids[i]);
        if (it == at.end()) continue;   // retired since
        Resident& r = s->res[it->second];
        const int32_t* c = ctr + i * kCtr;
        if (r.retiring) continue;
        if (c[C_ERR]) {
          r.retiring = true;
          r.err = c[C_ERR];
        } else if (c[C_DONE]) {
          r.retiring = true;
        }
      }
      st.uids.clear();
    }
    st.busy = false;
    --s->inflight;
  }
  return MHS_OK;
}

// Step part 1: read back and free the finished members.  The copies are
// queued first; the members leave the set only when all were queued.
int retire(mhs_server* s, Step& st) {
  size_t total = 0;
  for (const Resident& r : s->res)
    if (r.retiring && !r.err) total += align_up(r.h.L.off_fw + (size_t)r.h.m * 4, 256);
  if (total && !st.rb.get(total)) return set_error(MHS_EDEVICE, "pinned allocation failed");
  size_t o = 0;
  for (const Resident& r : s->res) {
    if (!r.retiring || r.err) continue;
    const size_t bytes = r.h.L.off_fw + (size_t)r.h.m * 4;
    if (hipMemcpyAsync(st.rb.p + o, r.h.slice, bytes, hipMemcpyDeviceToHost, s->stream) != hipSuccess)
      return set_error(MHS_EDEVICE, "result readback failed");
    Retired d;
    d.id = r.id;
    d.h = r.h;
    d.off = o;
    st.retired.push_back(d);
    o += align_up(bytes, 256);
  }
  std::vector<Resident> keep;
  keep.reserve(s->res.size());
  for (Resident& r : s->res) {
    if (!r.retiring) {
      keep.push_back(std::move(r));
      continue;
    }
    if (r.err) s->finished.emplace_back(r.id, make_failed_result(r.h, r.err));
    s->fl.release(r.off, r.size);
    s->dirty = true;
  }
  s->res.swap(keep);
  return MHS_OK;
}

// Step part 2: admission.  Requests leave the queue only when their upload
// and prepare have been queued; on a failure they go back to its front and
// their arena ranges are released.
int admit(mhs_server* s, Step& st) {
  std::vector<Request> take;
  std::vector<size_t> offs;
  {
    std::lock_guard<std::mutex> g(s->qmu);
    while (!s->queue.empty() && (int32_t)(s->res.size() + take.size()) < s->max_slots) {
      size_t off = 0;
      if (!s->fl.alloc(s->queue.front().footprint, &off)) break;   // FIFO: wait for space
      take.push_back(std::move(s->queue.front()));
      s->queue.pop_front();
      offs.push_back(off);
    }
  }
  if (take.empty()) return MHS_OK;
  auto rollback = [&](int rc) {
    for (size_t k = 0; k < take.size(); ++k) s->fl.release(offs[k], take[k].footprint);
    std::lock_guard<std::mutex> g(s->qmu);
    for (size_t k = take.size(); k-- > 0;) s->queue.push_front(std::move(take[k]));
    return rc;
  };
  const size_t K = take.size();
  std::vector<HostInst> hs(K);
  std::vector<size_t> po(K + 1, 0);
  for (size_t k = 0; k < K; ++k) {
    const Request& q = take[k];
    HostInst& h = hs[k];
    h.n = q.n;
    h.m = q.m;
    h.nnz = q.nnz;
    h.k = q.k;
    h.L = inst_layout(h.n, h.m, h.nnz, true, true);
    h.variant = q.variant;
    h.rule_se = (s->flags & MHS_RULE_SE) ? 1 : 0;
    h.rule_fe = (s->flags & MHS_RULE_FE) ? 1 : 0;
    h.slice = s->pool + offs[k];
    h.ptr = (const int64_t*)(h.slice + h.L.off_in_ptr);
    h.vtx = (const int32_t*)(h.slice + h.L.off_in_vtx);
    h.dem = (const int32_t*)(h.slice + h.L.off_in_dem);
    po[k + 1] = po[k] + (h.m > 0 ? align_up(q.C.bytes, 256) : 0);
  }
  // the requests' compact copies, one after the other behind their widening
  // jobs, in one pinned image; each copy lands in its slice's compact area
  // and is widened there on the device
  const size_t jb = align_up(K * sizeof(WidenJob), 256);
  char* img = st.up.get(jb + po[K] + 1);
  if (!img) return rollback(set_error(MHS_EDEVICE, "pinned allocation failed"));
  WidenJob* jobs = reinterpret_cast<WidenJob*>(img);
  parallel_for((int32_t)K, [&](int32_t k) {
    const HostInst& h = hs[k];
    const CompactLayout& C = take[k].C;
    WidenJob J;
    std::memset(&J, 0, sizeof(J));
    J.m = h.m;
    J.nnz = h.nnz;
    J.vtx16 = C.v16 ? 1 : 0;
    if (h.m > 0) {
      char* b = img + jb + po[k];
      std::memcpy(b, take[k].img.get(), C.bytes);
      // test hook: an out-of-range demand, which the device-side validation
      // reports for this request alone
      if ((int64_t)take[k].id == s->fail_id) reinterpret_cast<int32_t*>(b + C.dem)[0] = 0;
      char* c = h.slice + h.L.off_in_cmp;
      J.sptr = (const int32_t*)(c + C.ptr);
      J.svtx = c + C.vtx;
      J.sdem = (const int32_t*)(c + C.dem);
      J.dptr = (int64_t*)h.ptr;
      J.dvtx = (int32_t*)h.vtx;
      J.ddem = (int32_t*)h.dem;
    }
    jobs[k] = J;
  });
  for (size_t k = 0; k < K; ++k) {
    const HostInst& h = hs[k];
    if (h.m == 0) continue;
    if (hipMemcpyAsync(h.slice + h.L.off_in_cmp, img + jb + po[k], take[k].C.bytes, hipMemcpyHostToDevice,
                       s->stream) != hipSuccess)
      return rollback(set_error(MHS_EDEVICE, "request upload failed"));
  }
  if (hipMemcpyAsync(s->jobs, jobs, K * sizeof(WidenJob), hipMemcpyHostToDevice, s->stream) != hipSuccess)
    return rollback(set_error(MHS_EDEVICE, "request upload failed"));
  launch_widen(s->stream, s->jobs, (int)K);
  char* tab = st.tab.get(2 * s->ctrl_bytes);
  if (!tab) return rollback(set_error(MHS_EDEVICE, "pinned allocation failed"));
  Set prep;
  prep.variant = s->set.variant;
  prep.stage = tab;
  prep.stage_bytes = s->ctrl_bytes;
  int rc = prep.build(hs, s->ctrl_new, s->ctrl_bytes, s->stream);
  if (rc) return rollback(rc);
  launch_prepare(prep.ctx);
  if (hipGetLastError() != hipSuccess) return rollback(set_error(MHS_EDEVICE, "prepare launch failed"));
  // committed (the host copies go: the pinned image holds what the copies read)
  for (size_t k = 0; k < K; ++k) {
    Resident r;
    r.id = take[k].id;
    r.uid = s->next_uid++;
    r.off = offs[k];
    r.size = take[k].footprint;
    r.h = hs[k];
    s->res.push_back(std::move(r));
  }
  s->dirty = true;
  return MHS_OK;
}

// Queue one step (the slot of the next step is free: at most one step is in
// flight when this runs).
int launch_step(mhs_server* s) {
  Step& st = s->steps[s->next_step];
  st.retired.clear();
  st.uids.clear();
  int rc = retire(s, st);
  if (rc) return rc;
  rc = admit(s, st);
  if (rc) return rc;
  if (!s->res.empty()) {
    if (s->dirty) {
      std::vector<HostInst> hs;
      hs.reserve(s->res.size());
      for (const Resident& r : s->res) hs.push_back(r.h);
      char* tab = st.tab.get(2 * s->ctrl_bytes);
      if (!tab) return set_error(MHS_EDEVICE, "pinned allocation failed");
      s->set.stage = tab + s->ctrl_bytes;
      s->set.stage_bytes = s->ctrl_bytes;
      rc = s->set.build(hs, s->ctrl_set, s->ctrl_bytes, s->stream);
      if (rc) return rc;
      s->dirty = false;
    }
    rc = s->set.launch_round(false);
    if (rc) return rc;
    int32_t* c = (int32_t*)st.ctr.get(s->res.size() * kCtr * 4);
    if (!c) return set_error(MHS_EDEVICE, "pinned allocation failed");
    rc = s->set.enqueue_counters(c);
    if (rc) return rc;
    for (const Resident& r : s->res) st.uids.push_back(r.uid);
  }
  if (hipEventRecord(st.ev, s->stream) != hipSuccess) return set_error(MHS_EDEVICE, "event record failed");
  st.busy = true;
  ++s->inflight;
  s->next_step ^= 1;
  return MHS_OK;
}

}  // namespace

extern "C" {

int mhs_server_create(void* d_arena, size_t arena_bytes, int32_t max_slots, uint32_t flags, void* hip_stream,
                      mhs_server** out) {
  if (!out) return set_error(MHS_EINVAL, "NULL out");
  *out = nullptr;
  if (!d_arena || ((uintptr_t)d_arena & 255)) return set_error(MHS_EINVAL, "arena NULL or not 256-byte aligned");
  if (max_slots < 1) return set_error(MHS_EINVAL, "max_slots < 1");
  if (flags & ~(uint32_t)(MHS_VARIANT_MASK | MHS_TRACE_ROUNDS | MHS_NO_GRAPH | MHS_GRAPH | MHS_GRID_MASK |
                          MHS_GEMM_SCHED_MASK | MHS_RULE_SE | MHS_RULE_FE))
    return set_error(MHS_EINVAL, "unsupported server flags");
  const uint32_t v = flags & MHS_VARIANT_MASK;
  if (v > MHS_VARIANT_HYBRID) return set_error(MHS_EINVAL, "unknown contraction variant");
  if (((flags & MHS_GRID_MASK) >> 24) > 5) return set_error(MHS_EINVAL, "grid exponent above 4");
  mhs_server* s = new mhs_server();
  s->arena = (char*)d_arena;
  s->arena_bytes = arena_bytes;
  s->max_slots = max_slots;
  s->flags = flags;
  s->stream = (hipStream_t)hip_stream;
  s->ctrl_bytes = align_up(set_control_bytes(max_slots), 256);
  s->jobs_bytes = align_up((size_t)max_slots * sizeof(WidenJob), 256);
  const size_t fixed = 2 * s->ctrl_bytes + s->jobs_bytes;
  if (arena_bytes < fixed + 4096) {
    delete s;
    return set_error(MHS_ENOSPC, "arena smaller than the control blocks");
  }
  s->ctrl_set = s->arena;
  s->ctrl_new = s->arena + s->ctrl_bytes;
  s->jobs = reinterpret_cast<WidenJob*>(s->arena + 2 * s->ctrl_bytes);
  s->pool = s->arena + fixed;
  s->pool_bytes = (arena_bytes - fixed) / 256 * 256;
  s->fl.reset(s->pool_bytes);
  s->set.variant = variant_of(flags);
  s->set.per_cu = grid_per_cu(flags);
  s->set.gemm_sched = gemm_sched_of(flags);
  for (Step& st : s->steps)
    if (hipEventCreateWithFlags(&st.ev, hipEventDisableTiming) != hipSuccess) {
      for (Step& t : s->steps) if (t.ev) (void)hipEventDestroy(t.ev);
      delete s;
      return set_error(MHS_EDEVICE, "event creation failed");
    }
  const char* f = std::getenv("MHSK_SERVER_FAIL_ID");
  if (f && *f) s->fail_id = std::strtoll(f, nullptr, 10);
  *out = s;
  return MHS_OK;
}

int mhs_server_submit(mhs_server* s, const mhs_instance* in, uint64_t request_id) {
  if (!s || !in) return set_error(MHS_EINVAL, "NULL argument");
  Request r;
  std::string why;
  if (validate_shape(in, &r.nnz, &why)) return set_error(MHS_EINVAL, why);
  r.id = request_id;
  r.n = in->n;
  r.m = in->m;
  r.k = in->k;
  r.footprint = inst_layout(r.n, r.m, r.nnz, true, true).bytes;
  if (r.footprint > s->pool_bytes) {
    // an invalid request is reported as such before its size
    int64_t nnz = 0;
    if (validate_host_public(in, &nnz, &why)) return set_error(MHS_EINVAL, why);
    return set_error(MHS_EREJECT, "request footprint exceeds the arena");
  }
  r.C = compact_layout(r.n, r.m, r.nnz);
  if (r.m > 0) {
    r.img.reset(new (std::nothrow) char[r.C.bytes]);   // uninitialized: pack_compact writes every byte used
    if (!r.img) return set_error(MHS_ENOSPC, "host memory for the request copy");
  }
  double span = 0;
  if (pack_compact(in, r.nnz, r.C, r.img.get(), &span, &why)) return set_error(MHS_EINVAL, why);
  r.variant = variant_with_span(s->flags, in, span);
  std::lock_guard<std::mutex> g(s->qmu);
  s->queue.push_back(std::move(r));
  return MHS_OK;
}

int mhs_server_poll(mhs_server* s, int32_t cap, uint64_t* ids, mhs_result** results, int32_t* n_done) {
  if (!s || !n_done || cap < 0 || (cap > 0 && (!ids || !results))) return set_error(MHS_EINVAL, "bad poll arguments");
  *n_done = 0;
  int rc = harvest(s, false);
  if (rc) return rc;
  if (s->inflight < 2 && has_work(s)) {
    rc = launch_step(s);
    if (rc) return rc;
  }
  while (*n_done < cap && !s->finished.empty()) {
    ids[*n_done] = s->finished.front().first;
    results[*n_done] = s->finished.front().second;
    s->finished.pop_front();
    ++*n_done;
  }
  if (*n_done == 0) {
    if (s->inflight == 0 && s->finished.empty() && !has_work(s))
      return set_error(MHS_EAGAIN, "server idle: nothing queued or resident");
    return set_error(MHS_EAGAIN, "no request finished yet");
  }
  return MHS_OK;
}

int mhs_server_drain(mhs_server* s) {
  if (!s) return set_error(MHS_EINVAL, "NULL server");
  for (;;) {
    int rc = harvest(s, false);
    if (rc) return rc;
    if (s->inflight < 2 && has_work(s)) {
      rc = launch_step(s);
      if (rc) return rc;
      continue;
    }
    if (s->inflight == 0) return MHS_OK;   // nothing queued, resident or in flight
    rc = harvest(s, true);
    if (rc) return rc;
  }
}

int mhs_server_pending(const mhs_server* s, int32_t* queued, int32_t* resident) {
  if (!s) return set_error(MHS_EINVAL, "NULL server");
  mhs_server* w = const_cast<mhs_server*>(s);
  std::lock_guard<std::mutex> g(w->qmu);
  if (queued) *queued = (int32_t)w->queue.size();
  if (resident) *resident = (int32_t)w->res.size();
  return MHS_OK;
}

int mhs_server_arena_used(const mhs_server* s, size_t* used) {
  if (!s || !used) return set_error(MHS_EINVAL, "NULL argument");
  *used = s->fl.used() + 2 * s->ctrl_bytes + s->jobs_bytes;
  return MHS_OK;
}

void mhs_server_destroy(mhs_server* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  for (auto& f : s->finished) mhs_result_free(f.second);
  for (Step& st : s->steps) if (st.ev) (void)hipEventDestroy(st.ev);
  delete s;
}

}  // extern "C"
