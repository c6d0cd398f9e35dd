// server.cpp -- continuous batching over a caller-provided device arena.
//
// Requests are copied at submit and queued on the host.  Every poll admits
// queued requests in arrival order while a slot and enough arena space are
// free (first fit over a free list; nothing is ever overcommitted), prepares
// the newly admitted ones, runs ONE round of Algorithm 3 over every resident
// instance in shared launches, and retires the instances that reached their
// fixpoint, freeing their memory and slot at once.  Each instance keeps its
// own round counter, so an instance's result does not depend on what else
// is resident.
#include "host.h"

#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <mutex>
#include <string>
#include <vector>

using namespace mhsk;

struct mhs_result;  // defined in abi.cpp
namespace mhsk {
mhs_result* make_result_public(const HostInst& h, const std::vector<int32_t>& ctr, std::vector<int32_t>&& de,
                               std::vector<int32_t>&& dv, std::vector<int32_t>&& fw,
                               std::vector<uint8_t>&& forced);
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
  HostInst h;
  size_t off = 0, size = 0;
  Request req;      // host copy kept until the upload has completed
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
  char* pool = nullptr;          // instance slices
  size_t pool_bytes = 0;
  FreeList fl;
  std::mutex qmu;
  std::deque<Request> queue;
  std::vector<Resident> res;
  std::deque<std::pair<uint64_t, mhs_result*>> finished;
  Set set;
  bool dirty = true;
};

extern "C" {

int mhs_server_create(void* d_arena, size_t arena_bytes, int32_t max_slots, uint32_t flags, void* hip_stream,
                      mhs_server** out) {
  if (!out) return set_error(MHS_EINVAL, "NULL out");
  *out = nullptr;
  if (!d_arena || ((uintptr_t)d_arena & 255)) return set_error(MHS_EINVAL, "arena NULL or not 256-byte aligned");
  if (max_slots < 1) return set_error(MHS_EINVAL, "max_slots < 1");
  if (flags & ~(uint32_t)(MHS_VARIANT_MASK | MHS_NO_GRAPH | MHS_GRAPH | MHS_PROFILE | MHS_GRID_MASK | MHS_RULE_SE | MHS_RULE_FE))
    return set_error(MHS_EINVAL, "unsupported server flags");
  const uint32_t v = flags & MHS_VARIANT_MASK;
  if (v > MHS_VARIANT_SPARSE) return set_error(MHS_EINVAL, "unknown contraction variant");
  mhs_server* s = new mhs_server();
  s->arena = (char*)d_arena;
  s->arena_bytes = arena_bytes;
  s->max_slots = max_slots;
  s->flags = flags;
  s->stream = (hipStream_t)hip_stream;
  s->ctrl_bytes = align_up(set_control_bytes(max_slots), 256);
  if (arena_bytes < 2 * s->ctrl_bytes + 4096) {
    delete s;
    return set_error(MHS_ENOSPC, "arena smaller than the control blocks");
  }
  s->ctrl_set = s->arena;
  s->ctrl_new = s->arena + s->ctrl_bytes;
  s->pool = s->arena + 2 * s->ctrl_bytes;
  s->pool_bytes = (arena_bytes - 2 * s->ctrl_bytes) / 256 * 256;
  s->fl.reset(s->pool_bytes);
  s->set.variant = variant_of(flags);
  s->set.per_cu = grid_per_cu(flags);
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
  r.footprint = inst_layout(r.n, r.m, r.nnz, true).bytes;
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

static int admit(mhs_server* s, std::vector<size_t>* fresh) {
  std::lock_guard<std::mutex> g(s->qmu);
  while (!s->queue.empty() && (int32_t)s->res.size() < s->max_slots) {
    Request& q = s->queue.front();
    size_t off = 0;
    if (!s->fl.alloc(q.footprint, &off)) break;   // FIFO: wait for space, never overcommit
    Resident r;
    r.id = q.id;
    r.off = off;
    r.size = q.footprint;
    r.req = std::move(q);
    s->queue.pop_front();
    HostInst& h = r.h;
    h.n = r.req.n;
    h.m = r.req.m;
    h.nnz = r.req.nnz;
    h.k = r.req.k;
    h.L = inst_layout(h.n, h.m, h.nnz, true);
    h.variant = r.req.variant;
    h.rule_se = (s->flags & MHS_RULE_SE) ? 1 : 0;
    h.rule_fe = (s->flags & MHS_RULE_FE) ? 1 : 0;
    h.slice = s->pool + off;
    h.ptr = (const int64_t*)(h.slice + h.L.off_in_ptr);
    h.vtx = (const int32_t*)(h.slice + h.L.off_in_vtx);
    h.dem = (const int32_t*)(h.slice + h.L.off_in_dem);
    fresh->push_back(s->res.size());
    s->res.push_back(std::move(r));
  }
  return MHS_OK;
}

int mhs_server_poll(mhs_server* s, int32_t cap, uint64_t* ids, mhs_result** results, int32_t* n_done) {
  if (!s || !n_done || cap < 0 || (cap > 0 && (!ids || !results))) return set_error(MHS_EINVAL, "bad poll arguments");
  *n_done = 0;
  std::vector<size_t> fresh;
  admit(s, &fresh);
  if (!fresh.empty()) {
    // the admitted requests' inputs, laid out as their slices' staging areas
    // expect them, packed into one pinned image: one copy per request, from
    // pinned memory
    std::vector<size_t> po(fresh.size() + 1, 0);
    for (size_t k = 0; k < fresh.size(); ++k) {
      const HostInst& h = s->res[fresh[k]].h;
      po[k + 1] = po[k] + (h.m > 0 ? align_up(h.L.off_in_dem + (size_t)h.m * 4 - h.L.off_in_ptr, 256) : 0);
    }
    char* img = (char*)pinned_upload(std::max<size_t>(po.back(), 1));
    if (!img) return set_error(MHS_EDEVICE, "pinned allocation failed");
    // widened into the image on the host threads, then one copy each
    parallel_for((int32_t)fresh.size(), [&](int32_t k) {
      const Resident& r = s->res[fresh[k]];
      const HostInst& h = r.h;
      if (h.m == 0) return;
      char* b = img + po[k];
      const CompactLayout& C = r.req.C;
      const char* src = r.req.img.get();
      int64_t* dp = (int64_t*)b;
      const int32_t* sp = (const int32_t*)(src + C.ptr);
      for (int32_t e = 0; e <= h.m; ++e) dp[e] = sp[e];
      int32_t* dv = (int32_t*)(b + (h.L.off_in_vtx - h.L.off_in_ptr));
      if (C.v16) {
        const uint16_t* sv = (const uint16_t*)(src + C.vtx);
        for (int64_t q = 0; q < h.nnz; ++q) dv[q] = sv[q];
      } else if (h.nnz > 0) {
        std::memcpy(dv, src + C.vtx, (size_t)h.nnz * 4);
      }
      std::memcpy(b + (h.L.off_in_dem - h.L.off_in_ptr), src + C.dem, (size_t)h.m * 4);
    });
    std::vector<HostInst> hs;
    for (size_t k = 0; k < fresh.size(); ++k) {
      const HostInst& h = s->res[fresh[k]].h;
      if (h.m > 0) {
        const size_t span = h.L.off_in_dem + (size_t)h.m * 4 - h.L.off_in_ptr;
        if (hipMemcpyAsync((void*)h.ptr, img + po[k], span, hipMemcpyHostToDevice, s->stream) != hipSuccess)
          return set_error(MHS_EDEVICE, "request upload failed");
      }
      hs.push_back(h);
    }
    Set prep;
    prep.variant = s->set.variant;
    int rc = prep.build(hs, s->ctrl_new, s->ctrl_bytes, s->stream);
    if (rc) return rc;
    launch_prepare(prep.ctx);
    // the prepare tables live in host vectors of `prep`: finish before it goes
    if (hipStreamSynchronize(s->stream) != hipSuccess) return set_error(MHS_EDEVICE, "prepare failed");
    for (size_t i : fresh) s->res[i].req.img.reset();
    s->dirty = true;
  }
  if (!s->res.empty()) {
    if (s->dirty) {
      std::vector<HostInst> hs;
      for (const Resident& r : s->res) hs.push_back(r.h);
      int rc = s->set.build(hs, s->ctrl_set, s->ctrl_bytes, s->stream);
      if (rc) return rc;
      s->dirty = false;
    }
    int rc = s->set.launch_round(false);
    if (rc) return rc;
    std::vector<int32_t> ctrs;
    rc = s->set.read_counters(ctrs);
    if (rc) return rc;
    // the finished members' results (the front of each slice: counters,
    // deletion rounds, forced flags, working demands), read back together
    std::vector<size_t> fin, ro(1, 0);
    for (size_t x = 0; x < s->res.size(); ++x) {
      const int32_t* c = &ctrs[x * kCtr];
      if (c[C_DONE] || c[C_ERR]) {
        const HostInst& h = s->res[x].h;
        fin.push_back(x);
        ro.push_back(ro.back() + align_up(h.L.off_fw + (size_t)h.m * 4, 256));
      }
    }
    if (!fin.empty()) {
      char* p = (char*)pinned_buffer(ro.back());
      if (!p) return set_error(MHS_EDEVICE, "pinned allocation failed");
      for (size_t k = 0; k < fin.size(); ++k) {
        const HostInst& h = s->res[fin[k]].h;
        if (hipMemcpyAsync(p + ro[k], h.slice, h.L.off_fw + (size_t)h.m * 4, hipMemcpyDeviceToHost, s->stream) !=
            hipSuccess)
          return set_error(MHS_EDEVICE, "result readback failed");
      }
      if (hipStreamSynchronize(s->stream) != hipSuccess) return set_error(MHS_EDEVICE, "result readback failed");
      // results built on the host threads, handed out in member order
      std::vector<mhs_result*> made(fin.size(), nullptr);
      parallel_for((int32_t)fin.size(), [&](int32_t k) {
        const HostInst& h = s->res[fin[k]].h;
        const char* q = p + ro[k];
        std::vector<int32_t> ctr((const int32_t*)(q + h.L.off_ctr), (const int32_t*)(q + h.L.off_ctr) + kCtr);
        std::vector<int32_t> de((const int32_t*)(q + h.L.off_death_e), (const int32_t*)(q + h.L.off_death_e) + h.m);
        std::vector<int32_t> dv((const int32_t*)(q + h.L.off_death_v), (const int32_t*)(q + h.L.off_death_v) + h.n);
        std::vector<uint8_t> forced((const uint8_t*)(q + h.L.off_forced), (const uint8_t*)(q + h.L.off_forced) + h.n);
        std::vector<int32_t> fw((const int32_t*)(q + h.L.off_fw), (const int32_t*)(q + h.L.off_fw) + h.m);
        made[k] = make_result_public(h, ctr, std::move(de), std::move(dv), std::move(fw), std::move(forced));
      });
      for (size_t k = 0; k < fin.size(); ++k) {
        const Resident& r = s->res[fin[k]];
        s->finished.emplace_back(r.id, made[k]);
        s->fl.release(r.off, r.size);
      }
      s->dirty = true;
    }
    std::vector<Resident> keep;
    size_t k = 0;
    for (size_t x = 0; x < s->res.size(); ++x) {
      if (k < fin.size() && fin[k] == x) { ++k; continue; }
      keep.push_back(std::move(s->res[x]));
    }
    s->res.swap(keep);
  }
  while (*n_done < cap && !s->finished.empty()) {
    ids[*n_done] = s->finished.front().first;
    results[*n_done] = s->finished.front().second;
    s->finished.pop_front();
    ++*n_done;
  }
  if (*n_done == 0 && s->res.empty()) {
    std::lock_guard<std::mutex> g(s->qmu);
    if (s->queue.empty()) return set_error(MHS_EAGAIN, "server idle: nothing queued or resident");
  }
  return MHS_OK;
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
  *used = s->fl.used() + 2 * s->ctrl_bytes;
  return MHS_OK;
}

void mhs_server_destroy(mhs_server* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  for (auto& f : s->finished) mhs_result_free(f.second);
  delete s;
}

}  // extern "C"
