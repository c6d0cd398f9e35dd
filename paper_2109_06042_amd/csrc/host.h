// host.h -- host-side objects of the engine (sets of resident instances).
#pragma once
#include "engine.h"
#include "../../include/mhsk.h"

#include <functional>
#include <string>
#include <vector>

namespace mhsk {

// Runs f(0..count-1) on the library's pool of up to 16 host threads, the
// caller included (inline for small counts); returns when all have run.
void parallel_for(int32_t count, const std::function<void(int32_t)>& f);

// Records the thread-local error message and returns `code`.
int set_error(int code, const std::string& msg);
// 1: int8 MFMA, 2: bitset popcount (from the MHS_VARIANT_* flag bits).
int variant_of(uint32_t flags);
// Persistent contraction workgroups per CU (from the MHS_GRID_* bits).
int grid_per_cu(uint32_t flags);
// int8 operand staging k of MHS_GEMM_SCHED, or -1 (no bits: default).
int gemm_sched_of(uint32_t flags);
// Contraction variant of one instance (1 int8, 2 bitset, 3 sparse).
int instance_variant(uint32_t flags, const mhs_instance* in);

// A host instance's compact copy: 32-bit offsets, vertex ids as uint16 when
// every id fits (n <= 65536) else int32, demands; each part 256-aligned.
struct CompactLayout {
  size_t ptr = 0, vtx = 0, dem = 0, bytes = 0;
  bool v16 = false;
};
CompactLayout compact_layout(int32_t n, int32_t m, int64_t nnz);
// Sizes and pointers of a host instance (edge_ptr[0] and edge_ptr[m] only);
// *nnz receives edge_ptr[m].  Returns 0 or an error code, *why the reason.
int validate_shape(const mhs_instance* in, int64_t* nnz, std::string* why);
// One pass over an instance that passed validate_shape: every check of the
// full validation (same order and messages), the span sum the variant rule
// needs, and the compact copy written to b (compact_layout bytes).
int pack_compact(const mhs_instance* in, int64_t nnz, const CompactLayout& C, char* b, double* span,
                 std::string* why);
// instance_variant from a span sum pack_compact computed.
int variant_with_span(uint32_t flags, const mhs_instance* in, double span);

// One resident instance: its input arrays (device pointers: the caller's or
// the staged copy in its slice) and its slice of device memory.
struct HostInst {
  int32_t n = 0, m = 0;
  int64_t nnz = 0;
  int64_t k = 0;
  const int64_t* ptr = nullptr;
  const int32_t* vtx = nullptr;
  const int32_t* dem = nullptr;
  char* slice = nullptr;
  InstLayout L;
  int variant = 1;       // 1 int8, 2 bitset, 3 sparse
  int rule_se = 0;       // superedge rule SE in place of DP
  int rule_fe = 0;       // full-edge rule FE alternated with DP + MD
};

struct EventPool {
  std::vector<hipEvent_t> ev;
  hipEvent_t get(int i);
  ~EventPool();
};

DInst make_dinst(const HostInst& h);
void* pinned_buffer(size_t bytes);
void* pinned_upload(size_t bytes);
int32_t* pinned_flags(int32_t** dev);
int device_cu_count();

// A set of instances reduced together, round by round.
class Set {
 public:
  LaunchCtx ctx;
  std::vector<HostInst> members;
  bool profile = false;
  int variant = 1;
  int per_cu = 4;
  int gemm_sched = -1;   // int8 operand staging (MHS_GEMM_SCHED k), -1: default
  int32_t max_n = 0, max_m = 0;

  ~Set();
  // Lays the control block out in `control` and uploads the tables.
  int build(const std::vector<HostInst>& insts, char* control, size_t control_bytes, hipStream_t stream);
  // One round over every member that has not reached its fixpoint; with
  // `use_graph` the round is captured once into a hipGraph and replayed.
  int launch_round(bool use_graph) { return launch_rounds(use_graph, 1); }
  // k consecutive rounds (one graph of k rounds with `use_graph`).
  int launch_rounds(bool use_graph, int k);
  // Rounds per graph launch in run_to_fixpoint (1..kMaxRoundsPerLaunch):
  // fewer launches on the host and fewer graph boundaries on the device,
  // against up to 2k - 1 rounds of no-op kernels after the fixpoint.
  int rounds_per_launch = 2;
  // Rounds until no instance changes (max_iter bounds them); *iters receives
  // the number of iterations the host waited for.
  int run_to_fixpoint(bool use_graph, int64_t max_iter, int32_t* iters);
  int read_any(int* any);
  int read_counters(std::vector<int32_t>& out);
  // Queues the counters of every member (kCtr words each, member order)
  // for a copy into host memory at `dst` (pinned); no synchronization.
  int enqueue_counters(int32_t* dst);
  // Pinned host memory for the table upload of build() (at least the
  // control block's bytes), or null: then the upload reads a host vector,
  // and the caller must not rebuild before the copy has completed.
  char* stage = nullptr;
  size_t stage_bytes = 0;
  int read_member(int32_t x, std::vector<int32_t>& ctr, std::vector<int32_t>& de, std::vector<int32_t>& dv,
                  std::vector<uint8_t>* forced = nullptr, std::vector<int32_t>* fw = nullptr);
  enum { STEP_ROWS = 0, STEP_SPARSE_E, STEP_GEMM_E, STEP_SPARSE_V, STEP_GEMM_V, STEP_COMPACT, STEP_ROUND_END, kSteps };
  void collect_profile(double* step_ms);

 private:
  void launch_round_direct();
  bool split_branches() const;   // sparse and dense branches of a phase on two streams
  std::vector<DInst> h_dinst;
  std::vector<int32_t> h_pref;
  std::vector<int64_t> h_ooff;
  std::vector<char> h_image;     // host image of the uploaded table region
  int32_t* ctr_area = nullptr;
  EventPool ev_pool;
  int ev_used = 0;
};

}  // namespace mhsk
