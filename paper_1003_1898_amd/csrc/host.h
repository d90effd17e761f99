// Shared host-side declarations of libprng (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "internal.h"
#include "prng.h"

#define PRNG_API extern "C" __attribute__((visibility("default")))

namespace prng {

// Record a thread-local error message and return `code`.
int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
const char* last_error();

#define HIP_TRY(call)                                  \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return ::prng::hip_fail(e_, #call); \
  } while (0)

inline bool valid_kind(int k) { return k >= GGL && k < kKinds; }
inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }
inline size_t state_region_bytes(int kind, uint64_t n) {
  if (kind == MT19937) return align256(n * kMtStride * 4ull);
  return align256(n * (uint64_t)kStateWords[kind] * 4ull);
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) {
      if (hipSetDevice(dev) != hipSuccess) prev = -1;
    } else {
      prev = -1;
    }
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

// ------------------------------------------------------------ stream table
struct TableConfig {
  int lane_grid;
  int mt_grid;
  int concurrent;
};

// Device-resident jump data kept by a caller of make_plan (the server):
// lookup returns the device address of segment j's data for (kind, p) at
// segment length seg_len(kind), or nullptr.
struct JumpSource {
  virtual ~JumpSource() = default;
  virtual uint64_t seg_len(int kind) const = 0;
  virtual const uint32_t* lookup(int kind, uint32_t p, uint32_t j) const = 0;
  virtual const uint32_t* aux() const = 0;
};

// Everything a table needs in its workspace; pointers into the workspace are
// kept as offsets until the base address is known.
// Segment length per class of kind: 0 automatic, PRNG_SEG_NEVER never cut,
// otherwise that length (rounded as make_plan documents).
struct SegSpec {
  uint32_t lane = 0;    // GGL, XOR128, RANECU, RANLUX, DRAND48, RANNYU
  uint32_t ranmar = 0;  // RANMAR (automatic: four times the automatic lane length)
  uint32_t mt = 0;      // MT19937
};
// the single length of prng_table_create: the same for every kind
inline SegSpec seg_spec_of(uint32_t seg_len) { return SegSpec{seg_len, seg_len, seg_len}; }

struct Plan {
  std::vector<TableTask> lane_tasks[kLaneClasses], mt_tasks;
  std::vector<TableRow> rows;
  std::vector<uint8_t> row_snap;   // 1: `state` is the lane snapshot area, 2: the MT19937 one
  std::vector<int64_t> row_jump;   // >= 0: word offset of the row's segment-1 jump data in `jump`
  std::vector<int64_t> row_jslot;  // >= 0: MT19937 jumped-window slot of the row's segment 1
  std::vector<uint32_t> mt_jump_list;  // (row, segment) pairs whose window k_table_mt_jump builds
  std::vector<uint32_t> tails;         // rows of the tail tasks' lanes
  uint64_t n_jslots = 0, n_segments = 0;
  std::vector<SnapRow> snaps;
  std::vector<uint32_t> jump;
  std::vector<uint32_t> aux;
  std::vector<prng_gen*> gens;
  const uint32_t* ext_aux = nullptr;
  uint64_t total_draws = 0, max_draws = 0, max_task_draws = 0;
  SegSpec resolved{};  // the lengths used per class (0: not cut), before the per-row cap
  size_t o_tails = 0, o_lane[kLaneClasses] = {}, o_mt = 0, o_rows = 0, o_snaprows = 0, o_snap = 0, o_snap_mt = 0, o_jstate = 0, o_mtj = 0,
         o_jump = 0, o_aux = 0, total = 0;
};

int make_plan(prng_gen* const* gens, int n_gens, const prng_table_row* rows, uint64_t n_rows, const SegSpec& seg,
              const JumpSource* js, Plan& P);
// Upload a plan into d_work (>= P.total bytes) on `s` and build the table
// object; `sync` waits for the upload (otherwise the host vectors of P must
// stay alive until the upload has completed, i.e. until work queued behind
// it on `s` is done).
int table_from_plan(Plan& P, void* d_work, hipStream_t s, bool sync, bool graph_streams, prng_table** out);
hipError_t enqueue_run(prng_table* t, hipStream_t s);

}  // namespace prng

struct prng_gen {
  int kind;
  uint32_t p;
  uint64_t n;
  uint32_t* d_state;
  int device;
};

struct prng_table {
  std::vector<prng_gen*> gens;  // objects whose states the table advances
  uint32_t n_lane_tasks = 0, n_mt_tasks = 0, n_snaps = 0, snap_words = 98, n_mt_jumps = 0;
  uint32_t n_class_tasks[prng::kLaneClasses] = {};
  prng::TableTask* d_class_tasks[prng::kLaneClasses] = {};
  const uint32_t* d_mt_jumps = nullptr;
  const uint32_t* d_tails = nullptr;
  uint64_t total_draws = 0, max_draws = 0, max_task_draws = 0, n_segments = 0;
  uint32_t* d_counters = nullptr;
  prng::TableTask* d_mt_tasks = nullptr;
  prng::TableRow* d_rows = nullptr;
  prng::SnapRow* d_snaps = nullptr;
  const uint32_t* d_aux = nullptr;
  prng::TableConfig cfg{256, 512, 1};
  prng::SegSpec seg{};  // resolved segment lengths of the plan
  int device = 0;
  hipStream_t cap = nullptr, side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  // concurrency 2: lane classes 1.. on streams of their own, joined by events
  hipStream_t lane_side[prng::kLaneClasses - 1] = {};
  hipEvent_t lane_join[prng::kLaneClasses - 1] = {};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};
