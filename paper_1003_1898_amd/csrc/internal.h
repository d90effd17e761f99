// Internal interface between the host runtime (runtime.cpp) and the device
// code (kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

namespace prng {

enum Kind : int { GGL = 1, XOR128 = 2, RANECU = 3, RANMAR = 4, RANLUX = 5, MT19937 = 6 };
enum Dtype : int { U32 = 1, F32 = 2, F64 = 3 };

// Canonical per-stream state words (the blob layout).
constexpr int kStateWords[7] = {0, 1, 4, 2, 98, 26, 625};
// Seed tuple words per stream.
constexpr int kSeedWords[7] = {0, 1, 4, 2, 2, 1, 1};
// Native bit width of the integer draw.
constexpr int kBits[7] = {0, 31, 32, 31, 24, 24, 32};
// Device layout: lane-per-stream kinds keep the canonical words in
// structure-of-arrays order (word j of stream s at state[j*n + s]); MT19937
// keeps each stream's 625 words contiguous, padded to kMtStride words.
constexpr int kMtStride = 628;

inline bool lane_kind(int k) { return k >= GGL && k <= RANLUX; }
inline size_t elem_bytes(int dt) { return dt == F64 ? 8 : 4; }

// Largest number of draws per stream one kernel launch handles; the host
// splits longer requests into several launches.
constexpr uint64_t kMaxDrawsPerLaunch = 1ull << 30;

// Row descriptor of the stream-table kernel: one stream's work.
struct TableRow {
  uint32_t* state;    // device state base of the generator object
  uint64_t sn;        // that object's stream count (SoA stride)
  uint64_t si;        // stream index inside the object
  void* out;          // device pointer to element 0 of this row's output
  uint32_t draws;     // draws to produce (2 per element for f64)
  uint32_t pad;
};

// Work item of the stream-table kernel: up to 64 rows of one (kind, p, dtype).
struct TableTask {
  uint32_t kind;
  uint32_t p;
  uint32_t dtype;
  uint32_t nrows;     // rows in this task (lane-per-stream: <= 64; MT: 1)
  uint64_t row0;      // index of the first row in the row array
};

hipError_t launch_init(int kind, uint32_t* state, uint64_t n, const uint64_t* d_seeds, hipStream_t s);
hipError_t launch_generate(int kind, uint32_t p, uint32_t* state, uint64_t n, uint64_t draws, int dtype,
                           void* out, uint64_t row_elems, uint64_t elem_off, hipStream_t s);
hipError_t launch_fused(int kind, uint32_t p, uint32_t* state, uint64_t n, uint64_t draws, uint64_t* sum,
                        uint32_t* hist, bool accumulate, hipStream_t s);
hipError_t launch_table_reset(uint32_t* counters, int n, hipStream_t s);
hipError_t launch_table_lane(const TableTask* tasks, uint32_t ntasks, const TableRow* rows, uint32_t* counter,
                             int grid, hipStream_t s);
hipError_t launch_table_mt(const TableTask* tasks, uint32_t ntasks, const TableRow* rows, uint32_t* counter, int grid,
                           hipStream_t s);

}  // namespace prng
