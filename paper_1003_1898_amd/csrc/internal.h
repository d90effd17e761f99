// Internal interface between the host runtime (runtime.cpp, table.cpp,
// server.cpp) and the device code (device.h and the k_*.hip translation
// units).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

namespace prng {

enum Kind : int { GGL = 1, XOR128 = 2, RANECU = 3, RANMAR = 4, RANLUX = 5, MT19937 = 6, DRAND48 = 7, RANNYU = 8 };
constexpr int kKinds = 9;  // table size: kinds are 1 .. kKinds - 1
// F32P: single precision by the generator's own scaling as the paper writes it
// (plain generation only).
enum Dtype : int { U32 = 1, F32 = 2, F64 = 3, F32P = 4 };

// Canonical per-stream state words (the blob layout).
constexpr int kStateWords[kKinds] = {0, 1, 4, 2, 98, 26, 625, 2, 2};
// Seed tuple words per stream.
constexpr int kSeedWords[kKinds] = {0, 1, 4, 2, 2, 1, 1, 1, 1};
// Native bit width of the integer draw.
constexpr int kBits[kKinds] = {0, 31, 32, 31, 24, 24, 32, 32, 32};
// Device layout: lane-per-stream kinds keep the canonical words in
// structure-of-arrays order (word j of stream s at state[j*n + s]); MT19937
// keeps each stream's 625 words contiguous, padded to kMtStride words.
constexpr int kMtStride = 628;

inline bool lane_kind(int k) { return (k >= GGL && k <= RANLUX) || k == DRAND48 || k == RANNYU; }
inline size_t elem_bytes(int dt) { return dt == F64 ? 8 : 4; }

// Largest number of draws per stream one kernel launch handles; the host
// splits longer requests into several launches.
constexpr uint64_t kMaxDrawsPerLaunch = 1ull << 30;

// Row descriptor of the stream-table kernel: one segment of one stream.
// A stream's draws may be split into segments of `seg_len` virtual positions;
// segment j > 0 starts from the stream's state jumped ahead to position
// j * seg_len (jump data below), and only the last segment writes the final
// state back.
struct TableRow {
  uint32_t* state;       // where the starting state is read (snapshot when the row is cut)
  uint64_t sn;           // SoA stride of `state`
  uint64_t si;           // index inside `state`
  uint32_t* wstate;      // where the final state is written (by the last segment)
  uint64_t wsn;
  uint64_t wsi;
  void* out;             // address of the row's element 0
  uint32_t draws;        // the row's draws (2 per element for f64)
  uint32_t seg_len;      // positions per segment (0: not cut)
  uint64_t first;        // index of the row's segment 0 among its group's full segments
  uint32_t nseg;         // segments of the row
  uint32_t jstride;      // words per segment of `jump`
  const uint32_t* jump;  // jump data of segment 1 (segment j at jump + (j - 1) jstride)
  uint32_t* jstate;      // MT19937: jumped window of segment 1 (segment j at + (j - 1) kMtStride)
};

// Copy of one split stream's starting state, taken at the start of a run so
// that every segment reads it while the last one overwrites the original.
struct SnapRow {
  const uint32_t* src;
  uint64_t sn;
  uint64_t si;
  uint32_t* dst;
  uint64_t dn;
  uint64_t di;
  uint32_t words;
  uint32_t aos;          // 1: MT19937 layout (stream s at s * kMtStride), else structure of arrays
};

// Words of jump data per segment start: GGL a^J; XOR128 the 128x128 GF(2)
// matrix T^J as 128 rows of 4 words; RANECU a1^J, a2^J; RANMAR x^J mod the
// LFG's characteristic polynomial (97 coefficients) and J*D mod M; RANLUX
// the 576-bit multiplier b^-J' for J' SWB steps; MT19937 the exponents of
// the set coefficients of x^J mod its characteristic polynomial (a count,
// then up to 19937 16-bit exponents two per word); the 48-bit LCGs the affine
// map X -> A X + C of J steps (A and C as low, high words).
constexpr int kJumpWords[kKinds] = {0, 1, 512, 2, 98, 18, 1 + 19937 / 2 + 1, 4, 4};
// RANLUX auxiliary table: b^-d mod m for d = 0..24 (18 words each).
constexpr int kRanluxAuxWords = 25 * 18;
// RANLUX jumps by whole luxury blocks for plain generation and the in-kernel
// consumer: entry (d, v) = b^-(p v 256^d) mod m, d = 0..3, v = 0..255 (18
// words each, entry (d, 0) = 1), so that a jump of E < 2^32 blocks of p SWB
// steps is the product of the entries of E's four base-256 digits.  Built
// once per generator object (it depends on p only), so these calls need no
// jump data per segment length.
constexpr int kLuxDigits = 4;
constexpr int kLuxDigitWords = kLuxDigits * 256 * 18;
// XOR128 jumps for split plain generation: the transition matrix T raised
// to 2^k, k = 0..31 (512 words each), so that a jump of E < 2^32 positions is
// one matrix-vector product per set bit of E.  Built once per object.
constexpr int kXorPow2 = 32;
constexpr int kXorPow2Words = kXorPow2 * 512;

// Work item of the stream-table kernels: up to 64 segments of one (kind, p,
// dtype) group, one per lane.  A group numbers the segments of its cut rows
// other than their last ones row by row ("full" segments: segment g belongs
// to the row r of row0 .. row1 with first(r) <= g < first(r) + nseg(r) - 1);
// the rows' last segments (and uncut rows) form the group's tail, sorted
// longest first: a tail task's lane l takes the last segment of row
// tails[g0 + l].  An MT19937 task is segment g0 of row row0.
struct TableTask {
  uint32_t kind;
  uint32_t p;
  uint32_t dtype;
  uint32_t nseg;      // segments in this task (<= 64; MT19937: 1)
  uint64_t g0;        // first full segment, first tail entry, or the MT19937 segment
  uint32_t row0, row1;
  uint32_t tail;      // 1: a tail task
  uint32_t pad;
};

// Device scratch of prng_generate_noalloc: a file-scope array of this many
// bytes on every device; static_scratch gives its address on `device`, which
// must be the current device (looked up once per device, then cached).
constexpr size_t kStaticScratchBytes = (size_t)8 << 20;
hipError_t static_scratch(int device, void** out);

hipError_t launch_init(int kind, uint32_t* state, uint64_t n, const uint64_t* d_seeds, hipStream_t s);
hipError_t launch_generate(int kind, uint32_t p, uint32_t* state, uint64_t n, uint64_t draws, int dtype,
                           void* out, uint64_t row_elems, uint64_t elem_off, hipStream_t s);
// RANLUX plain generation with every stream cut into K >= 1 segments of S
// positions (a multiple of 24), 256 streams per block and segment.  snap: copy
// of the state taken before the launch (the state itself when K = 1); digits:
// the object's block-jump table (kLuxDigitWords words); aux: the 25
// block-completion multipliers.  Segment j > 0 starts j S / 24 - 1 blocks
// after the end of the stream's current block.
hipError_t launch_lux_plain(uint32_t p, uint32_t* st, const uint32_t* snap, uint64_t n, uint64_t draws, int dtype,
                            uint32_t S, uint32_t K, const uint32_t* digits, const uint32_t* aux, void* out,
                            uint64_t row_elems, uint64_t elem_off, hipStream_t s);
// RANLUX in-kernel consumer with every stream cut into K segments of S
// positions (a multiple of 24; 2 <= K <= kLuxSplitMax), one wavefront per
// stream.  snap, digits and aux as for launch_lux_plain.
constexpr uint32_t kLuxSplitMax = 64;
hipError_t launch_lux_fused_split(uint32_t p, uint32_t* st, const uint32_t* snap, uint64_t n, uint64_t draws,
                                  uint32_t S, uint32_t K, const uint32_t* digits, const uint32_t* aux, uint64_t* sum,
                                  uint32_t* hist, bool acc, hipStream_t s);
// XOR128 plain generation with every stream cut into K >= 2 segments of S
// positions (a multiple of 128), 256 streams per block and segment, so that
// several wavefronts per SIMD share the stores.  snap: copy of the state
// taken before the launch; pow2: the object's T^(2^k) table.  Segment j > 0
// starts j S positions ahead; the last segment writes the final state.
hipError_t launch_xor128_split(uint32_t* st, const uint32_t* snap, uint64_t n, uint64_t draws, int dtype, uint32_t S,
                               uint32_t K, const uint32_t* pow2, void* out, uint64_t row_elems, uint64_t elem_off,
                               hipStream_t s);
// Plain generation of a lane-per-stream kind with the streams interleaved four
// by four (element v of stream s at ((s / 4) row_elems + elem_off + v) * 4 + s % 4
// in 4-byte elements); dtype U32, F32 or F32P; n a multiple of 4.
hipError_t launch_generate_packed(int kind, uint32_t p, uint32_t* state, uint64_t n, uint64_t draws, int dtype,
                                  void* out, uint64_t row_elems, uint64_t elem_off, hipStream_t s);
// RANLUX plain generation with the lag table in an indexed LDS array
// (where = 1) or in HBM (where = 2): the paper's other two implementations.
hipError_t launch_ranlux_variant(int where, uint32_t p, uint32_t* state, uint64_t n, uint64_t draws, int dtype,
                                 void* out, uint64_t row_elems, uint64_t elem_off, hipStream_t s);
hipError_t launch_fused(int kind, uint32_t p, uint32_t* state, uint64_t n, uint64_t draws, uint64_t* sum,
                        uint32_t* hist, bool accumulate, hipStream_t s);
// Start of a table run: zero n_counters task counters and copy the n
// snapshot rows, in one kernel.
hipError_t launch_table_prepare(uint32_t* counters, int n_counters, const SnapRow* rows, uint32_t n,
                                uint32_t max_words, hipStream_t s);
// Lane-per-stream task classes of the stream table and the blocks (of four
// wavefronts) that fill the chip for each: GGL/XOR128/RANECU/DRAND48/RANNYU
// and RANLUX (its 96-draw chunks staged in three bytes), two per CU; RANMAR,
// one per CU.
constexpr int kLaneClasses = 2;
constexpr int kClassFullGrid[kLaneClasses] = {512, 256};
inline int lane_class(int kind) { return kind == RANMAR ? 1 : 0; }
hipError_t launch_table_lane(int cls, const TableTask* tasks, uint32_t ntasks, const TableRow* rows,
                             const uint32_t* tails, uint32_t* counter, const uint32_t* aux, int grid, hipStream_t s);
// list: n pairs (row, segment) of MT19937 segments whose windows to build
hipError_t launch_table_mt_jump(const uint32_t* list, uint32_t n, const TableRow* rows, hipStream_t s);
// one task per workgroup (four wavefronts per stream)
hipError_t launch_table_mt(const TableTask* tasks, uint32_t ntasks, const TableRow* rows, uint32_t* counter, int grid,
                           hipStream_t s);

}  // namespace prng
