// Host runtime of libprng: the C ABI declared in include/prng.h.
//
// Owns only host metadata.  All device memory (state buffers, outputs) is
// passed in by the caller.  Every entry point catches its own failures and
// reports them as negative status codes plus a thread-local message.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <tuple>
#include <unordered_set>
#include <vector>

#include "internal.h"
#include "jump.h"
#include "prng.h"

#define PRNG_API extern "C" __attribute__((visibility("default")))

using namespace prng;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(PRNG_EHIP, "%s failed: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(call)                                  \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return hip_fail(e_, #call);  \
  } while (0)

bool valid_kind(int k) { return k >= GGL && k <= MT19937; }

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

size_t state_region_bytes(int kind, uint64_t n) {
  if (kind == MT19937) return align256(n * kMtStride * 4ull);
  return align256(n * (uint64_t)kStateWords[kind] * 4ull);
}

// ---------------------------------------------------------------- seeding
uint64_t splitmix_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
// Output j (0-based) of SplitMix64 seeded with `state`.
uint64_t splitmix_at(uint64_t state, uint64_t j) { return splitmix_mix(state + (j + 1) * kGamma); }

constexpr int kRawWords[7] = {0, 1, 2, 2, 2, 1, 1};

void map_tuple(int kind, const uint64_t* w, uint64_t* t) {
  switch (kind) {
    case GGL:
      t[0] = 1 + w[0] % 2147483646ull;
      break;
    case XOR128:
      t[0] = w[0] & 0xFFFFFFFFull;
      t[1] = w[0] >> 32;
      t[2] = w[1] & 0xFFFFFFFFull;
      t[3] = w[1] >> 32;
      if ((t[0] | t[1] | t[2] | t[3]) == 0) t[3] = 1;
      break;
    case RANECU:
      t[0] = 1 + w[0] % 2147483562ull;
      t[1] = 1 + w[1] % 2147483398ull;
      break;
    case RANMAR:
      t[0] = w[0] % 31329ull;
      t[1] = w[1] % 30082ull;
      break;
    case RANLUX:
      t[0] = 1 + w[0] % 2147483562ull;
      break;
    case MT19937:
      t[0] = w[0] & 0xFFFFFFFFull;
      break;
  }
}

struct TupleHash {
  size_t operator()(const std::vector<uint64_t>& v) const {
    uint64_t h = 0;
    for (uint64_t x : v) h = splitmix_mix(h ^ x);
    return (size_t)h;
  }
};

bool seed_in_range(int kind, const uint64_t* t) {
  switch (kind) {
    case GGL:
      return t[0] >= 1 && t[0] <= 2147483646ull;
    case XOR128:
      for (int i = 0; i < 4; ++i)
        if (t[i] > 0xFFFFFFFFull) return false;
      return (t[0] | t[1] | t[2] | t[3]) != 0;
    case RANECU:
      return t[0] >= 1 && t[0] <= 2147483562ull && t[1] >= 1 && t[1] <= 2147483398ull;
    case RANMAR:
      return t[0] <= 31328 && t[1] <= 30081;
    case RANLUX:
      return t[0] >= 1 && t[0] <= 2147483562ull;
    case MT19937:
      return t[0] <= 0xFFFFFFFFull;
  }
  return false;
}

// Canonical-state validity (used by set_state).
bool state_valid(int kind, const uint32_t* w) {
  switch (kind) {
    case GGL:
      return w[0] >= 1 && w[0] <= 2147483646u;
    case XOR128:
      return (w[0] | w[1] | w[2] | w[3]) != 0;
    case RANECU:
      return w[0] >= 1 && w[0] <= 2147483562u && w[1] >= 1 && w[1] <= 2147483398u;
    case RANMAR:
      for (int i = 0; i < 97; ++i)
        if (w[i] >= (1u << 24)) return false;
      return w[97] < 16777213u;
    case RANLUX:
      for (int i = 0; i < 24; ++i)
        if (w[i] >= (1u << 24)) return false;
      return w[24] <= 1 && w[25] <= 24;
    case MT19937:
      return w[624] <= 624;
  }
  return false;
}

struct BlobHeader {
  uint32_t magic;  // "PRNG"
  uint32_t version;
  uint32_t kind;
  uint32_t p;
  uint64_t n;
  uint32_t words;
  uint32_t reserved;
};
static_assert(sizeof(BlobHeader) == 32, "blob header is 32 bytes");
constexpr uint32_t kMagic = 0x474E5250u;  // bytes 'P' 'R' 'N' 'G'

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

}  // namespace

struct prng_gen {
  int kind;
  uint32_t p;
  uint64_t n;
  uint32_t* d_state;
  int device;
};

PRNG_API const char* prng_last_error(void) { return g_err.c_str(); }

PRNG_API int prng_seed_tuple_words(int kind) { return valid_kind(kind) ? kSeedWords[kind] : PRNG_EINVAL; }

PRNG_API int prng_state_words(int kind) { return valid_kind(kind) ? kStateWords[kind] : PRNG_EINVAL; }

PRNG_API int prng_seed_words(int kind, uint64_t master, uint64_t n_streams, uint64_t* out) {
  if (!valid_kind(kind)) return fail(PRNG_EINVAL, "unknown generator kind %d", kind);
  if (!out && n_streams) return fail(PRNG_EINVAL, "out is NULL");
  try {
    const int R = kRawWords[kind], W = kSeedWords[kind];
    std::unordered_set<std::vector<uint64_t>, TupleHash> seen;
    seen.reserve(n_streams * 2);
    std::vector<uint64_t> tup(W);
    uint64_t raw[2];
    for (uint64_t s = 0; s < n_streams; ++s) {
      const uint64_t key = splitmix_at(master, s);
      for (uint64_t t = 0;; ++t) {
        for (int j = 0; j < R; ++j) raw[j] = splitmix_at(key, t * R + j);
        map_tuple(kind, raw, tup.data());
        if (seen.insert(tup).second) break;
      }
      memcpy(out + s * W, tup.data(), W * sizeof(uint64_t));
    }
  } catch (const std::bad_alloc&) {
    return fail(PRNG_ENOMEM, "out of host memory");
  }
  return PRNG_OK;
}

PRNG_API size_t prng_state_bytes(int kind, uint64_t n_streams) {
  if (!valid_kind(kind)) return 0;
  return state_region_bytes(kind, n_streams) + align256(n_streams * kSeedWords[kind] * 8ull);
}

PRNG_API int prng_create(prng_gen** g, int kind, uint32_t p, uint64_t n_streams, const uint64_t* h_seed_words,
                         void* d_state, size_t d_state_bytes, void* stream) {
  if (!g) return fail(PRNG_EINVAL, "g is NULL");
  *g = nullptr;
  if (!valid_kind(kind)) return fail(PRNG_EINVAL, "unknown generator kind %d", kind);
  if (n_streams == 0) return fail(PRNG_EINVAL, "n_streams must be > 0");
  if (n_streams > (1ull << 40)) return fail(PRNG_EINVAL, "n_streams too large");
  if (!h_seed_words) return fail(PRNG_EINVAL, "h_seed_words is NULL");
  if (kind == RANLUX) {
    if (p < 24) return fail(PRNG_EINVAL, "RANLUX p must be >= 24 (got %u)", p);
  } else {
    p = 0;
  }
  const int W = kSeedWords[kind];
  for (uint64_t s = 0; s < n_streams; ++s)
    if (!seed_in_range(kind, h_seed_words + s * W))
      return fail(PRNG_ERANGE, "seed tuple of stream %llu is outside the valid range", (unsigned long long)s);
  if (!d_state) return fail(PRNG_EINVAL, "d_state is NULL");
  if (reinterpret_cast<uintptr_t>(d_state) & 255) return fail(PRNG_EINVAL, "d_state must be 256-byte aligned");
  const size_t need = prng_state_bytes(kind, n_streams);
  if (d_state_bytes < need)
    return fail(PRNG_EINVAL, "d_state holds %zu bytes, %zu needed", d_state_bytes, need);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  hipStream_t s = static_cast<hipStream_t>(stream);
  uint32_t* st = static_cast<uint32_t*>(d_state);
  uint64_t* seeds = reinterpret_cast<uint64_t*>(static_cast<char*>(d_state) + state_region_bytes(kind, n_streams));
  HIP_TRY(hipMemcpyAsync(seeds, h_seed_words, n_streams * W * sizeof(uint64_t), hipMemcpyHostToDevice, s));
  HIP_TRY(launch_init(kind, st, n_streams, seeds, s));
  HIP_TRY(hipStreamSynchronize(s));
  prng_gen* obj = new (std::nothrow) prng_gen{kind, p, n_streams, st, dev};
  if (!obj) return fail(PRNG_ENOMEM, "out of host memory");
  *g = obj;
  return PRNG_OK;
}

PRNG_API void prng_destroy(prng_gen* g) { delete g; }

PRNG_API int prng_kind_of(const prng_gen* g) { return g ? g->kind : 0; }
PRNG_API uint32_t prng_luxury_of(const prng_gen* g) { return g ? g->p : 0; }
PRNG_API uint64_t prng_n_streams(const prng_gen* g) { return g ? g->n : 0; }

PRNG_API int prng_generate(prng_gen* g, uint64_t count, int dtype, void* d_out, size_t out_bytes, void* stream) {
  if (!g) return fail(PRNG_EINVAL, "g is NULL");
  if (dtype < U32 || dtype > F64) return fail(PRNG_EINVAL, "unknown dtype %d", dtype);
  if (count == 0) return PRNG_OK;
  if (!d_out) return fail(PRNG_EINVAL, "d_out is NULL");
  const size_t es = elem_bytes(dtype);
  if (count > (1ull << 40)) return fail(PRNG_EINVAL, "count too large");
  if (out_bytes / es / g->n < count)
    return fail(PRNG_EINVAL, "d_out holds %zu bytes, %llu needed", out_bytes,
                (unsigned long long)(g->n * count * es));
  DeviceGuard dg(g->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint64_t per = dtype == F64 ? 2 : 1;
  const uint64_t max_elems = kMaxDrawsPerLaunch / per;
  for (uint64_t off = 0; off < count; off += max_elems) {
    const uint64_t c = count - off < max_elems ? count - off : max_elems;
    HIP_TRY(launch_generate(g->kind, g->p, g->d_state, g->n, c * per, dtype, d_out, count, off, s));
  }
  return PRNG_OK;
}

PRNG_API int prng_fused_sum_hist(prng_gen* g, uint64_t draws, uint64_t* d_sum, uint32_t* d_hist, void* stream) {
  if (!g) return fail(PRNG_EINVAL, "g is NULL");
  if (!d_sum || !d_hist) return fail(PRNG_EINVAL, "d_sum / d_hist is NULL");
  if (draws > (1ull << 40)) return fail(PRNG_EINVAL, "draws too large");
  DeviceGuard dg(g->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  // draws == 0 still launches once: the kernel then writes zero sums and
  // histograms without advancing any stream.
  for (uint64_t off = 0; off == 0 || off < draws; off += kMaxDrawsPerLaunch) {
    const uint64_t d = draws - off < kMaxDrawsPerLaunch ? draws - off : kMaxDrawsPerLaunch;
    HIP_TRY(launch_fused(g->kind, g->p, g->d_state, g->n, d, d_sum, d_hist, off > 0, s));
  }
  return PRNG_OK;
}

PRNG_API size_t prng_blob_bytes(const prng_gen* g) {
  if (!g) return 0;
  return sizeof(BlobHeader) + g->n * (uint64_t)kStateWords[g->kind] * 4ull;
}

PRNG_API int prng_get_state(const prng_gen* g, void* h_blob, size_t bytes, void* stream) {
  if (!g) return fail(PRNG_EINVAL, "g is NULL");
  if (!h_blob) return fail(PRNG_EINVAL, "h_blob is NULL");
  if (bytes < prng_blob_bytes(g)) return fail(PRNG_EINVAL, "blob buffer too small");
  DeviceGuard dg(g->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int W = kStateWords[g->kind];
  const uint64_t n = g->n;
  std::vector<uint32_t> dev;
  try {
    dev.resize(state_region_bytes(g->kind, n) / 4);
  } catch (const std::bad_alloc&) {
    return fail(PRNG_ENOMEM, "out of host memory");
  }
  HIP_TRY(hipMemcpyAsync(dev.data(), g->d_state, dev.size() * 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  BlobHeader h{kMagic, 1u, (uint32_t)g->kind, g->p, n, (uint32_t)W, 0u};
  memcpy(h_blob, &h, sizeof h);
  uint32_t* w = reinterpret_cast<uint32_t*>(static_cast<char*>(h_blob) + sizeof h);
  if (g->kind == MT19937) {
    for (uint64_t i = 0; i < n; ++i) memcpy(w + i * W, dev.data() + i * kMtStride, W * 4);
  } else {
    for (uint64_t i = 0; i < n; ++i)
      for (int j = 0; j < W; ++j) w[i * W + j] = dev[j * n + i];
  }
  return PRNG_OK;
}

PRNG_API int prng_set_state(prng_gen* g, const void* h_blob, size_t bytes, void* stream) {
  if (!g) return fail(PRNG_EINVAL, "g is NULL");
  if (!h_blob) return fail(PRNG_EINVAL, "h_blob is NULL");
  BlobHeader h;
  if (bytes < sizeof h) return fail(PRNG_ESTATE, "blob shorter than its header");
  memcpy(&h, h_blob, sizeof h);
  const int W = kStateWords[g->kind];
  if (h.magic != kMagic) return fail(PRNG_ESTATE, "bad blob magic");
  if (h.version != 1) return fail(PRNG_ESTATE, "unsupported blob version %u", h.version);
  if ((int)h.kind != g->kind) return fail(PRNG_ESTATE, "blob kind %u does not match %d", h.kind, g->kind);
  if (h.p != g->p) return fail(PRNG_ESTATE, "blob luxury %u does not match %u", h.p, g->p);
  if (h.n != g->n) return fail(PRNG_ESTATE, "blob has %llu streams, object %llu", (unsigned long long)h.n,
                              (unsigned long long)g->n);
  if ((int)h.words != W) return fail(PRNG_ESTATE, "blob words per stream %u, expected %d", h.words, W);
  if (bytes < prng_blob_bytes(g)) return fail(PRNG_ESTATE, "blob truncated");
  const uint32_t* w = reinterpret_cast<const uint32_t*>(static_cast<const char*>(h_blob) + sizeof h);
  const uint64_t n = g->n;
  for (uint64_t i = 0; i < n; ++i)
    if (!state_valid(g->kind, w + i * W))
      return fail(PRNG_ESTATE, "stream %llu holds an invalid state", (unsigned long long)i);
  std::vector<uint32_t> dev;
  try {
    dev.assign(state_region_bytes(g->kind, n) / 4, 0u);
  } catch (const std::bad_alloc&) {
    return fail(PRNG_ENOMEM, "out of host memory");
  }
  if (g->kind == MT19937) {
    for (uint64_t i = 0; i < n; ++i) memcpy(dev.data() + i * kMtStride, w + i * W, W * 4);
  } else {
    for (uint64_t i = 0; i < n; ++i)
      for (int j = 0; j < W; ++j) dev[j * n + i] = w[i * W + j];
  }
  DeviceGuard dg(g->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(hipMemcpyAsync(g->d_state, dev.data(), dev.size() * 4, hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  return PRNG_OK;
}

// ================================================================ stream table
// Batched generation (not in the paper, whose instances are independent and
// launched together): rows of (generator object, stream, count, dtype,
// output buffer) are planned into wave-sized tasks and run by two persistent
// kernels (lane-per-stream kinds; MT19937), optionally captured into a graph.
// Long lane-per-stream rows are cut into segments that start from jumped-ahead
// states, so that no single lane carries a whole long stream.
namespace {

struct TableConfig {
  int lane_grid;
  int mt_grid;
  int concurrent;
};

// relative cost of one draw, used only to order tasks longest first
double draw_cost(int kind, uint32_t p) {
  switch (kind) {
    case RANMAR:
      return 1.1;
    case RANLUX:
      return 1.5 + (p > 24 ? (p - 24) / 24.0 * 0.35 : 0.0);
    case MT19937:
      return 1.3;
    default:
      return 1.0;
  }
}

constexpr uint32_t kSegAlign = 384;             // multiple of 24 (luxury blocks) and of 128 (chunks)
constexpr uint32_t kSegAuto = 0, kSegNever = 0xFFFFFFFFu;
constexpr uint64_t kMaxSegments = 4096;         // per row

std::mutex g_tune_mu;
std::map<std::tuple<uint64_t, uint64_t, uint64_t, uint64_t>, TableConfig> g_tune_cache;

uint32_t jump_stride(int kind) { return (uint32_t)((kJumpWords[kind] + 3) & ~3); }  // 16-byte aligned slots

struct RowRef {
  prng_gen* g;
  uint64_t stream;
  void* out;
  uint32_t draws;
  int dtype;
};

// Everything a table needs in its workspace, with pointers into the
// workspace stored as byte offsets until the base address is known.
struct Plan {
  std::vector<TableTask> lane_tasks, mt_tasks;
  std::vector<TableRow> rows;      // state/jump fields of split rows hold offsets (flags below)
  std::vector<uint8_t> row_snap;   // 1: `state` is an offset into the snapshot area
  std::vector<int64_t> row_jump;   // >= 0: word offset of the segment's jump data
  std::vector<SnapRow> snaps;      // dst holds nothing until patched
  std::vector<uint32_t> jump;      // all jump data
  std::vector<uint32_t> aux;       // RANLUX b^-d table (d = 0..24)
  std::vector<prng_gen*> gens;
  uint64_t total_draws = 0, max_draws = 0, max_task_draws = 0;
  size_t o_lane = 0, o_mt = 0, o_rows = 0, o_snaprows = 0, o_snap = 0, o_jump = 0, o_aux = 0, total = 0;
};

int make_plan(prng_gen* const* gens, int n_gens, const prng_table_row* rows, uint64_t n_rows, uint32_t seg_len,
              Plan& P) {
  if (!gens || n_gens <= 0) return fail(PRNG_EINVAL, "no generator objects");
  if (!rows && n_rows) return fail(PRNG_EINVAL, "rows is NULL");
  for (int i = 0; i < n_gens; ++i)
    if (!gens[i]) return fail(PRNG_EINVAL, "generator %d is NULL", i);
  std::vector<RowRef> all;
  all.reserve(n_rows);
  std::set<std::pair<const uint32_t*, uint64_t>> seen;
  uint64_t lane_draws = 0;
  for (uint64_t i = 0; i < n_rows; ++i) {
    const prng_table_row& r = rows[i];
    if (r.gen >= (uint32_t)n_gens) return fail(PRNG_EINVAL, "row %llu: generator index out of range", (unsigned long long)i);
    prng_gen* g = gens[r.gen];
    if (r.dtype < U32 || r.dtype > F64) return fail(PRNG_EINVAL, "row %llu: unknown dtype", (unsigned long long)i);
    if (r.stream >= g->n) return fail(PRNG_EINVAL, "row %llu: stream out of range", (unsigned long long)i);
    if (r.count == 0) continue;
    const uint64_t per = r.dtype == F64 ? 2 : 1;
    if (r.count > kMaxDrawsPerLaunch / per)
      return fail(PRNG_EINVAL, "row %llu: count too large for one run", (unsigned long long)i);
    if (!r.d_out || (reinterpret_cast<uintptr_t>(r.d_out) % elem_bytes(r.dtype)))
      return fail(PRNG_EINVAL, "row %llu: output pointer NULL or misaligned", (unsigned long long)i);
    if (!seen.insert({g->d_state, r.stream}).second)
      return fail(PRNG_EINVAL, "row %llu: stream listed twice", (unsigned long long)i);
    const uint32_t d = (uint32_t)(r.count * per);
    all.push_back(RowRef{g, r.stream, r.d_out, d, (int)r.dtype});
    if (std::find(P.gens.begin(), P.gens.end(), g) == P.gens.end()) P.gens.push_back(g);
    P.total_draws += d;
    P.max_draws = std::max<uint64_t>(P.max_draws, d);
    if (g->kind != MT19937) lane_draws += d;
  }
  // ---- segment length per kind
  auto roundup = [](uint64_t v, uint64_t a) { return (v + a - 1) / a * a; };
  uint64_t base = 0;
  if (seg_len == kSegAuto)
    base = roundup(std::max<uint64_t>(lane_draws / 131072, 3072), kSegAlign);
  else if (seg_len != kSegNever)
    base = roundup(std::max<uint64_t>(seg_len, kSegAlign), kSegAlign);
  auto seg_for = [&](int kind) -> uint64_t {
    if (base == 0 || kind == MT19937) return 0;
    if (kind == RANMAR && seg_len == kSegAuto) return std::max<uint64_t>(base, 32768);  // its jump costs ~20k ops
    return base;
  };
  // ---- segments: (row, j) pairs; rows longer than one segment are split
  struct Seg {
    uint64_t row;
    uint32_t j, K;
    uint32_t len;  // approximate draws of this segment (for ordering)
  };
  std::vector<Seg> segs;
  std::vector<int64_t> snap_of(all.size(), -1);
  std::map<std::tuple<int, uint32_t, uint64_t>, uint64_t> jump_base;  // (kind, p, L) -> word offset of j = 1
  std::map<std::tuple<int, uint32_t, uint64_t>, uint32_t> jump_count;
  std::vector<uint64_t> seg_len_of(all.size(), 0);
  for (uint64_t i = 0; i < all.size(); ++i) {
    const int k = all[i].g->kind;
    uint64_t L = seg_for(k);
    const uint64_t D = all[i].draws;
    if (L && (D + L - 1) / L > kMaxSegments) L = roundup((D + kMaxSegments - 1) / kMaxSegments, kSegAlign);
    const uint64_t K = L ? (D + L - 1) / L : 1;  // (K - 1) L < D: the last segment is never empty
    if (K > 1) {
      seg_len_of[i] = L;
      snap_of[i] = (int64_t)P.snaps.size();
      P.snaps.push_back(SnapRow{all[i].g->d_state, all[i].g->n, all[i].stream, nullptr, 0, 0,
                                (uint32_t)kStateWords[k], 0u});
      const auto key = std::make_tuple(k, all[i].g->p, L);
      jump_count[key] = std::max<uint32_t>(jump_count[key], (uint32_t)K - 1);
      for (uint32_t j = 0; j < K; ++j) {
        const uint64_t len = j + 1 < K ? L : D - (K - 1) * L;
        segs.push_back(Seg{i, j, (uint32_t)K, (uint32_t)len});
      }
    } else {
      segs.push_back(Seg{i, 0, 1, all[i].draws});
    }
  }
  // jump data for every (kind, p, L): segment j starts J_j positions ahead
  for (auto& kc : jump_count) {
    const int k = std::get<0>(kc.first);
    const uint32_t p = std::get<1>(kc.first);
    const uint64_t L = std::get<2>(kc.first);
    const uint32_t nj = kc.second, stride = jump_stride(k);
    jump_base[kc.first] = P.jump.size();
    P.jump.resize(P.jump.size() + (size_t)nj * stride, 0u);
    uint32_t* dst = P.jump.data() + jump_base[kc.first];
    switch (k) {
      case GGL:
        for (uint32_t j = 1; j <= nj; ++j) dst[(j - 1) * stride] = powmod31(16807, (uint64_t)j * L, 2147483647u);
        break;
      case RANECU:
        for (uint32_t j = 1; j <= nj; ++j) {
          dst[(j - 1) * stride] = powmod31(40014, (uint64_t)j * L, 2147483563u);
          dst[(j - 1) * stride + 1] = powmod31(40692, (uint64_t)j * L, 2147483399u);
        }
        break;
      case XOR128: {
        std::vector<uint32_t> step(512);
        xor128_power(L, step.data());
        memcpy(dst, step.data(), 512 * 4);
        for (uint32_t j = 2; j <= nj; ++j) xor128_compose(step.data(), dst + (j - 2) * stride, dst + (j - 1) * stride);
        break;
      }
      case RANMAR: {
        uint32_t step[97];
        ranmar_power(L, step);
        memcpy(dst, step, sizeof step);
        dst[97] = ranmar_c_shift(L);
        for (uint32_t j = 2; j <= nj; ++j) {
          ranmar_polymul(dst + (j - 2) * stride, step, dst + (j - 1) * stride);
          dst[(j - 1) * stride + 97] = ranmar_c_shift((uint64_t)j * L);
        }
        break;
      }
      case RANLUX: {
        // segment j starts at the block boundary j L (skip pending): from the
        // end of the stream's current block that is (j L / 24 - 1) blocks of p
        for (uint32_t j = 1; j <= nj; ++j) ranlux_power(((uint64_t)j * L / 24 - 1) * p, dst + (j - 1) * stride);
        break;
      }
    }
  }
  bool need_aux = false;
  for (auto& kc : jump_count)
    if (std::get<0>(kc.first) == RANLUX) need_aux = true;
  if (need_aux) {
    P.aux.resize(kRanluxAuxWords);
    for (int d = 0; d <= 24; ++d) ranlux_power((uint64_t)d, P.aux.data() + d * 18);
  }
  // ---- tasks: group by (kind, p, dtype), longest segments first, 64 per task
  std::vector<uint64_t> order(segs.size());
  for (uint64_t i = 0; i < order.size(); ++i) order[i] = i;
  auto kind_of = [&](uint64_t si) { return all[segs[si].row].g->kind; };
  auto lux_of = [&](uint64_t si) { return all[segs[si].row].g->p; };
  auto dt_of = [&](uint64_t si) { return all[segs[si].row].dtype; };
  std::sort(order.begin(), order.end(), [&](uint64_t a, uint64_t b) {
    if (kind_of(a) != kind_of(b)) return kind_of(a) < kind_of(b);
    if (lux_of(a) != lux_of(b)) return lux_of(a) < lux_of(b);
    if (dt_of(a) != dt_of(b)) return dt_of(a) < dt_of(b);
    if (segs[a].len != segs[b].len) return segs[a].len > segs[b].len;
    return a < b;
  });
  struct TP {
    double cost;
    TableTask task;
    uint32_t len;
  };
  std::vector<TP> lane_plan, mt_plan;
  uint64_t i = 0;
  while (i < order.size()) {
    const uint64_t a = order[i];
    const int k = kind_of(a);
    uint64_t j = i;
    const uint64_t lim = k == MT19937 ? 1 : 64;
    while (j < order.size() && j - i < lim && kind_of(order[j]) == k && lux_of(order[j]) == lux_of(a) &&
           dt_of(order[j]) == dt_of(a))
      ++j;
    TableTask task{(uint32_t)k, lux_of(a), (uint32_t)dt_of(a), (uint32_t)(j - i), (uint64_t)P.rows.size()};
    for (uint64_t q = i; q < j; ++q) {
      const Seg& sg = segs[order[q]];
      const RowRef& rr = all[sg.row];
      TableRow tr{};
      const bool split = sg.K > 1;
      const uint64_t Lr = seg_len_of[sg.row];
      if (split) {
        tr.state = nullptr;  // patched: snapshot area
        tr.sn = P.snaps.size();
        tr.si = (uint64_t)snap_of[sg.row];
      } else {
        tr.state = rr.g->d_state;
        tr.sn = rr.g->n;
        tr.si = rr.stream;
      }
      tr.wstate = rr.g->d_state;
      tr.wsn = rr.g->n;
      tr.wsi = rr.stream;
      tr.out = rr.out;
      tr.draws = rr.draws;
      tr.seg = sg.j;
      tr.seg_len = (uint32_t)Lr;
      tr.last = sg.j + 1 == sg.K ? 1u : 0u;
      tr.jump = nullptr;
      P.rows.push_back(tr);
      P.row_snap.push_back(split ? 1 : 0);
      int64_t jo = -1;
      if (split && sg.j > 0)
        jo = (int64_t)(jump_base[std::make_tuple(k, rr.g->p, Lr)] + (uint64_t)(sg.j - 1) * jump_stride(k));
      P.row_jump.push_back(jo);
    }
    const uint32_t len = segs[order[i]].len;
    const double cost = len * draw_cost(k, lux_of(a)) + (segs[order[i]].j ? 3000.0 : 0.0);
    (k == MT19937 ? mt_plan : lane_plan).push_back(TP{cost, task, len});
    P.max_task_draws = std::max<uint64_t>(P.max_task_draws, len);
    i = j;
  }
  auto by_cost = [](const TP& x, const TP& y) { return x.cost > y.cost; };
  std::stable_sort(lane_plan.begin(), lane_plan.end(), by_cost);
  std::stable_sort(mt_plan.begin(), mt_plan.end(), by_cost);
  for (auto& t : lane_plan) P.lane_tasks.push_back(t.task);
  for (auto& t : mt_plan) P.mt_tasks.push_back(t.task);
  // ---- workspace layout
  size_t off = 256;  // two task counters
  P.o_lane = off;
  off += align256(P.lane_tasks.size() * sizeof(TableTask));
  P.o_mt = off;
  off += align256(P.mt_tasks.size() * sizeof(TableTask));
  P.o_rows = off;
  off += align256(P.rows.size() * sizeof(TableRow));
  P.o_snaprows = off;
  off += align256(P.snaps.size() * sizeof(SnapRow));
  P.o_snap = off;
  off += align256(P.snaps.size() * 98ull * 4ull);
  P.o_jump = off;
  off += align256(P.jump.size() * 4ull);
  P.o_aux = off;
  off += align256(P.aux.size() * 4ull);
  P.total = off;
  return PRNG_OK;
}

}  // namespace

struct prng_table {
  std::vector<prng_gen*> gens;  // objects whose states the table advances
  uint32_t n_lane_tasks = 0, n_mt_tasks = 0, n_snaps = 0;
  uint64_t total_draws = 0, max_draws = 0, max_task_draws = 0, n_segments = 0;
  uint32_t* d_counters = nullptr;
  TableTask* d_lane_tasks = nullptr;
  TableTask* d_mt_tasks = nullptr;
  TableRow* d_rows = nullptr;
  SnapRow* d_snaps = nullptr;
  const uint32_t* d_aux = nullptr;
  TableConfig cfg{256, 512, 1};
  int device = 0;
  hipStream_t cap = nullptr, side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

void drop_graph(prng_table* t) {
  if (t->exec) (void)hipGraphExecDestroy(t->exec);
  if (t->graph) (void)hipGraphDestroy(t->graph);
  t->exec = nullptr;
  t->graph = nullptr;
}

// Enqueue one run: reset counters, copy the starting states of split streams,
// then the two persistent kernels (the MT one forked onto the side stream
// when `concurrent`).
hipError_t enqueue_run(prng_table* t, hipStream_t s) {
  hipError_t e = launch_table_reset(t->d_counters, 2, s);
  if (e != hipSuccess) return e;
  if ((e = launch_table_snapshot(t->d_snaps, t->n_snaps, s)) != hipSuccess) return e;
  const bool fork = t->cfg.concurrent && t->n_lane_tasks && t->n_mt_tasks;
  if (fork) {
    if ((e = hipEventRecord(t->fork, s)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(t->side, t->fork, 0)) != hipSuccess) return e;
  }
  if (t->n_lane_tasks) {
    const int g = std::min<int>(t->cfg.lane_grid, (int)((t->n_lane_tasks + 3) / 4));
    if ((e = launch_table_lane(t->d_lane_tasks, t->n_lane_tasks, t->d_rows, t->d_counters, t->d_aux, g, s)) !=
        hipSuccess)
      return e;
  }
  if (t->n_mt_tasks) {
    const int g = std::min<int>(t->cfg.mt_grid, (int)((t->n_mt_tasks + 3) / 4));
    if ((e = launch_table_mt(t->d_mt_tasks, t->n_mt_tasks, t->d_rows, t->d_counters + 1, g, fork ? t->side : s)) !=
        hipSuccess)
      return e;
  }
  if (fork) {
    if ((e = hipEventRecord(t->join, t->side)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(s, t->join, 0)) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

PRNG_API size_t prng_table_work_bytes(prng_gen* const* gens, int n_gens, const prng_table_row* rows, uint64_t n_rows,
                                      uint32_t seg_len) {
  try {
    Plan P;
    if (make_plan(gens, n_gens, rows, n_rows, seg_len, P) != PRNG_OK) return 0;
    return P.total;
  } catch (const std::bad_alloc&) {
    fail(PRNG_ENOMEM, "out of host memory");
    return 0;
  }
}

PRNG_API int prng_table_create(prng_table** out, prng_gen* const* gens, int n_gens, const prng_table_row* rows,
                               uint64_t n_rows, uint32_t seg_len, void* d_work, size_t work_bytes, void* stream) {
  if (!out) return fail(PRNG_EINVAL, "t is NULL");
  *out = nullptr;
  try {
    Plan P;
    const int rc = make_plan(gens, n_gens, rows, n_rows, seg_len, P);
    if (rc != PRNG_OK) return rc;
    if (!d_work || work_bytes < P.total)
      return fail(PRNG_EINVAL, "workspace holds %zu bytes, %zu needed", work_bytes, P.total);
    if (reinterpret_cast<uintptr_t>(d_work) & 255) return fail(PRNG_EINVAL, "workspace must be 256-byte aligned");
    std::unique_ptr<prng_table> t(new prng_table());
    char* w = static_cast<char*>(d_work);
    uint32_t* snap = reinterpret_cast<uint32_t*>(w + P.o_snap);
    const uint32_t* jump = reinterpret_cast<const uint32_t*>(w + P.o_jump);
    const uint64_t ns = P.snaps.size();
    for (uint64_t i = 0; i < ns; ++i) {
      P.snaps[i].dst = snap;
      P.snaps[i].dn = ns;
      P.snaps[i].di = i;
    }
    for (uint64_t i = 0; i < P.rows.size(); ++i) {
      if (P.row_snap[i]) P.rows[i].state = snap;  // sn = ns, si = snapshot index (set by the plan)
      if (P.row_jump[i] >= 0) P.rows[i].jump = jump + P.row_jump[i];
    }
    t->gens = P.gens;
    t->n_lane_tasks = (uint32_t)P.lane_tasks.size();
    t->n_mt_tasks = (uint32_t)P.mt_tasks.size();
    t->n_snaps = (uint32_t)ns;
    t->total_draws = P.total_draws;
    t->max_draws = P.max_draws;
    t->max_task_draws = P.max_task_draws;
    t->n_segments = P.rows.size();
    t->d_counters = reinterpret_cast<uint32_t*>(w);
    t->d_lane_tasks = reinterpret_cast<TableTask*>(w + P.o_lane);
    t->d_mt_tasks = reinterpret_cast<TableTask*>(w + P.o_mt);
    t->d_rows = reinterpret_cast<TableRow*>(w + P.o_rows);
    t->d_snaps = reinterpret_cast<SnapRow*>(w + P.o_snaprows);
    t->d_aux = P.aux.empty() ? nullptr : reinterpret_cast<const uint32_t*>(w + P.o_aux);
    HIP_TRY(hipGetDevice(&t->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto up = [&](size_t off, const void* src, size_t bytes) -> hipError_t {
      return bytes ? hipMemcpyAsync(w + off, src, bytes, hipMemcpyHostToDevice, s) : hipSuccess;
    };
    HIP_TRY(up(P.o_lane, P.lane_tasks.data(), P.lane_tasks.size() * sizeof(TableTask)));
    HIP_TRY(up(P.o_mt, P.mt_tasks.data(), P.mt_tasks.size() * sizeof(TableTask)));
    HIP_TRY(up(P.o_rows, P.rows.data(), P.rows.size() * sizeof(TableRow)));
    HIP_TRY(up(P.o_snaprows, P.snaps.data(), P.snaps.size() * sizeof(SnapRow)));
    HIP_TRY(up(P.o_jump, P.jump.data(), P.jump.size() * 4));
    HIP_TRY(up(P.o_aux, P.aux.data(), P.aux.size() * 4));
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipStreamCreateWithFlags(&t->cap, hipStreamNonBlocking));
    HIP_TRY(hipStreamCreateWithFlags(&t->side, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&t->fork, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&t->join, hipEventDisableTiming));
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tune_cache.find({t->n_lane_tasks, t->n_mt_tasks, t->total_draws, t->max_task_draws});
      if (it != g_tune_cache.end()) t->cfg = it->second;
    }
    *out = t.release();
  } catch (const std::bad_alloc&) {
    return fail(PRNG_ENOMEM, "out of host memory");
  }
  return PRNG_OK;
}

PRNG_API void prng_table_destroy(prng_table* t) {
  if (!t) return;
  drop_graph(t);
  if (t->fork) (void)hipEventDestroy(t->fork);
  if (t->join) (void)hipEventDestroy(t->join);
  if (t->cap) (void)hipStreamDestroy(t->cap);
  if (t->side) (void)hipStreamDestroy(t->side);
  delete t;
}

PRNG_API int prng_table_get_config(const prng_table* t, int* lane_grid, int* mt_grid, int* concurrent) {
  if (!t) return fail(PRNG_EINVAL, "t is NULL");
  if (lane_grid) *lane_grid = t->cfg.lane_grid;
  if (mt_grid) *mt_grid = t->cfg.mt_grid;
  if (concurrent) *concurrent = t->cfg.concurrent;
  return PRNG_OK;
}

PRNG_API int prng_table_set_config(prng_table* t, int lane_grid, int mt_grid, int concurrent) {
  if (!t) return fail(PRNG_EINVAL, "t is NULL");
  if (lane_grid < 1 || lane_grid > 65536 || mt_grid < 1 || mt_grid > 65536)
    return fail(PRNG_EINVAL, "grid sizes must be in [1, 65536]");
  t->cfg = TableConfig{lane_grid, mt_grid, concurrent ? 1 : 0};
  drop_graph(t);
  return PRNG_OK;
}

PRNG_API int prng_table_run(prng_table* t, int use_graph, void* stream) {
  if (!t) return fail(PRNG_EINVAL, "t is NULL");
  DeviceGuard dg(t->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!use_graph) {
    HIP_TRY(enqueue_run(t, s));
    return PRNG_OK;
  }
  if (!t->exec) {
    HIP_TRY(hipStreamBeginCapture(t->cap, hipStreamCaptureModeThreadLocal));
    hipError_t e = enqueue_run(t, t->cap);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(t->cap, &g);
    if (e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return hip_fail(e, "enqueue_run (capture)");
    }
    if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
    t->graph = g;
    HIP_TRY(hipGraphInstantiate(&t->exec, t->graph, nullptr, nullptr, 0));
  }
  HIP_TRY(hipGraphLaunch(t->exec, s));
  return PRNG_OK;
}

// Autotuner: times candidate (lane grid, MT grid, concurrency) settings on
// the real rows, restoring every referenced stream state after each trial so
// that tuning leaves the streams where they were (the output buffers are
// overwritten by the trials).  The best setting is cached per table shape.
PRNG_API int prng_table_autotune(prng_table* t, int repeats, void* stream) {
  if (!t) return fail(PRNG_EINVAL, "t is NULL");
  if (repeats < 1) repeats = 1;
  DeviceGuard dg(t->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<std::vector<char>> saved(t->gens.size());
  try {
    for (size_t i = 0; i < t->gens.size(); ++i) saved[i].resize(state_region_bytes(t->gens[i]->kind, t->gens[i]->n));
  } catch (const std::bad_alloc&) {
    return fail(PRNG_ENOMEM, "out of host memory");
  }
  HIP_TRY(hipStreamSynchronize(s));
  for (size_t i = 0; i < t->gens.size(); ++i)
    HIP_TRY(hipMemcpy(saved[i].data(), t->gens[i]->d_state, saved[i].size(), hipMemcpyDeviceToHost));
  auto restore = [&]() -> hipError_t {
    for (size_t i = 0; i < t->gens.size(); ++i) {
      hipError_t e = hipMemcpy(t->gens[i]->d_state, saved[i].data(), saved[i].size(), hipMemcpyHostToDevice);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  hipEvent_t a, b;
  HIP_TRY(hipEventCreate(&a));
  HIP_TRY(hipEventCreate(&b));
  const TableConfig keep = t->cfg;
  TableConfig best = keep;
  float best_ms = 1e30f;
  const int lane_opts[] = {64, 128, 256};
  const int mt_opts[] = {128, 256, 512, 1024, 2048};
  hipError_t err = hipSuccess;
  for (int conc = 0; conc < 2 && err == hipSuccess; ++conc)
    for (int lg : lane_opts)
      for (int mg : mt_opts) {
        if (err != hipSuccess) break;
        if (!t->n_lane_tasks && lg != lane_opts[0]) continue;
        if (!t->n_mt_tasks && mg != mt_opts[0]) continue;
        t->cfg = TableConfig{lg, mg, conc};
        float total = 0;
        for (int r = 0; r < repeats && err == hipSuccess; ++r) {
          if ((err = hipEventRecord(a, s)) != hipSuccess) break;
          if ((err = enqueue_run(t, s)) != hipSuccess) break;
          if ((err = hipEventRecord(b, s)) != hipSuccess) break;
          if ((err = hipEventSynchronize(b)) != hipSuccess) break;
          float ms = 0;
          if ((err = hipEventElapsedTime(&ms, a, b)) != hipSuccess) break;
          total += ms;
          if ((err = restore()) != hipSuccess) break;
        }
        if (err == hipSuccess && total / repeats < best_ms) {
          best_ms = total / repeats;
          best = t->cfg;
        }
      }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (err != hipSuccess) {
    t->cfg = keep;
    (void)restore();
    return hip_fail(err, "autotune trial");
  }
  t->cfg = best;
  drop_graph(t);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache[{t->n_lane_tasks, t->n_mt_tasks, t->total_draws, t->max_task_draws}] = best;
  return PRNG_OK;
}

PRNG_API int prng_table_info(const prng_table* t, uint32_t* n_lane_tasks, uint32_t* n_mt_tasks, uint64_t* total_draws,
                             uint64_t* max_draws, uint64_t* n_segments) {
  if (!t) return fail(PRNG_EINVAL, "t is NULL");
  if (n_lane_tasks) *n_lane_tasks = t->n_lane_tasks;
  if (n_mt_tasks) *n_mt_tasks = t->n_mt_tasks;
  if (total_draws) *total_draws = t->total_draws;
  if (max_draws) *max_draws = t->max_draws;
  if (n_segments) *n_segments = t->n_segments;
  return PRNG_OK;
}
