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

#include "host.h"
#include "jump.h"

using namespace prng;

namespace prng {

namespace {
thread_local std::string g_err;
}

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

const char* last_error() { return g_err.c_str(); }

int hip_fail(hipError_t e, const char* what) {
  return fail(PRNG_EHIP, "%s failed: %s", what, hipGetErrorString(e));
}

namespace {

// ---------------------------------------------------------------- seeding
uint64_t splitmix_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
// Output j (0-based) of SplitMix64 seeded with `state`.
uint64_t splitmix_at(uint64_t state, uint64_t j) { return splitmix_mix(state + (j + 1) * kGamma); }

constexpr int kRawWords[kKinds] = {0, 1, 2, 2, 2, 1, 1, 1, 1};

constexpr uint64_t kMask48 = (1ull << 48) - 1;

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
    case DRAND48:
      t[0] = w[0] & kMask48;
      break;
    case RANNYU:  // odd seeds only
      t[0] = (w[0] & kMask48) | 1u;
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
    case DRAND48:
      return t[0] <= kMask48;
    case RANNYU:
      return t[0] <= kMask48 && (t[0] & 1u);
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
    case DRAND48:
      return w[1] <= 0xFFFFu;
    case RANNYU:
      return w[1] <= 0xFFFFu && (w[0] & 1u);
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

}  // namespace
}  // namespace prng

PRNG_API const char* prng_last_error(void) { return prng::last_error(); }

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

// Behind the state region: the seed tuples read by the initialisation kernel
// and, for the kinds whose plain generation cuts streams into jumped segments
// (RANLUX, XOR128), the snapshot the segments jump from (the seed area is free
// again once the object exists); then the object's jump tables, written once
// by prng_create: for RANLUX the 25 block-completion multipliers and the
// block-jump table of its luxury, for XOR128 the powers T^(2^k).
namespace {
bool splits(int kind) { return kind == RANLUX || kind == XOR128; }
size_t scratch_bytes(int kind, uint64_t n) {
  size_t b = n * kSeedWords[kind] * 8ull;
  if (splits(kind)) b = std::max<size_t>(b, state_region_bytes(kind, n));
  return align256(b);
}
size_t table_bytes(int kind) {
  if (kind == RANLUX) return align256((size_t)(kRanluxAuxWords + kLuxDigitWords) * 4);
  if (kind == XOR128) return align256((size_t)kXorPow2Words * 4);
  return 0;
}
uint32_t* snapshot_area(const prng_gen* g) {
  return reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(g->d_state) + state_region_bytes(g->kind, g->n));
}
const uint32_t* object_tables(const prng_gen* g) {
  return reinterpret_cast<const uint32_t*>(reinterpret_cast<char*>(g->d_state) + state_region_bytes(g->kind, g->n) +
                                           scratch_bytes(g->kind, g->n));
}
const uint32_t* lux_aux(const prng_gen* g) { return object_tables(g); }
const uint32_t* lux_digits(const prng_gen* g) { return object_tables(g) + kRanluxAuxWords; }
}  // namespace

PRNG_API size_t prng_state_bytes(int kind, uint64_t n_streams) {
  if (!valid_kind(kind)) return 0;
  return state_region_bytes(kind, n_streams) + scratch_bytes(kind, n_streams) + table_bytes(kind);
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
  std::vector<uint32_t> tables;
  if (table_bytes(kind)) {
    try {
      tables.resize(table_bytes(kind) / 4);
    } catch (const std::bad_alloc&) {
      return fail(PRNG_ENOMEM, "out of host memory");
    }
    if (kind == RANLUX) {
      fill_ranlux_aux(tables.data());
      fill_ranlux_digits(p, tables.data() + kRanluxAuxWords);
    } else {
      fill_xor128_pow2(tables.data());
    }
    char* at = static_cast<char*>(d_state) + state_region_bytes(kind, n_streams) + scratch_bytes(kind, n_streams);
    HIP_TRY(hipMemcpyAsync(at, tables.data(), tables.size() * 4, hipMemcpyHostToDevice, s));
  }
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

namespace {
// prng_generate with the pre-launch snapshot of RANLUX and XOR128 (the kinds
// whose streams are cut into jumped segments) at `snap_area` (the object's
// scratch area, or the device's static scratch for prng_generate_noalloc).
int generate_with(prng_gen* g, uint64_t count, int dtype, void* d_out, size_t out_bytes, void* stream,
                  uint32_t* snap_area);
}  // namespace

PRNG_API int prng_generate(prng_gen* g, uint64_t count, int dtype, void* d_out, size_t out_bytes, void* stream) {
  if (!g) return fail(PRNG_EINVAL, "g is NULL");
  return generate_with(g, count, dtype, d_out, out_bytes, stream, splits(g->kind) ? snapshot_area(g) : nullptr);
}

PRNG_API int prng_generate_noalloc(prng_gen* g, uint64_t count, int dtype, void* d_out, size_t out_bytes,
                                   void* stream) {
  if (!g) return fail(PRNG_EINVAL, "g is NULL");
  uint32_t* snap = nullptr;
  if (splits(g->kind)) {
    const size_t need = state_region_bytes(g->kind, g->n);
    if (need > kStaticScratchBytes)
      return fail(PRNG_EINVAL, "prng_generate_noalloc: an object of kind %d with %llu streams needs %zu bytes of "
                  "scratch, the static scratch holds %zu (at most %zu streams)", g->kind, (unsigned long long)g->n,
                  need, kStaticScratchBytes, kStaticScratchBytes / (kStateWords[g->kind] * 4));
    DeviceGuard dg(g->device);
    void* p = nullptr;
    HIP_TRY(static_scratch(g->device, &p));
    snap = static_cast<uint32_t*>(p);
  }
  return generate_with(g, count, dtype, d_out, out_bytes, stream, snap);
}

namespace {
int generate_with(prng_gen* g, uint64_t count, int dtype, void* d_out, size_t out_bytes, void* stream,
                  uint32_t* snap_area) {
  if (dtype < U32 || dtype > F32P) return fail(PRNG_EINVAL, "unknown dtype %d", dtype);
  if (dtype == F32P && (g->kind == DRAND48 || g->kind == RANNYU))
    return fail(PRNG_EUNSUPPORTED, "no paper single-precision rule for generator kind %d", g->kind);
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
    if (g->kind == RANLUX) {
      // The borrow chain runs one step at a time per lane; the kernel needs
      // two wavefronts per SIMD to overlap it with the stores.  Cut each
      // stream into K segments (jumped starts) so that about 2048 wavefronts
      // run, each segment at least 1536 draws long.
      const uint64_t d = c * per;
      const uint64_t waves = (g->n + 63) / 64;
      uint64_t K = std::min<uint64_t>({kLuxSplitMax, (2048 + waves - 1) / waves, std::max<uint64_t>(1, d / 1536)});
      uint64_t S = d;
      if (K > 1) {
        S = ((d + K - 1) / K + 95) / 96 * 96;
        K = (d + S - 1) / S;  // (K - 1) S < d: no segment is empty
      }
      uint32_t* snap = g->d_state;
      if (K > 1) {
        snap = snap_area;
        HIP_TRY(hipMemcpyAsync(snap, g->d_state, state_region_bytes(RANLUX, g->n), hipMemcpyDeviceToDevice, s));
      }
      HIP_TRY(launch_lux_plain(g->p, g->d_state, snap, g->n, d, dtype, (uint32_t)S, (uint32_t)K, lux_digits(g),
                               lux_aux(g), d_out, count, off, s));
      continue;
    }
    if (g->kind == XOR128) {
      // Cut each stream into K segments (jumped starts, each at least 2048
      // draws) so that about 4096 wavefronts are launched: at small stream
      // counts they fill SIMDs that one lane per stream would leave idle.
      // A workgroup's 128-draw stage takes 134 KB of LDS, so one runs per
      // CU and at 65536 streams the segments run one after another.
      const uint64_t d = c * per;
      const uint64_t waves = (g->n + 63) / 64;
      uint64_t K = std::min<uint64_t>({8, (4096 + waves - 1) / waves, std::max<uint64_t>(1, d / 2048)});
      if (K > 1) {
        const uint64_t S = ((d + K - 1) / K + 127) / 128 * 128;
        K = (d + S - 1) / S;  // (K - 1) S < d: no segment is empty
        if (K > 1) {
          HIP_TRY(hipMemcpyAsync(snap_area, g->d_state, state_region_bytes(XOR128, g->n), hipMemcpyDeviceToDevice, s));
          HIP_TRY(launch_xor128_split(g->d_state, snap_area, g->n, d, dtype, (uint32_t)S, (uint32_t)K,
                                      object_tables(g), d_out, count, off, s));
          continue;
        }
      }
    }
    HIP_TRY(launch_generate(g->kind, g->p, g->d_state, g->n, c * per, dtype, d_out, count, off, s));
  }
  return PRNG_OK;
}
}  // namespace

PRNG_API int prng_generate_packed4(prng_gen* g, uint64_t count, int dtype, void* d_out, size_t out_bytes,
                                   void* stream) {
  if (!g) return fail(PRNG_EINVAL, "g is NULL");
  if (!lane_kind(g->kind)) return fail(PRNG_EUNSUPPORTED, "no interleaved layout for generator kind %d", g->kind);
  if (dtype != U32 && dtype != F32 && dtype != F32P)
    return fail(PRNG_EINVAL, "interleaved layout takes 4-byte dtypes (got %d)", dtype);
  if (dtype == F32P && (g->kind == DRAND48 || g->kind == RANNYU))
    return fail(PRNG_EUNSUPPORTED, "no paper single-precision rule for generator kind %d", g->kind);
  if (g->n % 4) return fail(PRNG_EINVAL, "interleaved layout needs a multiple of 4 streams (got %llu)",
                            (unsigned long long)g->n);
  if (count == 0) return PRNG_OK;
  if (!d_out) return fail(PRNG_EINVAL, "d_out is NULL");
  if (reinterpret_cast<uintptr_t>(d_out) & 15) return fail(PRNG_EINVAL, "d_out must be 16-byte aligned");
  if (count > (1ull << 40)) return fail(PRNG_EINVAL, "count too large");
  if (out_bytes / 4 / g->n < count)
    return fail(PRNG_EINVAL, "d_out holds %zu bytes, %llu needed", out_bytes, (unsigned long long)(g->n * count * 4));
  DeviceGuard dg(g->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (uint64_t off = 0; off < count; off += kMaxDrawsPerLaunch) {
    const uint64_t c = count - off < kMaxDrawsPerLaunch ? count - off : kMaxDrawsPerLaunch;
    HIP_TRY(launch_generate_packed(g->kind, g->p, g->d_state, g->n, c, dtype, d_out, count, off, s));
  }
  return PRNG_OK;
}

PRNG_API int prng_ranlux_generate_variant(prng_gen* g, int variant, uint64_t count, int dtype, void* d_out,
                                          size_t out_bytes, void* stream) {
  if (!g) return fail(PRNG_EINVAL, "g is NULL");
  if (g->kind != RANLUX) return fail(PRNG_EINVAL, "not a RANLUX object (kind %d)", g->kind);
  if (variant == PRNG_LAG_REGISTERS) return prng_generate(g, count, dtype, d_out, out_bytes, stream);
  if (variant != PRNG_LAG_LDS && variant != PRNG_LAG_HBM) return fail(PRNG_EINVAL, "unknown variant %d", variant);
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
    HIP_TRY(launch_ranlux_variant(variant, g->p, g->d_state, g->n, c * per, dtype, d_out, count, off, s));
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
    if (g->kind == RANLUX && g->n <= 65536 && d >= 4 * 1440) {
      // RANLUX's borrow chain runs one step at a time per lane: cut each
      // stream into up to 64 segments (one wavefront per stream) of at least
      // 1440 draws, started from jumped states
      const uint64_t K0 = std::min<uint64_t>(kLuxSplitMax, d / 1440);
      const uint64_t S = ((d + K0 - 1) / K0 + 143) / 144 * 144;
      const uint64_t K = (d + S - 1) / S;  // (K - 1) S < d: no segment is empty
      uint32_t* snap = snapshot_area(g);
      HIP_TRY(hipMemcpyAsync(snap, g->d_state, state_region_bytes(RANLUX, g->n), hipMemcpyDeviceToDevice, s));
      HIP_TRY(launch_lux_fused_split(g->p, g->d_state, snap, g->n, d, (uint32_t)S, (uint32_t)K, lux_digits(g),
                                     lux_aux(g), d_sum, d_hist, off > 0, s));
      continue;
    }
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

