#pragma once
// Device code shared by the HIP translation units of libprng (gfx950,
// MI355X): generators, output staging and emission, the lane loop, the
// stream-table task decoder and the MT19937 block machinery.  The kernels
// and their launchers live in k_plain.hip, k_lux.hip, k_fused.hip,
// k_table.hip and k_init.hip; each includes this header (everything here is
// internal to its translation unit).
//
// Bulk uniform generation for the six
// generators of arXiv:1003.1898 (GGL, XOR128, RANECU, RANMAR, RANLUX, MT19937)
// and two more members of its LCG family, DRAND48 and RANNYU.
//
// Layout of the work
// ------------------
// * GGL, XOR128, RANECU, RANMAR, RANLUX, DRAND48, RANNYU: one lane per stream
//   (Section 3.1: independent sequences, one lag table per instance).  The
//   whole lag table lives in VGPRs (1, 4, 2, 97+1, 24+2 and 2 words) and is read from HBM once per
//   launch and written back once.  Tables with more than one lag (RANMAR,
//   RANLUX) are register rings whose slot for each step is fixed at compile
//   time; a chunk ends with a static renaming of the ring.  This is the
//   paper's "planar" idea (Section 3.6, the state held in registers instead of
//   global memory) taken to the CDNA4 register file.
// * Output: every lane writes its draws of one chunk into a per-wave LDS
//   stage, pairs of draws interleaved (draw j of lane l at
//   stage[(j >> 1) * 130 + 2 l + (j & 1)]); the wave then stores the chunk row
//   by row, each lane writing 8 bytes, so one store instruction writes up to
//   512 contiguous bytes of one stream instead of 64 scattered words.
// * MT19937: one wavefront per stream.  Its 624-word state (2.5 KB) sits in
//   LDS and the 64 lanes twist it cooperatively in ten rounds of 64 words
//   (words >= 227 read values made at least three rounds earlier), then
//   temper and store a block of 624 outputs with fully coalesced row stores.
//   The paper had to keep this table in global memory because 128 registers
//   per thread could not hold it (Section 3.7).
// * Segments (not in the paper): a long stream can be cut into segments that
//   start from states jumped ahead on the host-built data of jump.cpp, so
//   that the stream table, the serving loop and the RANLUX in-kernel consumer
//   keep the chip busy whatever the stream lengths.
//
// Per-lane virtual positions
// --------------------------
// A lane works on the virtual draw positions [vbeg, vend) of its stream.
// vbeg is 0 except for RANLUX, where it is the number of values already taken
// from the current luxury block, so that block boundaries of all lanes fall on
// the same positions and the skip code stays static.  Chunks where every lane
// is active run without per-step predication; the first and last chunks of
// uneven lanes run predicated.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "bigint576.h"
#include "internal.h"

namespace prng {
namespace {

constexpr int kPitch = 65;       // fused histogram: words per bin row (64 lanes + 1 pad word)
constexpr int kPairPitch = 130;  // stage: words per pair row (64 lanes x 2 draws + 2 pad words)

typedef uint32_t v2u __attribute__((ext_vector_type(2)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) uint32_t gu32;
typedef __attribute__((address_space(1))) float gf32;
typedef __attribute__((address_space(1))) double gf64;

// Output store of one element (or vector) at byte address `addr`.  NT makes
// it non-temporal: the line streams past the caches.  Measured on the full
// plain launches, that pays where much ALU and LDS work sits between the
// stores (MT19937: 7-10% faster; RANECU's leapfrog kernel: 3%) and costs 1-5%
// in the store-bound lane kernels, so each kernel picks.
template <class T, bool NT = false>
__device__ __forceinline__ void put(uint64_t addr, T v) {
  auto* p = reinterpret_cast<__attribute__((address_space(1))) T*>(addr);
  if constexpr (NT)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

// Stage of one wavefront for a chunk of T draws: draw j of lane l at
// stage[(j >> 1) * kPairPitch + 2 l + (j & 1)], so that lane L of the store
// phase reads draws 2L, 2L+1 of any row with one 8-byte LDS read.  One extra
// row holds each lane's last draw of the previous chunk (odd fp64 pairing).
template <int T>
constexpr int stage_words() { return (T / 2) * kPairPitch + 64; }
template <int T>
constexpr int carry_at() { return (T / 2) * kPairPitch; }

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Truth-table immediate of v_bitop3_b32 for a three-input bitwise function
// f(a, b, c): bit (a << 2 | b << 1 | c) of the table is f's value there.
template <class F>
constexpr int lut3(F f) {
  int r = 0;
  for (int i = 0; i < 8; ++i)
    if (f((i >> 2) & 1, (i >> 1) & 1, i & 1) & 1) r |= 1 << i;
  return r;
}
constexpr int kLutXorAnd = lut3([](int a, int b, int c) { return a ^ (b & c); });  // a ^ (b & c)
constexpr int kLutSelect = lut3([](int a, int b, int c) { return c ? a : b; });    // c picks a, else b

__device__ __forceinline__ uint32_t uni(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
__device__ __forceinline__ uint32_t rdlane(uint32_t v, int l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}
__device__ __forceinline__ uint64_t rdlane64(uint64_t v, int l) {
  return ((uint64_t)rdlane((uint32_t)(v >> 32), l) << 32) | rdlane((uint32_t)v, l);
}
__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o));
  return uni(v);
}
__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o));
  return uni(v);
}

// ------------------------------------------------------------ conversions
template <int BITS>
__device__ __forceinline__ float to_f32(uint32_t u) {
  return (float)(u >> (BITS - 24)) * 0x1p-24f;
}
template <int BITS>
__device__ __forceinline__ double to_f64(uint32_t u1, uint32_t u2) {
  if constexpr (BITS == 24) {
    return (double)u1 * 0x1p-24 + (double)u2 * 0x1p-48;
  } else {
    return (double)(u1 >> (BITS - 27)) * 0x1p-27 + (double)(u2 >> (BITS - 26)) * 0x1p-53;
  }
}

// ------------------------------------------------------------ arithmetic
// x * a mod m for m = 2^31 - c (c = 1 for GGL; 85 and 249 for RANECU):
// 2^31 = c (mod m), so the 47-bit product folds as hi * c + lo, which stays
// below 2m and needs at most one subtraction (min picks the in-range value).
template <uint32_t A, uint32_t C>
__device__ __forceinline__ uint32_t mul_mod_2p31(uint32_t x) {
  constexpr uint32_t M = 0x80000000u - C;
  uint64_t p = (uint64_t)x * A;
  uint32_t lo = (uint32_t)p & 0x7FFFFFFFu;
  uint32_t hi = (uint32_t)(p >> 31);
  uint32_t r = (C == 1) ? lo + hi : hi * C + lo;
  return min(r, r - M);
}

// x * a mod m for m = 2^31 - c and any a < m (jump-ahead multipliers).
template <uint32_t C>
__device__ __forceinline__ uint32_t mulmod_2p31(uint32_t x, uint32_t a) {
  constexpr uint32_t M = 0x80000000u - C;
  const uint64_t p = (uint64_t)x * a;
  uint64_t r = (p >> 31) * C + (p & 0x7FFFFFFFull);
  r = (r >> 31) * C + (r & 0x7FFFFFFFull);
  const uint32_t t = (uint32_t)r;
  return t >= M ? t - M : t;
}

// --------------------------------------------------------------- sinks
// The per-wave LDS stage of one chunk.  Draw j of lane l sits in slot
// (j >> 1) * 130 + 2 l + (j & 1), so the two draws of a pair are adjacent and
// the store phase reads draws 2P, 2P+1 of any row with one LDS read; each lane
// also keeps a carry word (its last draw of the previous chunk, for fp64
// pairs that straddle chunks).  StageWord32 holds 32-bit slots.  StageSplit24
// holds 24-bit draws as a 16-bit and an 8-bit array, three bytes a draw: a
// 96-draw stage then takes 18.7 KB instead of 25 KB and two wavefronts per
// SIMD fit in LDS.
template <int T>
struct StageWord32 {
  static constexpr int kBytes = stage_words<T>() * 4;
  uint32_t* s;
  __device__ __forceinline__ static int slot(int lane, int j) { return (j >> 1) * kPairPitch + 2 * lane + (j & 1); }
  __device__ __forceinline__ void put(int lane, int j, uint32_t u) const { s[slot(lane, j)] = u; }
  __device__ __forceinline__ uint32_t get(int lane, int j) const { return s[slot(lane, j)]; }
  __device__ __forceinline__ v2u pair(int prow, int lane) const {
    return *reinterpret_cast<const v2u*>(s + prow * kPairPitch + 2 * lane);
  }
  __device__ __forceinline__ uint32_t& carry(int lane) const { return s[carry_at<T>() + lane]; }
};

template <int T>
struct StageSplit24 {
  static constexpr int kSlots = (T / 2) * kPairPitch;
  static constexpr int kBytes = kSlots * 3 + 256;  // u16 low bits, u8 high bits, 64 carry words
  static_assert(kSlots % 2 == 0, "carry words stay 4-byte aligned");
  uint8_t* b;
  __device__ __forceinline__ uint16_t* lo() const { return reinterpret_cast<uint16_t*>(b); }
  __device__ __forceinline__ uint8_t* hi() const { return b + 2 * kSlots; }
  __device__ __forceinline__ static int slot(int lane, int j) { return (j >> 1) * kPairPitch + 2 * lane + (j & 1); }
  // One 16-bit and one 8-bit LDS store per draw, with no VALU work.  The empty
  // asm keeps the compiler from merging the stores of draws j and j + 1 into
  // wider ones, which costs about three VALU instructions per draw to pack.
  __device__ __forceinline__ void put(int lane, int j, uint32_t u) const {
    lo()[slot(lane, j)] = (uint16_t)u;
    hi()[slot(lane, j)] = (uint8_t)(u >> 16);
    asm volatile("" ::: "memory");
  }
  __device__ __forceinline__ uint32_t get(int lane, int j) const {
    return (uint32_t)lo()[slot(lane, j)] | ((uint32_t)hi()[slot(lane, j)] << 16);
  }
  // Draws 2 prow, 2 prow + 1 of a lane: each is one byte permute of the pair's
  // low halves l2 and high bytes h2 (v_perm_b32 selector bytes 0-3 pick l2,
  // 4-7 pick h2, 0x0C gives zero): (0, h2.b0, l2.b1, l2.b0) and (0, h2.b1,
  // l2.b3, l2.b2), most significant byte first.
  __device__ __forceinline__ v2u pair(int prow, int lane) const {
    const int i = prow * kPairPitch + 2 * lane;
    const uint32_t l2 = *reinterpret_cast<const uint32_t*>(lo() + i);
    const uint32_t h2 = *reinterpret_cast<const uint16_t*>(hi() + i);
    return v2u{__builtin_amdgcn_perm(h2, l2, 0x0C040100u), __builtin_amdgcn_perm(h2, l2, 0x0C050302u)};
  }
  __device__ __forceinline__ uint32_t& carry(int lane) const {
    return reinterpret_cast<uint32_t*>(b + 3 * kSlots)[lane];
  }
};

template <int T, bool SPLIT>
using StageOf = std::conditional_t<SPLIT, StageSplit24<T>, StageWord32<T>>;
template <int T, bool SPLIT>
__device__ __forceinline__ StageOf<T, SPLIT> stage_view(uint32_t* p) {
  if constexpr (SPLIT)
    return StageSplit24<T>{reinterpret_cast<uint8_t*>(p)};
  else
    return StageWord32<T>{p};
}

template <class SV>
struct StageSink {  // generation: draw j of the chunk goes to the wave's stage
  SV st;
  int lane;
  __device__ __forceinline__ void operator()(int j, uint32_t u) { st.put(lane, j, u); }
};

template <int BITS>
struct FusedSink {  // in-kernel consumer: mantissa sum and 64-bin histogram
  uint32_t acc;
  uint32_t* hcol;
  __device__ __forceinline__ void operator()(int, uint32_t u) {
    uint32_t k = u >> (BITS - 24);
    acc += k;
    __hip_atomic_fetch_add(&hcol[(k >> 18) * kPitch], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
  }
};

__device__ __forceinline__ bool active(uint32_t v, uint32_t vbeg, uint32_t vend) { return v >= vbeg && v < vend; }

// ============================================================ generators
// Each generator: T draws per chunk, BITS native width, load/store of the
// SoA state, and chunk<PRED>(lo, vbeg, vend, sink) producing the draws of
// virtual positions lo .. lo+T-1 (only the active ones when PRED).

// GGL: x <- 16807 x mod (2^31 - 1) (Appendix A.1).
template <int TT = 128>
struct Ggl {
  static constexpr int T = TT, BITS = 31;
  uint32_t x;
  __device__ void zero() { x = 1; }
  __device__ void load(const uint32_t* st, uint64_t, uint64_t si, uint32_t& vbeg) {
    x = st[si];
    vbeg = 0;
  }
  __device__ void store(uint32_t* st, uint64_t, uint64_t si, uint32_t, uint32_t) { st[si] = x; }
  // the paper's scaling x / 2147483647.0 in fp32, where that constant is 2^31
  static __device__ float paper_f32(uint32_t u) { return (float)u * 0x1p-31f; }
  // state J draws ahead: x a^J, with jd[0] = a^J mod m
  __device__ uint32_t load_jumped(const uint32_t* st, uint64_t, uint64_t si, const uint32_t* jd, const uint32_t*,
                                  uint32_t*) {
    x = mulmod_2p31<1u>(st[si], jd[0]);
    return 0;
  }
  template <bool PRED, class S>
  __device__ __forceinline__ void chunk(uint32_t lo, uint32_t vbeg, uint32_t vend, S& sink) {
#pragma unroll
    for (int j = 0; j < T; ++j) {
      if (!PRED || active(lo + j, vbeg, vend)) {
        x = mul_mod_2p31<16807u, 1u>(x);
        sink(j, x);
      }
    }
  }
};

// XOR128 (Appendix A.4.2): t = x ^ (x << 11); (x,y,z) <- (y,z,w);
// w <- (w ^ (w >> 19)) ^ (t ^ (t >> 8)).
template <int TT = 128>
struct Xor128 {
  static constexpr int T = TT, BITS = 32;
  uint32_t x, y, z, w;
  __device__ void zero() { x = y = z = 0; w = 1; }
  __device__ void load(const uint32_t* st, uint64_t sn, uint64_t si, uint32_t& vbeg) {
    x = st[si];
    y = st[sn + si];
    z = st[2 * sn + si];
    w = st[3 * sn + si];
    vbeg = 0;
  }
  __device__ void store(uint32_t* st, uint64_t sn, uint64_t si, uint32_t, uint32_t) {
    st[si] = x;
    st[sn + si] = y;
    st[2 * sn + si] = z;
    st[3 * sn + si] = w;
  }
  // the paper's scaling w / 4294967295.0 in fp32, where that constant is 2^32
  static __device__ float paper_f32(uint32_t u) { return (float)u * 0x1p-32f; }
  // state J steps ahead: the state's 128 bits times the GF(2) matrix T^J, whose
  // row i (jd[4i..4i+3]) is the image of state bit i (bit i % 32 of word i / 32)
  __device__ uint32_t load_jumped(const uint32_t* st, uint64_t sn, uint64_t si, const uint32_t* jd, const uint32_t*,
                                  uint32_t*) {
    const uint32_t in[4] = {st[si], st[sn + si], st[2 * sn + si], st[3 * sn + si]};
    uint32_t o[4] = {0u, 0u, 0u, 0u};
#pragma unroll 8
    for (int i = 0; i < 128; ++i) {
      const uint32_t mask = 0u - ((in[i >> 5] >> (i & 31)) & 1u);
      const v4u row = *reinterpret_cast<const v4u*>(jd + 4 * i);
      o[0] ^= row.x & mask;
      o[1] ^= row.y & mask;
      o[2] ^= row.z & mask;
      o[3] ^= row.w & mask;
    }
    x = o[0];
    y = o[1];
    z = o[2];
    w = o[3];
    return 0;
  }
  // state E steps ahead of the one at `st`: one product with T^(2^k) from
  // the object's table for every set bit k of E (E uniform over the wave)
  __device__ void load_jumped_pow2(const uint32_t* st, uint64_t sn, uint64_t si, uint32_t E, const uint32_t* pow2) {
    uint32_t s[4] = {st[si], st[sn + si], st[2 * sn + si], st[3 * sn + si]};
    for (int k = 0; k < kXorPow2; ++k) {
      if (!((E >> k) & 1u)) continue;
      const uint32_t* m = pow2 + 512 * k;
      uint32_t o[4] = {0u, 0u, 0u, 0u};
#pragma unroll 8
      for (int i = 0; i < 128; ++i) {
        const uint32_t mask = 0u - ((s[i >> 5] >> (i & 31)) & 1u);
        const v4u row = *reinterpret_cast<const v4u*>(m + 4 * i);
        o[0] ^= row.x & mask;
        o[1] ^= row.y & mask;
        o[2] ^= row.z & mask;
        o[3] ^= row.w & mask;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) s[q] = o[q];
    }
    x = s[0];
    y = s[1];
    z = s[2];
    w = s[3];
  }
  template <bool PRED, class S>
  __device__ __forceinline__ void chunk(uint32_t lo, uint32_t vbeg, uint32_t vend, S& sink) {
#pragma unroll
    for (int j = 0; j < T; ++j) {
      if (!PRED || active(lo + j, vbeg, vend)) {
        uint32_t t = x ^ (x << 11);
        x = y;
        y = z;
        z = w;
        w = (w ^ (w >> 19)) ^ (t ^ (t >> 8));
        sink(j, w);
      }
    }
  }
};

// RANECU (Appendix A.4.1): MLCGs (40014, 2^31-85) and (40692, 2^31-249),
// combined as s1 - s2, plus 2147483562 when <= 0.
template <int TT = 128>
struct Ranecu {
  static constexpr int T = TT, BITS = 31;
  uint32_t s1, s2;
  __device__ void zero() { s1 = s2 = 1; }
  __device__ void load(const uint32_t* st, uint64_t sn, uint64_t si, uint32_t& vbeg) {
    s1 = st[si];
    s2 = st[sn + si];
    vbeg = 0;
  }
  __device__ void store(uint32_t* st, uint64_t sn, uint64_t si, uint32_t, uint32_t) {
    st[si] = s1;
    st[sn + si] = s2;
  }
  // the paper's scaling Z * 2^-31
  static __device__ float paper_f32(uint32_t u) { return (float)u * 0x1p-31f; }
  // state J steps ahead: s1 a1^J mod m1, s2 a2^J mod m2 (jd = {a1^J, a2^J})
  __device__ uint32_t load_jumped(const uint32_t* st, uint64_t sn, uint64_t si, const uint32_t* jd, const uint32_t*,
                                  uint32_t*) {
    s1 = mulmod_2p31<85u>(st[si], jd[0]);
    s2 = mulmod_2p31<249u>(st[sn + si], jd[1]);
    return 0;
  }
  template <bool PRED, class S>
  __device__ __forceinline__ void chunk(uint32_t lo, uint32_t vbeg, uint32_t vend, S& sink) {
#pragma unroll
    for (int j = 0; j < T; ++j) {
      if (!PRED || active(lo + j, vbeg, vend)) {
        s1 = mul_mod_2p31<40014u, 85u>(s1);
        s2 = mul_mod_2p31<40692u, 249u>(s2);
        int32_t z = (int32_t)s1 - (int32_t)s2;
        z += (z <= 0) ? 2147483562 : 0;
        sink(j, (uint32_t)z);
      }
    }
  }
};

// 48-bit LCGs X <- a X + c mod 2^48 (Appendix A.1: DRAND48 with a =
// 25214903917, c = 11; RANNYU of Section 2 with a = 31167285, c = 0).  x0 holds
// the low 32 bits of X, x1 the rest; between steps x1 may carry garbage above
// bit 16, which only ever reaches bits >= 48 of the products and is cleared at
// store.  One step is a 32x32->64 multiply-add for the low word and the low
// halves of the two cross products for the high one.  The draw is X >> 16.
template <int TT, uint64_t A, uint32_t C>
struct Lcg48 {
  static constexpr int T = TT, BITS = 32;
  static constexpr uint32_t AL = (uint32_t)A, AH = (uint32_t)(A >> 32);
  uint32_t x0, x1;
  __device__ void zero() { x0 = 1; x1 = 0; }
  __device__ void load(const uint32_t* st, uint64_t sn, uint64_t si, uint32_t& vbeg) {
    x0 = st[si];
    x1 = st[sn + si];
    vbeg = 0;
  }
  __device__ void store(uint32_t* st, uint64_t sn, uint64_t si, uint32_t, uint32_t) {
    st[si] = x0;
    st[sn + si] = x1 & 0xFFFFu;
  }
  // state J steps ahead: A_J X + C_J mod 2^48, jd = {A_J lo, hi, C_J lo, hi}
  __device__ uint32_t load_jumped(const uint32_t* st, uint64_t sn, uint64_t si, const uint32_t* jd, const uint32_t*,
                                  uint32_t*) {
    const uint64_t x = (uint64_t)st[si] | ((uint64_t)st[sn + si] << 32);
    const uint64_t a = (uint64_t)jd[0] | ((uint64_t)jd[1] << 32), c = (uint64_t)jd[2] | ((uint64_t)jd[3] << 32);
    const uint64_t y = a * x + c;
    x0 = (uint32_t)y;
    x1 = (uint32_t)(y >> 32) & 0xFFFFu;
    return 0;
  }
  template <bool PRED, class S>
  __device__ __forceinline__ void chunk(uint32_t lo, uint32_t vbeg, uint32_t vend, S& sink) {
#pragma unroll
    for (int j = 0; j < T; ++j) {
      if (!PRED || active(lo + j, vbeg, vend)) {
        const uint64_t p = (uint64_t)x0 * AL + C;
        uint32_t h = (uint32_t)(p >> 32) + x1 * AL;
        if constexpr (AH != 0) h += x0 * AH;
        x0 = (uint32_t)p;
        x1 = h;
        sink(j, (x1 << 16) | (x0 >> 16));
      }
    }
  }
};
template <int TT = 128>
using Drand48 = Lcg48<TT, 25214903917ull, 11u>;
template <int TT = 128>
using Rannyu = Lcg48<TT, 31167285ull, 0u>;

// RANMAR (Appendix A.4.4): Y_n = Y_{n-97} - Y_{n-33} mod 2^24,
// C_n = C_{n-1} - 7654321 mod (2^24 - 3), X_n = Y_n - C_n mod 2^24.
// R[0..96] holds Y_{lo-97} .. Y_{lo-1} (oldest first).  A chunk computes T
// new values Y[j] from the concatenation R ++ Y with static indices; the new
// window is (R ++ Y)[T .. T+97).  A lane that stops inside the chunk after k steps
// writes its final window (R ++ Y)[k .. k+97) straight to its state words and
// rewinds C in closed form, C_k = C_0 - k D mod M; it takes no further steps.
template <int TT = 128>
struct Ranmar {
  static constexpr int T = TT, BITS = 24;
  static constexpr uint32_t D = 7654321u, M = 16777213u, MASK = 0xFFFFFFu;
  // the paper works on floats that are multiples of 2^-24: X * 2^-24, exact
  static __device__ float paper_f32(uint32_t u) { return (float)u * 0x1p-24f; }
  uint32_t R[97];
  uint32_t C;
  uint32_t* st_;
  uint64_t sn_, si_;
  bool stored_;
  __device__ void zero() {
#pragma unroll
    for (int m = 0; m < 97; ++m) R[m] = 0;
    C = 0;
    st_ = nullptr;
    stored_ = true;
  }
  __device__ void load(uint32_t* st, uint64_t sn, uint64_t si, uint32_t& vbeg) {
#pragma unroll
    for (int m = 0; m < 97; ++m) R[m] = st[m * sn + si];
    C = st[97 * sn + si];
    st_ = st;
    sn_ = sn;
    si_ = si;
    stored_ = false;
    vbeg = 0;
  }
  // where a lane that stops mid-chunk writes its final state (nullptr: nowhere)
  __device__ void retarget(uint32_t* st, uint64_t sn, uint64_t si) {
    st_ = st;
    sn_ = sn;
    si_ = si;
    stored_ = st == nullptr;
  }
  // Window J steps ahead.  With x^k standing for Y_{n-97+k}, the recurrence
  // reads x^97 = 1 - x^64, and Y_{n-97+J+t} is the dot product of the window
  // with the coefficients of x^{J+t} mod (x^97 + x^64 - 1).  jd[0..96] holds
  // x^J mod that polynomial; each further t multiplies by x (shift, fold the
  // top coefficient into x^0 and x^64).  New window values go through the
  // lane's LDS column `col` (stride 64 words) because t is a loop index.
  // jd[97] = J D mod M rewinds C.
  __device__ uint32_t load_jumped(uint32_t* st, uint64_t sn, uint64_t si, const uint32_t* jd, const uint32_t*,
                                  uint32_t* col) {
    uint32_t unused;
    load(st, sn, si, unused);
    uint32_t c[97];
#pragma unroll
    for (int i = 0; i < 97; ++i) c[i] = jd[i];
    for (int t = 0; t < 97; ++t) {
      uint32_t acc[4] = {0u, 0u, 0u, 0u};  // four independent sums
#pragma unroll
      for (int i = 0; i < 97; ++i) acc[i & 3] += __umul24(c[i], R[i]);
      col[t * 64] = (acc[0] + acc[1] + acc[2] + acc[3]) & MASK;
      const uint32_t top = c[96];
#pragma unroll
      for (int i = 96; i > 0; --i) c[i] = c[i - 1];
      c[0] = top;
      c[64] -= top;
    }
#pragma unroll
    for (int m = 0; m < 97; ++m) R[m] = col[m * 64];
    const uint32_t r = jd[97];
    C = C >= r ? C - r : C + (M - r);
    return 0;
  }
  __device__ void store(uint32_t* st, uint64_t sn, uint64_t si, uint32_t, uint32_t) {
    if (stored_) return;
#pragma unroll
    for (int m = 0; m < 97; ++m) st[m * sn + si] = R[m];
    st[97 * sn + si] = C;
  }
  template <bool PRED, class S>
  __device__ __forceinline__ void chunk(uint32_t lo, uint32_t vbeg, uint32_t vend, S& sink) {
    // fewest and most steps taken by the lanes that stop inside this chunk
    // (taken while every lane of the wave is active)
    uint32_t kmin = T, kmax = 0;
    if constexpr (PRED) {
      const bool stops = vend > lo && vend < lo + (uint32_t)T && vbeg < lo + (uint32_t)T;
      kmin = wave_min(stops ? vend - lo : (uint32_t)T);
      kmax = wave_max(stops ? vend - lo : 0u);
    }
    // a lane that finished, or starts in a later chunk, keeps its state (starts
    // are multiples of T: 0 or a segment boundary)
    if (PRED && (vend <= lo || vbeg >= lo + (uint32_t)T)) return;
    // C after step j is C_0 - (j+1) D mod M: a constant offset from the
    // chunk's start, so the steps do not wait on each other
    const uint32_t c0 = C;
    uint32_t Y[T];
#pragma unroll
    for (int j = 0; j < T; ++j) {
      const uint32_t a = j < 97 ? R[j] : Y[j - 97];
      const uint32_t b = j + 64 < 97 ? R[j + 64] : Y[j - 33];
      const uint32_t y = (a - b) & MASK;
      Y[j] = y;
      const uint32_t off = (uint32_t)(((uint64_t)(j + 1) * D) % M);
      const uint32_t cj = c0 >= off ? c0 - off : c0 + (M - off);
      if (!PRED || active(lo + j, vbeg, vend)) sink(j, (y - cj) & MASK);
    }
    {
      constexpr uint32_t offT = (uint32_t)(((uint64_t)T * D) % M);
      C = c0 >= offT ? c0 - offT : c0 + (M - offT);
    }
    if (PRED && vend < lo + (uint32_t)T) {
      // this lane stops after k steps (1 <= k < T): its window is
      // (R ++ Y)[k .. k + 97), oldest first, i.e. R[k ..] then Y[k - 97 .. k)
      // (only Y once k >= 97).  The wave visits, sixteen at a time, only the
      // values some stopping lane keeps.
      const uint32_t k = vend - lo;
      uint32_t* const base = st_ + si_;
#pragma unroll
      for (int i0 = 0; i0 < 97; i0 += 16) {
        constexpr int kEnd = 97;
        if ((uint32_t)(i0 + 16 < kEnd ? i0 + 16 : kEnd) <= kmin) continue;
#pragma unroll
        for (int i = i0; i < (i0 + 16 < kEnd ? i0 + 16 : kEnd); ++i)
          if ((uint32_t)i >= k) base[(uint64_t)((uint32_t)i - k) * sn_] = R[i];
      }
#pragma unroll
      for (int j0 = 0; j0 < T; j0 += 16) {
        if ((uint32_t)j0 >= kmax) break;
        if ((uint32_t)(j0 + 16 + 97) <= kmin) continue;
#pragma unroll
        for (int j = j0; j < j0 + 16; ++j)
          if ((uint32_t)j < k && (uint32_t)j + 97u >= k) base[(uint64_t)((uint32_t)j + 97u - k) * sn_] = Y[j];
      }
      const uint32_t r = (k * D) % M;
      st_[97 * sn_ + si_] = c0 >= r ? c0 - r : c0 + (M - r);
      stored_ = true;
    } else {
      // the new window is (R ++ Y)[T .. T + 97); ascending m reads R[m + T]
      // before it is overwritten
#pragma unroll
      for (int m = 0; m < 97; ++m) R[m] = m + T < 97 ? R[m + T] : Y[m + T - 97];
    }
  }
};

// RANLUX (Appendix A.4.5-A.4.6): SWB X_n = X_{n-10} - X_{n-24} - c mod 2^24
// (borrow c = 1 when negative); after 24 kept values the next p - 24 are
// discarded.  Register ring R[24]: the slot of step j is j mod 24.  A chunk
// holds five blocks of 24 kept values; the skip before a block runs
// (p - 24) / 24 whole revolutions plus (p - 24) % 24 steps and then renames
// the ring by that remainder so that every block starts at slot 0.
// One SWB step on 24-bit values held in 32-bit registers: the borrow out of
// the 32-bit a - x - c is exactly the borrow of the 24-bit subtraction, so the
// carry chain maps onto the hardware subtract-with-borrow and each step costs
// two VALU instructions (subtract with borrow, mask).
__device__ __forceinline__ void swb(uint32_t& x, uint32_t a, uint32_t& c) {
  uint32_t co;
  const uint32_t t = __builtin_subc(a, x, c, &co);
  c = co;
  x = t & 0xFFFFFFu;
}

// P > 0 fixes the luxury at compile time (the skip becomes straight-line
// code); P = 0 reads it from the member p.
template <int TT = 120, int P = 0>
struct Ranlux {
  static constexpr int T = TT, BITS = 24;
  // plain rows are stored non-temporally (see emit_full_plain)
  static constexpr bool kNtOut = true;
  // the paper's scaling X * 2^-24 (exact)
  static __device__ float paper_f32(uint32_t u) { return (float)u * 0x1p-24f; }
  uint32_t R[24];
  uint32_t c;
  uint32_t p;
  __device__ void zero() {
#pragma unroll
    for (int m = 0; m < 24; ++m) R[m] = 0;
    c = 0;
  }
  // Position k (values taken from the current block, 0..24) becomes the
  // lane's first virtual position, and the ring is placed so that the oldest
  // lag sits in slot k % 24.
  __device__ void load(const uint32_t* st, uint64_t sn, uint64_t si, uint32_t& vbeg) {
    const uint32_t k = st[25 * sn + si];
    const uint32_t ph = k % 24u;
#pragma unroll
    for (int m = 0; m < 24; ++m) {
      uint32_t t = (uint32_t)m + 24u - ph;
      t = t >= 24u ? t - 24u : t;
      R[m] = st[t * sn + si];
    }
    c = st[24 * sn + si];
    vbeg = k;
  }
  __device__ void store(uint32_t* st, uint64_t sn, uint64_t si, uint32_t vbeg, uint32_t vend) {
    const uint32_t ph = vend % 24u;
    const uint32_t k = (vend > vbeg) ? (vend - 1u) % 24u + 1u : vbeg;
#pragma unroll
    for (int m = 0; m < 24; ++m) {
      uint32_t t = (uint32_t)m + 24u - ph;
      t = t >= 24u ? t - 24u : t;
      st[t * sn + si] = R[m];
    }
    st[24 * sn + si] = c;
    st[25 * sn + si] = k;
  }
  // State at the next block boundary J' = jump multiplier's steps ahead:
  // convert lags and borrow to the LCG number S, finish the current block
  // (b^-(24-k) from aux), apply the segment's multiplier, convert back.  The
  // result sits at a block boundary: ring slot 0, borrow folded into S.
  __device__ uint32_t load_jumped(const uint32_t* st, uint64_t sn, uint64_t si, const uint32_t* jd,
                                  const uint32_t* aux, uint32_t*) {
    uint32_t S[18], A[18];
    const uint32_t k0 = lcg_at_block_end(st, sn, si, aux, S);
#pragma unroll
    for (int i = 0; i < 18; ++i) A[i] = jd[i];
    mulmod576(S, A, S);
    set_from_lcg(S);
    return k0;
  }
  // The same jump, E whole luxury blocks past the end of the current block,
  // with the multiplier taken digit by digit from the object's block-jump
  // table (entry (d, v) = b^-(p v 256^d)): one product per nonzero base-256
  // digit of E.
  __device__ uint32_t load_jumped_blocks(const uint32_t* st, uint64_t sn, uint64_t si, uint32_t E,
                                         const uint32_t* digits, const uint32_t* aux) {
    uint32_t S[18], A[18];
    const uint32_t k0 = lcg_at_block_end(st, sn, si, aux, S);
    for (int d = 0; d < kLuxDigits; ++d) {
      const uint32_t v = (E >> (8 * d)) & 255u;
      if (v == 0u) continue;
      const uint32_t* e = digits + ((uint32_t)d * 256u + v) * 18u;
#pragma unroll
      for (int i = 0; i < 18; ++i) A[i] = e[i];
      mulmod576(S, A, S);
    }
    set_from_lcg(S);
    return k0;
  }
  // The stream's state as the LCG number S, moved to the end of its current
  // block (b^-(24-k) from aux); returns k, the values already taken from it.
  __device__ uint32_t lcg_at_block_end(const uint32_t* st, uint64_t sn, uint64_t si, const uint32_t* aux,
                                       uint32_t* S) {
    uint32_t lag[24], A[18];
#pragma unroll
    for (int t = 0; t < 24; ++t) lag[t] = st[t * sn + si];
    const uint32_t c0 = st[24 * sn + si];
    const uint32_t k0 = st[25 * sn + si];
    swb_to_lcg(lag, c0, S);
    if (k0 < 24u) {
#pragma unroll
      for (int i = 0; i < 18; ++i) A[i] = aux[(24u - k0) * 18u + i];
      mulmod576(S, A, S);
    }
    return k0;
  }
  // Lags from S at a block boundary: ring slot 0, borrow folded into S.
  __device__ void set_from_lcg(const uint32_t* S) {
    uint32_t lag[24];
    lcg_to_swb(S, lag);
#pragma unroll
    for (int m = 0; m < 24; ++m) R[m] = lag[m];
    c = 0;
  }
  __device__ __forceinline__ void revolution() {
#pragma unroll
    for (int j = 0; j < 24; ++j) {
      swb(R[j], R[(j + 14) % 24], c);
    }
  }
  template <int D>
  __device__ __forceinline__ void tail_and_rename() {
#pragma unroll
    for (int j = 0; j < D; ++j) {
      swb(R[j], R[(j + 14) % 24], c);
    }
    uint32_t S[24];
#pragma unroll
    for (int m = 0; m < 24; ++m) S[m] = R[(m + D) % 24];
#pragma unroll
    for (int m = 0; m < 24; ++m) R[m] = S[m];
  }
  __device__ __forceinline__ void skip() {
    if constexpr (P > 0) {
      static_assert(P >= 24, "luxury below 24");
#pragma unroll
      for (int i = 0; i < (P - 24) / 24; ++i) revolution();
      if constexpr ((P - 24) % 24 != 0) tail_and_rename<(P - 24) % 24>();
      return;
    }
    const uint32_t q = uni((p - 24u) / 24u);
    for (uint32_t i = 0; i < q; ++i) revolution();
    switch (uni(p % 24u)) {
#define PRNG_RLX_CASE(d) \
  case d:                \
    tail_and_rename<d>(); \
    break;
      PRNG_RLX_CASE(1) PRNG_RLX_CASE(2) PRNG_RLX_CASE(3) PRNG_RLX_CASE(4) PRNG_RLX_CASE(5) PRNG_RLX_CASE(6)
      PRNG_RLX_CASE(7) PRNG_RLX_CASE(8) PRNG_RLX_CASE(9) PRNG_RLX_CASE(10) PRNG_RLX_CASE(11)
      PRNG_RLX_CASE(12) PRNG_RLX_CASE(13) PRNG_RLX_CASE(14) PRNG_RLX_CASE(15) PRNG_RLX_CASE(16)
      PRNG_RLX_CASE(17) PRNG_RLX_CASE(18) PRNG_RLX_CASE(19) PRNG_RLX_CASE(20) PRNG_RLX_CASE(21)
      PRNG_RLX_CASE(22) PRNG_RLX_CASE(23)
#undef PRNG_RLX_CASE
      default:
        break;
    }
  }
  template <bool PRED, class S>
  __device__ __forceinline__ void chunk(uint32_t lo, uint32_t vbeg, uint32_t vend, S& sink) {
#pragma unroll
    for (int b = 0; b < T / 24; ++b) {
      const uint32_t v0 = lo + 24u * b;
      // lazy skip: before a block (not the stream's first), and only for a
      // lane that generates a value of it
      if (v0 >= 24u && (!PRED || (v0 >= vbeg && v0 < vend))) skip();
#pragma unroll
      for (int j = 0; j < 24; ++j) {
        if (!PRED || active(v0 + j, vbeg, vend)) {
          swb(R[j], R[(j + 14) % 24], c);
          sink(24 * b + j, R[j]);
        }
      }
    }
  }
};

// RANLUX with its lag table outside the registers, for the comparison of the
// paper's three implementations (Section 3.6, Table 3).  kLagHbm keeps the 24
// lags in the stream's own state words and reads and writes them there at
// every step (the direct translation that updates the state in global
// memory); kLagLds keeps them in an indexed array in LDS (the temporary
// array).  Both walk the ring with a running index, as the classic algorithm
// does, and discard p - 24 values with a loop; the borrow stays in a register.
// Same chunk structure and virtual positions as Ranlux, so that the three
// variants share the emission and differ only in where the lag table lives.
constexpr int kLagLds = 1, kLagHbm = 2;

template <int TT, int WHERE>
struct RanluxMem {
  static constexpr int T = TT, BITS = 24;
  static_assert(T % 24 == 0, "chunks hold whole blocks of 24 kept values");
  uint32_t* lag;  // ring slot m at lag[m * ls]
  uint64_t ls;
  uint32_t i;     // ring slot of the oldest lag X_{n-24}
  uint32_t c;
  uint32_t p;
  __device__ void zero() {
    i = 0;
    c = 0;
  }
  // the wave's [24][64] LDS array, column `lane`: the ring of kLagLds, and
  // for kLagHbm the place where a lane without a stream steps harmlessly
  __device__ void bind(uint32_t* lds, int lane) {
    lag = lds + lane;
    ls = 64;
  }
  __device__ void load(uint32_t* st, uint64_t sn, uint64_t si, uint32_t& vbeg) {
    if constexpr (WHERE == kLagHbm) {
      lag = st + si;
      ls = sn;
    } else {
      for (int t = 0; t < 24; ++t) lag[t * ls] = st[t * sn + si];
    }
    i = 0;
    c = st[24 * sn + si];
    vbeg = st[25 * sn + si];
  }
  __device__ void store(uint32_t* st, uint64_t sn, uint64_t si, uint32_t vbeg, uint32_t vend) {
    uint32_t w[24];  // oldest first
    for (int t = 0; t < 24; ++t) {
      uint32_t m = i + (uint32_t)t;
      m = m >= 24u ? m - 24u : m;
      w[t] = lag[m * ls];
    }
    for (int t = 0; t < 24; ++t) st[t * sn + si] = w[t];
    st[24 * sn + si] = c;
    st[25 * sn + si] = (vend > vbeg) ? (vend - 1u) % 24u + 1u : vbeg;
  }
  __device__ __forceinline__ uint32_t step() {
    uint32_t j = i + 14u;  // X_{n-10}
    j = j >= 24u ? j - 24u : j;
    uint32_t x = lag[i * ls];
    swb(x, lag[j * ls], c);
    lag[i * ls] = x;
    i = i == 23u ? 0u : i + 1u;
    return x;
  }
  template <bool PRED, class S>
  __device__ __forceinline__ void chunk(uint32_t lo, uint32_t vbeg, uint32_t vend, S& sink) {
    for (int b = 0; b < T / 24; ++b) {
      const uint32_t v0 = lo + 24u * b;
      if (v0 >= 24u && (!PRED || (v0 >= vbeg && v0 < vend)))
        for (uint32_t d = 24; d < p; ++d) step();
#pragma unroll 4
      for (int j = 0; j < 24; ++j) {
        if (!PRED || active(v0 + j, vbeg, vend)) sink(24 * b + j, step());
      }
    }
  }
};

// ============================================================ emission
// Full chunk of a plain launch: all 64 rows of the wave are consecutive
// streams, every lane is active for the whole chunk and all lanes share the
// same virtual offset.  Row r is written at byte r * row_bytes of the buffer
// resource (which starts at row 0's first element of the chunk); lane L
// writes 8 bytes at 8 L: elements 2L, 2L+1 (u32/f32) or element L (f64).
// Chunks of at most 64 draws fill at most 32 pairs per row, so one store
// instruction covers two rows (lanes 0..31 the first, 32..63 the second).
template <int T>
struct RowSplit {
  static_assert(T <= 128, "the store phase covers at most 64 pairs per row");
  static constexpr int NP = T / 2;             // pairs per row in a chunk
  static constexpr int RPI = NP <= 32 ? 2 : 1;  // rows per store instruction
  static constexpr int LPR = 64 / RPI;         // lanes per row
};

// Single-precision element of draw u: the exact rule, or (F32P) the
// generator's own scaling as the paper's kernels write it.
template <class G, int DT>
__device__ __forceinline__ float cvt32(uint32_t u) {
  if constexpr (DT == F32P)
    return G::paper_f32(u);
  else
    return to_f32<G::BITS>(u);
}

template <class G, int DT>
__device__ __forceinline__ v2u convert_pair(v2u d) {
  v2u o;
  if constexpr (DT == U32) {
    o = d;
  } else if constexpr (DT == F32 || DT == F32P) {
    o.x = __float_as_uint(cvt32<G, DT>(d.x));
    o.y = __float_as_uint(cvt32<G, DT>(d.y));
  } else {
    const uint64_t b = (uint64_t)__double_as_longlong(to_f64<G::BITS>(d.x, d.y));
    o.x = (uint32_t)b;
    o.y = (uint32_t)(b >> 32);
  }
  return o;
}

// Non-temporal row stores for generators that ask for them (G::kNtOut).
// Measured on the full plain step: RANLUX's launches, which spend the most
// instructions between stores, gain 1-2% and leave less in the caches for the
// launch after them; GGL's, XOR128's and RANMAR's lose 4-6%.
template <class G>
constexpr int store_aux() {
  if constexpr (requires { G::kNtOut; })
    return G::kNtOut ? 2 : 0;  // buffer cache-policy bit 1: non-temporal
  else
    return 0;
}

template <class G, int DT, int T, class SV>
__device__ __forceinline__ void emit_full_plain(const SV& st, int lane, __amdgpu_buffer_rsrc_t rs,
                                                uint32_t row_bytes) {
  using RS = RowSplit<T>;
  const int h = lane / RS::LPR, P = lane % RS::LPR;  // row within the instruction, pair
  if (P >= RS::NP) return;
  const uint32_t voff = (uint32_t)P * 8u + (uint32_t)h * row_bytes;
#pragma unroll
  for (int r = 0; r < 64; r += RS::RPI) {
    const v2u d = st.pair(P, r + h);
    __builtin_amdgcn_raw_buffer_store_b64(convert_pair<G, DT>(d), rs, voff, (uint32_t)r * row_bytes, store_aux<G>());
  }
}

// Any chunk: row r emits the positions of this chunk inside its own
// [ebeg, vend); f64 pairs start at positions of the same parity as ebeg.
template <class G, int DT, int T, int ES = 4, class SV>
__device__ __forceinline__ void emit_general(const SV& st, int lane, uint32_t lo, uint64_t q,
                                             uint32_t ebeg, uint32_t vend) {
  static_assert(ES == 4 || DT != F64, "interleaved rows hold 4-byte elements");
  static_assert(T <= 128, "the store phase covers at most 64 pairs per row");
  constexpr int NP = T / 2;
  for (int r = 0; r < 64; ++r) {
    const uint32_t rb = rdlane(ebeg, r), re = rdlane(vend, r);
    if (re <= rb || re <= lo || rb >= lo + T) continue;
    const uint64_t rq = rdlane64(q, r);
    if (lane < NP) {
      const uint32_t v0 = lo + 2u * lane;
      const v2u d = st.pair(lane, r);
      if constexpr (DT != F64) {
        if (v0 >= rb && v0 < re) {
          if constexpr (DT == U32)
            put<uint32_t>(rq + (uint64_t)ES * v0, d.x);
          else
            put<float>(rq + (uint64_t)ES * v0, cvt32<G, DT>(d.x));
        }
        if (v0 + 1u >= rb && v0 + 1u < re) {
          if constexpr (DT == U32)
            put<uint32_t>(rq + (uint64_t)ES * (v0 + 1u), d.y);
          else
            put<float>(rq + (uint64_t)ES * (v0 + 1u), cvt32<G, DT>(d.y));
        }
      } else {
        if (((lo - rb) & 1u) == 0u) {
          if (v0 >= rb && v0 + 1u < re) put<double>(rq + 4ull * v0, to_f64<G::BITS>(d.x, d.y));
        } else {
          const uint32_t prev = lane == 0 ? st.carry(r) : st.get(r, 2 * lane - 1);
          if (v0 >= rb + 1u && v0 < re) put<double>(rq + 4ull * (v0 - 1u), to_f64<G::BITS>(prev, d.x));
        }
      }
    }
  }
}

// Chunk whose 64 rows are arbitrary output rows and each emits only the
// positions of its own range [ebeg, vend) inside the chunk (the first and last
// chunks of uneven segments): stores as in emit_full_rows, with a pair cut by
// its row's range, or a row not 8-byte aligned, written as 4-byte elements.
// fp64 needs every row's pairs to start at even positions (ebeg even).
template <class G, int DT, int T, class SV>
__device__ __forceinline__ void emit_partial_rows(const SV& st, int lane, uint32_t lo, uint64_t q, uint32_t ebeg,
                                                  uint32_t vend) {
  using RS = RowSplit<T>;
  const int h = lane / RS::LPR, P = lane % RS::LPR;
#pragma unroll 4
  for (int r = 0; r < 64; r += RS::RPI) {
    uint32_t rb = rdlane(ebeg, r), re = rdlane(vend, r);
    uint64_t rq = rdlane64(q, r);
    if constexpr (RS::RPI == 2) {
      const uint32_t rb1 = rdlane(ebeg, r + 1), re1 = rdlane(vend, r + 1);
      const uint64_t rq1 = rdlane64(q, r + 1);
      if (h) {
        rb = rb1;
        re = re1;
        rq = rq1;
      }
    }
    const uint32_t v0 = lo + 2u * (uint32_t)P;
    if (P >= RS::NP || re <= rb || v0 >= re || v0 + 2u <= rb) continue;
    const v2u d = st.pair(P, r + h);
    const bool in0 = v0 >= rb, in1 = v0 + 1u < re;
    if constexpr (DT == F64) {
      if (in0 && in1) put<double>(rq + 4ull * v0, to_f64<G::BITS>(d.x, d.y));
    } else {
      const v2u o = convert_pair<G, DT>(d);
      if (in0 && in1 && ((rq & 7u) == 0u)) {
        put<v2u>(rq + 4ull * v0, o);
      } else {
        if (in0) put<uint32_t>(rq + 4ull * v0, o.x);
        if (in1) put<uint32_t>(rq + 4ull * v0 + 4ull, o.y);
      }
    }
  }
}

// Full chunk whose 64 rows are arbitrary output rows (stream table): same
// 8-byte-per-lane stores as the plain path; row r's element for virtual
// position v sits at q_r + 4 v (q from row r's lane).
template <class G, int DT, int T, class SV>
__device__ __forceinline__ void emit_full_rows(const SV& st, int lane, uint32_t lo, uint64_t q) {
  using RS = RowSplit<T>;
  const int h = lane / RS::LPR, P = lane % RS::LPR;
#pragma unroll 8
  for (int r = 0; r < 64; r += RS::RPI) {
    const uint64_t q0 = rdlane64(q, r);
    const uint64_t rq = RS::RPI == 2 ? (h ? rdlane64(q, r + 1) : q0) : q0;
    if (P < RS::NP) {
      const v2u d = st.pair(P, r + h);
      put<v2u>(rq + 4ull * lo + 8ull * (uint32_t)P, convert_pair<G, DT>(d));
    }
  }
}

// Full chunk of a four-way interleaved launch: streams 4g .. 4g+3 (lanes
// 4g .. 4g+3) share one row whose element v is a 16-byte vector of their four
// draws of position v, as the paper's kernels store the four subthreads of a
// register.  Per group, lane L writes the vector of position lo + L (+ 64),
// so one store instruction covers 1 KB of the group's row; q of lane 4g is
// the group's row address at position 0.
template <class G, int DT, int T, class SV>
__device__ __forceinline__ void emit_full_pack4(const SV& st, int lane, uint32_t lo, uint64_t q) {
  static_assert(DT != F64, "interleaved rows hold 4-byte elements");
#pragma unroll 4
  for (int gi = 0; gi < 16; ++gi) {
    const uint64_t base = rdlane64(q, 4 * gi) + 16ull * lo;
#pragma unroll
    for (int h = 0; h < (T + 63) / 64; ++h) {
      const int j = lane + 64 * h;
      if (j < T) {
        v4u o{st.get(4 * gi, j), st.get(4 * gi + 1, j), st.get(4 * gi + 2, j), st.get(4 * gi + 3, j)};
        if constexpr (DT != U32)
          o = v4u{__float_as_uint(cvt32<G, DT>(o.x)), __float_as_uint(cvt32<G, DT>(o.y)),
                  __float_as_uint(cvt32<G, DT>(o.z)), __float_as_uint(cvt32<G, DT>(o.w))};
        put<v4u>(base + 16ull * (uint32_t)j, o);
      }
    }
  }
}

// Chunk loop of one wavefront of lane-per-stream work.  Per lane: the state
// stands at virtual position gbeg; positions [gbeg, vend) are generated and
// [ebeg, vend) emitted; the element of position v (the first draw of an f64
// pair) is written at byte address q + 4 v.  `plain` says the 64 rows are
// consecutive streams `row_bytes` apart (q of lane r = q of lane 0 + r
// row_bytes).
template <class G, int DT, bool PACK = false, bool SPLIT = false>
__device__ __forceinline__ void lane_loop(G& g, uint32_t* stage, int lane, uint32_t gbeg, uint32_t ebeg, uint32_t vend,
                                          uint64_t q, bool plain, uint64_t row_bytes) {
  constexpr uint32_t T = G::T;
  static_assert(!SPLIT || G::BITS == 24, "the three-byte stage holds 24-bit draws");
  const auto st = stage_view<T, SPLIT>(stage);
  const bool has = vend > ebeg;
  const uint32_t maxb = wave_max(has ? ebeg : 0u);
  const uint32_t minb = wave_min(has ? ebeg : 0xFFFFFFFFu);
  const uint32_t minE = wave_min(has ? vend : 0xFFFFFFFFu);
  const uint32_t maxE = wave_max(has ? vend : 0u);
  const uint32_t ming = wave_min(has ? gbeg : 0xFFFFFFFFu);
  const uint32_t nlive = uni((uint32_t)__popcll(__ballot(has)));
  const uint32_t nalign = uni((uint32_t)__popcll(__ballot(has && (q & 7u) == 0u)));
  // fp64 pairs of every row start at even positions (so a chunk's pairs are the rows' pairs)
  const bool even_pairs = DT != F64 || uni((uint32_t)__popcll(__ballot(has && ((ebeg & 1u) || (q & 7u))))) == 0u;
  // every row live and 8-byte aligned at even positions: unchecked 8-byte stores
  const bool even = nlive == 64u && nalign == 64u;
  // the rows must also sit exactly row_bytes apart (streams at different
  // positions of their blocks may share a segment-local start)
  const uint64_t q0 = rdlane64(q, 0);
  const uint32_t nstride = uni((uint32_t)__popcll(__ballot(q == q0 + (uint64_t)lane * row_bytes)));
  plain = plain && even && nstride == 64u && minb == maxb && 63ull * row_bytes + 4ull * T < 0x7FFFFFFFull;
  // row 0's element at the common first position (lane 0 is live when plain)
  uint8_t* const wave_base = reinterpret_cast<uint8_t*>(q0 + 4ull * minb);
  // interleaved rows: every lane live, a common start, and each group's row
  // 16-byte aligned with lanes 4g+1 .. 4g+3 at 4, 8, 12 bytes after lane 4g
  bool pack_full = false;
  if constexpr (PACK) {
    const uint64_t qg = __shfl(q, lane & ~3);
    const bool ok = has && (qg & 15u) == 0u && q == qg + 4ull * (uint64_t)(lane & 3);
    pack_full = nlive == 64u && minb == maxb && uni((uint32_t)__popcll(__ballot(ok))) == 64u;
  }
  const uint32_t first = ming == 0xFFFFFFFFu ? 0u : ming / T;  // chunks before every lane's start are skipped
  const uint32_t nchunks = (maxE + T - 1) / T;
  StageSink<StageOf<T, SPLIT>> sink{st, lane};
  for (uint32_t c = first; c < nchunks; ++c) {
    const uint32_t lo = c * T;
    if (lo >= maxb && lo + T <= minE) {
      g.template chunk<false>(lo, gbeg, vend, sink);
      wave_sync();
      if constexpr (PACK) {
        if (pack_full)
          emit_full_pack4<G, DT, T>(st, lane, lo, q);
        else
          emit_general<G, DT, T, 16>(st, lane, lo, q, ebeg, vend);
      } else if (plain) {
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            wave_base + 4ull * (uint64_t)(lo - minb), (short)0, (int)(63u * (uint32_t)row_bytes + 4u * T),
            0x00020000);
        emit_full_plain<G, DT, T>(st, lane, rs, (uint32_t)row_bytes);
      } else if (even) {
        emit_full_rows<G, DT, T>(st, lane, lo, q);
      } else if (even_pairs) {
        emit_partial_rows<G, DT, T>(st, lane, lo, q, ebeg, vend);
      } else {
        emit_general<G, DT, T>(st, lane, lo, q, ebeg, vend);
      }
    } else {
      g.template chunk<true>(lo, gbeg, vend, sink);
      wave_sync();
      if constexpr (PACK)
        emit_general<G, DT, T, 16>(st, lane, lo, q, ebeg, vend);
      else if (even_pairs)
        emit_partial_rows<G, DT, T>(st, lane, lo, q, ebeg, vend);
      else
        emit_general<G, DT, T>(st, lane, lo, q, ebeg, vend);
    }
    wave_sync();
    if constexpr (DT == F64) {  // keep each lane's last draw for a pair that straddles chunks
      st.carry(lane) = st.get(lane, T - 1);
      wave_sync();
    }
  }
}

// Row holding full segment g of a task's group: binary search over the
// task's rows, whose first segments increase.
__device__ __forceinline__ uint32_t segment_row(const TableRow* __restrict__ rows, const TableTask& task, uint64_t g) {
  uint32_t lo = task.row0, hi = task.row1;
  while (lo < hi) {
    const uint32_t mid = lo + (hi - lo + 1u) / 2u;
    if (rows[mid].first <= g)
      lo = mid;
    else
      hi = mid - 1u;
  }
  return lo;
}

// One task of the stream table: up to 64 segments of one (kind, p, dtype), one
// per lane, each with its own state, output row and virtual range.  Virtual
// positions count from where the stream stands at the start of the run (for
// RANLUX: k, the values already taken from its current luxury block).
// Segment j covers [j L, (j+1) L) of that axis (the first from k, the last to
// k + draws); an f64 pair straddling a boundary goes to the earlier segment,
// which then generates one position more.
template <class G, int DT, bool SPLIT = false>
__device__ __forceinline__ void lane_task(uint32_t* stage, int lane, const TableRow* __restrict__ rows,
                                          const uint32_t* __restrict__ tails, const TableTask& task, uint32_t p,
                                          const uint32_t* aux) {
  G g;
  if constexpr (requires { g.p; }) g.p = p;
  const bool live = (uint32_t)lane < task.nseg;
  uint32_t k0 = 0, gbeg = 0, ebeg = 0, vend = 0, last = 0;
  uint64_t q = 0;
  uint32_t* wst = nullptr;
  uint64_t wsn = 0, wsi = 0;
  if (live) {
    uint32_t r, j;
    if (task.tail) {
      r = tails[task.g0 + (uint32_t)lane];
      j = rows[r].nseg - 1u;
    } else {
      r = segment_row(rows, task, task.g0 + (uint32_t)lane);
      j = (uint32_t)(task.g0 + (uint32_t)lane - rows[r].first);
    }
    const TableRow& rw = rows[r];
    const uint32_t S = rw.seg_len;
    if (j == 0) {
      g.load(rw.state, rw.sn, rw.si, k0);
      gbeg = k0;
    } else {
      k0 = g.load_jumped(rw.state, rw.sn, rw.si, rw.jump + (j - 1u) * rw.jstride, aux, stage + lane);
      gbeg = j * S;
    }
    constexpr bool f64 = DT == F64;
    last = j + 1u == rw.nseg ? 1u : 0u;
    vend = last ? k0 + rw.draws : (j + 1u) * S + ((f64 && (((j + 1u) * S - k0) & 1u)) ? 1u : 0u);
    ebeg = j == 0 ? k0 : j * S + ((f64 && ((j * S - k0) & 1u)) ? 1u : 0u);
    q = reinterpret_cast<uint64_t>(rw.out) - 4ull * k0;
    // Work in coordinates local to the segment so that the lanes of a task,
    // whatever their segment index, cover about the same chunks.  The shift
    // is a multiple of 384 (luxury blocks, chunks); a RANLUX segment keeps its
    // pending skip by starting at local position 24.  With the three-byte
    // stage (RANLUX, 96-draw chunks) the shift is instead chosen per lane as
    // in k_lux_plain: a multiple of 24 congruent to k0 mod 32 when k0 is a
    // multiple of 8, so that the row's chunk pieces start on 128-byte lines.
    int32_t off = j == 0 ? 0 : (int32_t)(requires { g.p; } ? j * S - 24u : j * S);
    if constexpr (SPLIT) {
      if (k0 % 8u == 0u) {
        const uint32_t w = (k0 / 8u) & 3u;
        off = j == 0 ? -24 * (int32_t)w : (int32_t)(j * S) - 24 * (int32_t)(((w + 3u) & 3u) + 1u);
      }
    }
    gbeg = (uint32_t)((int32_t)gbeg - off);
    ebeg = (uint32_t)((int32_t)ebeg - off);
    vend = (uint32_t)((int32_t)vend - off);
    q += (uint64_t)(4ll * off);
    wst = rw.wstate;
    wsn = rw.wsn;
    wsi = rw.wsi;
  } else {
    g.zero();
  }
  if constexpr (requires { g.retarget(wst, wsn, wsi); }) g.retarget(last ? wst : nullptr, wsn, wsi);
  wave_sync();
  lane_loop<G, DT, false, SPLIT>(g, stage, lane, gbeg, ebeg, vend, q, false, 0);
  if (live && last) g.store(wst, wsn, wsi, gbeg, vend);
}

// ============================================================ MT19937
constexpr uint32_t kMtUpper = 0x80000000u, kMtLower = 0x7FFFFFFFu, kMtA = 0x9908B0DFu;

// Tempering; each masked step t ^ ((t << k) & M) is one three-input bitwise
// instruction after the shift.
__device__ __forceinline__ uint32_t mt_temper(uint32_t t) {
  t ^= t >> 11;
  t = __builtin_amdgcn_bitop3_b32(t, t << 7, 0x9D2C5680u, kLutXorAnd);
  t = __builtin_amdgcn_bitop3_b32(t, t << 15, 0xEFC60000u, kLutXorAnd);
  t ^= t >> 18;
  return t;
}

// Cooperative block twist of one stream by one wavefront: round r updates
// words 64r .. 64r+63 in place.  Word i reads words i and i+1 before the
// block's update (i+1 in the same or the next round) and word i+397, or for
// i >= 227 the new word i-227 (written at least 3.5 rounds earlier; word 623
// reads the new word 0).  Rounds are therefore taken three at a time, all
// reads of a group before its writes: groups {0,1,2}, {3,4,5}, {6,7,8}, {9}.
__device__ __forceinline__ void mt_twist(uint32_t* mt, int lane) {
#pragma unroll
  for (int r0 = 0; r0 < 10; r0 += 3) {
    uint32_t a[3], b[3], x[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int i = (r0 + q) * 64 + lane;
      a[q] = b[q] = x[q] = 0;
      if (r0 + q < 10 && i < 624) {
        a[q] = mt[i];
        b[q] = mt[i + 1 == 624 ? 0 : i + 1];
        x[q] = mt[i + 397 >= 624 ? i - 227 : i + 397];
      }
    }
    wave_sync();
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int i = (r0 + q) * 64 + lane;
      if (r0 + q < 10 && i < 624) {
        // y = upper bit of a, lower 31 bits of b (one select instruction);
        // bit 0 of y is bit 0 of b
        const uint32_t y = __builtin_amdgcn_bitop3_b32(a[q], b[q], kMtUpper, kLutSelect);
        mt[i] = x[q] ^ (y >> 1) ^ ((b[q] & 1u) ? kMtA : 0u);
      }
    }
    wave_sync();
  }
}

// The block twist of mt_twist that also hands every word of the current block,
// as it is read for the twist, to emit(i, word) (lane l: words 64 r + l).  A
// group's words are emitted after the next group's reads are issued, so the
// tempering and stores of one group fill the LDS latency of the next.  The
// table then holds the next block: callers use it only when draws remain
// after the emitted block.
template <class E>
__device__ __forceinline__ void mt_twist_emit(uint32_t* mt, int lane, E& emit) {
  uint32_t a[3], b[3], x[3];
  auto fetch = [&](int r0) {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int i = (r0 + q) * 64 + lane;
      a[q] = b[q] = x[q] = 0;
      if (r0 + q < 10 && i < 624) {
        a[q] = mt[i];
        b[q] = mt[i + 1 == 624 ? 0 : i + 1];
        x[q] = mt[i + 397 >= 624 ? i - 227 : i + 397];
      }
    }
  };
  fetch(0);
#pragma unroll
  for (int r0 = 0; r0 < 10; r0 += 3) {
    uint32_t nw[3], old[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const uint32_t y = __builtin_amdgcn_bitop3_b32(a[q], b[q], kMtUpper, kLutSelect);
      nw[q] = x[q] ^ (y >> 1) ^ ((b[q] & 1u) ? kMtA : 0u);
      old[q] = a[q];
    }
    wave_sync();  // every read of the group before any of its writes
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int i = (r0 + q) * 64 + lane;
      if (r0 + q < 10 && i < 624) mt[i] = nw[q];
    }
    wave_sync();
    if (r0 + 3 < 10) fetch(r0 + 3);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int i = (r0 + q) * 64 + lane;
      if (r0 + q < 10 && i < 624) emit(i, old[q]);
    }
  }
  wave_sync();
}

// Single-precision MT19937 element: the exact rule, or (F32P) the paper's
// (y + 0.5) / 4294967296.0 in fp32 (the integer rounded, then the sum; the
// division by 2^32 is exact).
template <int DT>
__device__ __forceinline__ float mt_f32(uint32_t u) {
  if constexpr (DT == F32P)
    return ((float)u + 0.5f) * 0x1p-32f;
  else
    return to_f32<32>(u);
}

// Stores m staged draws (stage words 1 .. m) of a block from launch draw
// `done`, by the 256 threads of a workgroup.
template <int DT>
__device__ __forceinline__ void mt_emit(const uint32_t* st, int tid, uint32_t done, uint32_t m, uint64_t outp) {
  constexpr uint32_t NT = 256;
  if constexpr (DT != F64) {
    for (uint32_t j = tid; j < m; j += NT) {
      const uint32_t u = st[1 + j];
      if constexpr (DT == U32)
        put<uint32_t, true>(outp + 4ull * (done + j), u);
      else
        put<float, true>(outp + 4ull * (done + j), mt_f32<DT>(u));
    }
  } else {
    // pairs (2e, 2e+1) of the launch's draws whose second draw is in this block
    const uint32_t first = (done & 1u) ? done : done + 1u;
    for (uint32_t v2 = first + 2u * tid; v2 < done + m; v2 += 2u * NT) {
      const uint32_t s2 = v2 - done + 1u;
      put<double, true>(outp + 8ull * (v2 >> 1), to_f64<32>(st[s2 - 1u], st[s2]));
    }
  }
}

// Block twist by the 256 threads of a workgroup (four wavefronts on one
// stream): word i reads words i, i+1 and i+397 of the old block, or for
// i >= 227 the new word i-227, so the block is updated in three phases of at
// most 227 words ([0,227), [227,454), [454,624)), each reading only old words
// and words of earlier phases; every read of a phase precedes its writes.
__device__ __forceinline__ void mt_twist_block(uint32_t* mt, int tid) {
#pragma unroll
  for (int ph = 0; ph < 3; ++ph) {
    const int i = ph * 227 + tid;
    const bool on = tid < 227 && i < 624;
    uint32_t a = 0, b = 0, x = 0;
    if (on) {
      a = mt[i];
      b = mt[i + 1 == 624 ? 0 : i + 1];
      x = mt[i + 397 >= 624 ? i - 227 : i + 397];
    }
    __syncthreads();
    if (on) {
      const uint32_t y = __builtin_amdgcn_bitop3_b32(a, b, kMtUpper, kLutSelect);
      mt[i] = x ^ (y >> 1) ^ ((b & 1u) ? kMtA : 0u);
    }
    __syncthreads();
  }
}

// One stream of MT19937 by the 256 threads of a workgroup (every argument
// block-uniform, so every barrier is reached by all of them): load the table
// from `src` into LDS (unless src is null and it is there already) at
// position pos0 (skipping `skip` draws of a fresh block when pos0 is 624),
// produce `draws` draws into the output row `outp`
// (address of element 0), and store the table to `sdst` unless it is null.
// Used by the plain kernel and by the stream-table kernel.
template <int DT>
__device__ __forceinline__ void mt_body(uint32_t* mt, uint32_t* st, int tid, const uint32_t* src, uint32_t pos0,
                                        uint32_t skip, uint32_t draws, uint64_t outp, uint32_t* sdst) {
  constexpr uint64_t es = DT == F64 ? 8 : 4;
  constexpr uint32_t per = DT == F64 ? 2 : 1;
  constexpr uint32_t NT = 256;
  if (src) {  // null: the caller has put the table into LDS already
    for (int i = tid; i < 624; i += NT) mt[i] = src[i];
    __syncthreads();
  }
  uint32_t pos = pos0;
  if (skip) {
    mt_twist_block(mt, tid);
    pos = skip;
  }
  uint32_t done = 0;
  while (done < draws) {
    if (pos >= 624u) {
      mt_twist_block(mt, tid);
      pos = 0;
    }
    const uint32_t m = min(624u - pos, draws - done);
    // byte address of the block's first output; u32/f32 draws and f64 pairs
    // both take 4 bytes per draw, so draw w of the block lands at dst + 4 w
    const uint64_t dst = outp + (uint64_t)(done / per) * es;
    if (pos == 0u && m == 624u && (dst & 15u) == 0u && (DT != F64 || (done & 1u) == 0u)) {
      // whole block, 16-byte aligned: four consecutive words per thread
      const int w0 = 4 * tid;
      if (w0 < 624) {
        const v4u x = *reinterpret_cast<const v4u*>(mt + w0);
        const uint32_t t0 = mt_temper(x.x), t1 = mt_temper(x.y), t2 = mt_temper(x.z), t3 = mt_temper(x.w);
        v4u o;
        if constexpr (DT == U32) {
          o = v4u{t0, t1, t2, t3};
        } else if constexpr (DT == F32 || DT == F32P) {
          o = v4u{__float_as_uint(mt_f32<DT>(t0)), __float_as_uint(mt_f32<DT>(t1)),
                  __float_as_uint(mt_f32<DT>(t2)), __float_as_uint(mt_f32<DT>(t3))};
        } else {
          const uint64_t a = (uint64_t)__double_as_longlong(to_f64<32>(t0, t1));
          const uint64_t b = (uint64_t)__double_as_longlong(to_f64<32>(t2, t3));
          o = v4u{(uint32_t)a, (uint32_t)(a >> 32), (uint32_t)b, (uint32_t)(b >> 32)};
        }
        put<v4u, true>(dst + 4ull * (uint64_t)w0, o);
      }
      if constexpr (DT == F64) {
        if (tid == 0) st[0] = mt_temper(mt[623]);
      }
    } else if (DT != F64 && (pos & 3u) == 0u && (dst & 15u) == 0u) {
      // part of a block from a multiple of four, 16-byte aligned: four
      // consecutive words per thread as above, then the last m mod 4 one by one
      const uint32_t m4 = m & ~3u;
      for (uint32_t w0 = 4u * (uint32_t)tid; w0 < m4; w0 += 4u * NT) {
        const v4u x = *reinterpret_cast<const v4u*>(mt + pos + w0);
        const uint32_t t0 = mt_temper(x.x), t1 = mt_temper(x.y), t2 = mt_temper(x.z), t3 = mt_temper(x.w);
        v4u o;
        if constexpr (DT == U32)
          o = v4u{t0, t1, t2, t3};
        else
          o = v4u{__float_as_uint(mt_f32<DT>(t0)), __float_as_uint(mt_f32<DT>(t1)), __float_as_uint(mt_f32<DT>(t2)),
                  __float_as_uint(mt_f32<DT>(t3))};
        put<v4u, true>(dst + 4ull * w0, o);
      }
      for (uint32_t j = m4 + (uint32_t)tid; j < m; j += NT) {
        const uint32_t t = mt_temper(mt[pos + j]);
        if constexpr (DT == U32)
          put<uint32_t, true>(dst + 4ull * j, t);
        else
          put<float, true>(dst + 4ull * j, mt_f32<DT>(t));
      }
    } else {
      for (uint32_t j = tid; j < m; j += NT) st[1 + j] = mt_temper(mt[pos + j]);
      __syncthreads();
      mt_emit<DT>(st, tid, done, m, outp);
      __syncthreads();
      if constexpr (DT == F64) {
        if (tid == 0) st[0] = st[m];
      }
    }
    __syncthreads();
    pos += m;
    done += m;
  }
  if (sdst) {
    for (int i = tid; i < 624; i += NT) sdst[i] = mt[i];
    if (tid == 0) sdst[624] = pos;
  }
  __syncthreads();
}

// ============================================================ stream table
// Persistent kernels of the stream table.  Every wavefront pulls task
// indices from an atomic counter until the list is exhausted, so every wave
// reaches the exit; tasks are ordered longest first on the host.
__device__ __forceinline__ uint32_t next_task(uint32_t* counter, int lane) {
  uint32_t t = 0;
  if (lane == 0) t = atomicAdd(counter, 1u);
  return uni((uint32_t)__shfl((int)t, 0));
}

// Lane-per-stream tasks come in two kernels (classes).  GGL, XOR128, RANECU,
// DRAND48 and RANNYU take 64-draw chunks (a 16.5 KB LDS stage per
// wavefront) and RANLUX 96-draw chunks in the three-byte stage (18.7 KB), so
// two blocks share a CU: a second wavefront per SIMD overlaps its work (for
// RANLUX the borrow chain) with the other's stores.  RANMAR (97-word window
// plus a chunk of new values in registers, and a 97 x 97 jump) needs most of
// the register file, one wavefront per SIMD; with the CU to itself it takes
// 128-draw chunks (a 32.8 KB stage per wavefront), which halves the window
// moves per draw.
constexpr int kClassT[kLaneClasses] = {64, 128};
constexpr int kLuxTableT = 96;

}  // namespace
}  // namespace prng
