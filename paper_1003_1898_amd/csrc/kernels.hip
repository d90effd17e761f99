// HIP kernels for gfx950 (MI355X): bulk uniform generation for the six
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
struct StageSink {  // generation: draw j of the chunk goes to the wave's stage
  uint32_t* base;   // stage + 2 * lane
  __device__ __forceinline__ void operator()(int j, uint32_t u) { base[(j >> 1) * kPairPitch + (j & 1)] = u; }
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
      const uint32_t k = vend - lo;
#pragma unroll
      for (int i = 0; i < 97 + T; ++i) {
        const uint32_t t = (uint32_t)i - k;
        if (t < 97u) st_[t * sn_ + si_] = i < 97 ? R[i] : Y[i - 97];
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
    uint32_t lag[24];
#pragma unroll
    for (int t = 0; t < 24; ++t) lag[t] = st[t * sn + si];
    const uint32_t c0 = st[24 * sn + si];
    const uint32_t k0 = st[25 * sn + si];
    uint32_t S[18], A[18];
    swb_to_lcg(lag, c0, S);
    if (k0 < 24u) {
#pragma unroll
      for (int i = 0; i < 18; ++i) A[i] = aux[(24u - k0) * 18u + i];
      mulmod576(S, A, S);
    }
#pragma unroll
    for (int i = 0; i < 18; ++i) A[i] = jd[i];
    mulmod576(S, A, S);
    lcg_to_swb(S, lag);
#pragma unroll
    for (int m = 0; m < 24; ++m) R[m] = lag[m];
    c = 0;
    return k0;
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

template <class G, int DT, int T>
__device__ __forceinline__ void emit_full_plain(const uint32_t* stage, int lane, __amdgpu_buffer_rsrc_t rs,
                                                uint32_t row_bytes) {
  using RS = RowSplit<T>;
  const int h = lane / RS::LPR, P = lane % RS::LPR;  // row within the instruction, pair
  if (P >= RS::NP) return;
  const uint32_t* src = stage + P * kPairPitch + 2 * h;
  const uint32_t voff = (uint32_t)P * 8u + (uint32_t)h * row_bytes;
#pragma unroll
  for (int r = 0; r < 64; r += RS::RPI) {
    const v2u d = *reinterpret_cast<const v2u*>(src + 2 * r);
    __builtin_amdgcn_raw_buffer_store_b64(convert_pair<G, DT>(d), rs, voff, (uint32_t)r * row_bytes, 0);
  }
}

// Any chunk: row r emits the positions of this chunk inside its own
// [ebeg, vend); f64 pairs start at positions of the same parity as ebeg.
template <class G, int DT, int T, int ES = 4>
__device__ __forceinline__ void emit_general(const uint32_t* stage, int lane, uint32_t lo, uint64_t q,
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
      const v2u d = *reinterpret_cast<const v2u*>(stage + lane * kPairPitch + 2 * r);
      if constexpr (DT != F64) {
        if (v0 >= rb && v0 < re) {
          if constexpr (DT == U32)
            *reinterpret_cast<gu32*>(rq + (uint64_t)ES * v0) = d.x;
          else
            *reinterpret_cast<gf32*>(rq + (uint64_t)ES * v0) = cvt32<G, DT>(d.x);
        }
        if (v0 + 1u >= rb && v0 + 1u < re) {
          if constexpr (DT == U32)
            *reinterpret_cast<gu32*>(rq + (uint64_t)ES * (v0 + 1u)) = d.y;
          else
            *reinterpret_cast<gf32*>(rq + (uint64_t)ES * (v0 + 1u)) = cvt32<G, DT>(d.y);
        }
      } else {
        if (((lo - rb) & 1u) == 0u) {
          if (v0 >= rb && v0 + 1u < re) *reinterpret_cast<gf64*>(rq + 4ull * v0) = to_f64<G::BITS>(d.x, d.y);
        } else {
          const uint32_t prev = lane == 0 ? stage[carry_at<T>() + r] : stage[(lane - 1) * kPairPitch + 2 * r + 1];
          if (v0 >= rb + 1u && v0 < re) *reinterpret_cast<gf64*>(rq + 4ull * (v0 - 1u)) = to_f64<G::BITS>(prev, d.x);
        }
      }
    }
  }
}

// Full chunk whose 64 rows are arbitrary output rows (stream table): same
// 8-byte-per-lane stores as the plain path; row r's element for virtual
// position v sits at q_r + 4 v (q from row r's lane).
template <class G, int DT, int T>
__device__ __forceinline__ void emit_full_rows(const uint32_t* stage, int lane, uint32_t lo, uint64_t q) {
  using RS = RowSplit<T>;
  const int h = lane / RS::LPR, P = lane % RS::LPR;
  const uint32_t* src = stage + P * kPairPitch + 2 * h;
#pragma unroll 8
  for (int r = 0; r < 64; r += RS::RPI) {
    const uint64_t q0 = rdlane64(q, r);
    const uint64_t rq = RS::RPI == 2 ? (h ? rdlane64(q, r + 1) : q0) : q0;
    if (P < RS::NP) {
      const v2u d = *reinterpret_cast<const v2u*>(src + 2 * r);
      reinterpret_cast<__attribute__((address_space(1))) v2u*>(rq + 4ull * lo)[P] = convert_pair<G, DT>(d);
    }
  }
}

// Full chunk of a four-way interleaved launch: streams 4g .. 4g+3 (lanes
// 4g .. 4g+3) share one row whose element v is a 16-byte vector of their four
// draws of position v, as the paper's kernels store the four subthreads of a
// register.  Per group, lane L writes the vector of position lo + L (+ 64),
// so one store instruction covers 1 KB of the group's row; q of lane 4g is
// the group's row address at position 0.
template <class G, int DT, int T>
__device__ __forceinline__ void emit_full_pack4(const uint32_t* stage, int lane, uint32_t lo, uint64_t q) {
  static_assert(DT != F64, "interleaved rows hold 4-byte elements");
#pragma unroll 4
  for (int gi = 0; gi < 16; ++gi) {
    const uint64_t base = rdlane64(q, 4 * gi) + 16ull * lo;
#pragma unroll
    for (int h = 0; h < (T + 63) / 64; ++h) {
      const int j = lane + 64 * h;
      if (j < T) {
        const uint32_t* src = stage + (j >> 1) * kPairPitch + 8 * gi + (j & 1);
        v4u o{src[0], src[2], src[4], src[6]};
        if constexpr (DT != U32)
          o = v4u{__float_as_uint(cvt32<G, DT>(o.x)), __float_as_uint(cvt32<G, DT>(o.y)),
                  __float_as_uint(cvt32<G, DT>(o.z)), __float_as_uint(cvt32<G, DT>(o.w))};
        *reinterpret_cast<__attribute__((address_space(1))) v4u*>(base + 16ull * (uint32_t)j) = o;
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
template <class G, int DT, bool PACK = false>
__device__ __forceinline__ void lane_loop(G& g, uint32_t* stage, int lane, uint32_t gbeg, uint32_t ebeg, uint32_t vend,
                                          uint64_t q, bool plain, uint64_t row_bytes) {
  constexpr uint32_t T = G::T;
  const bool has = vend > ebeg;
  const uint32_t maxb = wave_max(has ? ebeg : 0u);
  const uint32_t minb = wave_min(has ? ebeg : 0xFFFFFFFFu);
  const uint32_t minE = wave_min(has ? vend : 0xFFFFFFFFu);
  const uint32_t maxE = wave_max(has ? vend : 0u);
  const uint32_t ming = wave_min(has ? gbeg : 0xFFFFFFFFu);
  const uint32_t nlive = uni((uint32_t)__popcll(__ballot(has)));
  const uint32_t nalign = uni((uint32_t)__popcll(__ballot(has && (q & 7u) == 0u)));
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
  StageSink sink{stage + 2 * lane};
  for (uint32_t c = first; c < nchunks; ++c) {
    const uint32_t lo = c * T;
    if (lo >= maxb && lo + T <= minE) {
      g.template chunk<false>(lo, gbeg, vend, sink);
      wave_sync();
      if constexpr (PACK) {
        if (pack_full)
          emit_full_pack4<G, DT, T>(stage, lane, lo, q);
        else
          emit_general<G, DT, T, 16>(stage, lane, lo, q, ebeg, vend);
      } else if (plain) {
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            wave_base + 4ull * (uint64_t)(lo - minb), (short)0, (int)(63u * (uint32_t)row_bytes + 4u * T),
            0x00020000);
        emit_full_plain<G, DT, T>(stage, lane, rs, (uint32_t)row_bytes);
      } else if (even) {
        emit_full_rows<G, DT, T>(stage, lane, lo, q);
      } else {
        emit_general<G, DT, T>(stage, lane, lo, q, ebeg, vend);
      }
    } else {
      g.template chunk<true>(lo, gbeg, vend, sink);
      wave_sync();
      emit_general<G, DT, T, PACK ? 16 : 4>(stage, lane, lo, q, ebeg, vend);
    }
    wave_sync();
    if constexpr (DT == F64) {  // keep each lane's last draw for a pair that straddles chunks
      stage[carry_at<T>() + lane] = stage[(T / 2 - 1) * kPairPitch + 2 * lane + 1];
      wave_sync();
    }
  }
}

// ============================================================ lane kernels
// PACK: streams interleaved four by four (element v of stream s at
// ((s / 4) row_elems + elem_off + v) 16 + (s % 4) 4 bytes); 4-byte dtypes only.
template <class G, int DT, bool PACK = false>
__global__ __launch_bounds__(256) void k_lane_generate(uint32_t* __restrict__ state, uint64_t n, uint32_t draws,
                                                       uint32_t p, void* __restrict__ out, uint64_t row_elems,
                                                       uint64_t elem_off) {
  constexpr uint32_t T = G::T;
  __shared__ __attribute__((aligned(16))) uint32_t stage_all[4][stage_words<T>()];
  const int lane = threadIdx.x & 63;
  uint32_t* stage = stage_all[threadIdx.x >> 6];
  const uint64_t si = (uint64_t)blockIdx.x * 256u + threadIdx.x;
  G g;
  if constexpr (requires { g.p; }) g.p = p;
  uint32_t vbeg = 0;
  const bool live = si < n;
  if (live)
    g.load(state, n, si, vbeg);
  else
    g.zero();
  const uint32_t vend = live ? vbeg + draws : vbeg;
  constexpr uint64_t es = DT == F64 ? 8 : 4;
  // element of position v at q + 4 v, or q + 16 v when PACK (element 0 is position vbeg)
  uint64_t q = 0;
  if (live) {
    if constexpr (PACK)
      q = reinterpret_cast<uint64_t>(out) + ((si >> 2) * row_elems + elem_off) * 16ull + (si & 3u) * 4ull - 16ull * vbeg;
    else
      q = reinterpret_cast<uint64_t>(out) + (si * row_elems + elem_off) * es - 4ull * vbeg;
  }
  lane_loop<G, DT, PACK>(g, stage, lane, vbeg, vbeg, vend, q, !PACK, row_elems * es);
  if (live) g.store(state, n, si, vbeg, vend);
}

// Plain generation with the RANLUX lag table in HBM or in LDS (see
// RanluxMem); otherwise the same as k_lane_generate.
template <int WHERE, int DT>
__global__ __launch_bounds__(256) void k_ranlux_mem(uint32_t* __restrict__ state, uint64_t n, uint32_t draws,
                                                    uint32_t p, void* __restrict__ out, uint64_t row_elems,
                                                    uint64_t elem_off) {
  using G = RanluxMem<96, WHERE>;
  constexpr uint32_t T = G::T;
  __shared__ __attribute__((aligned(16))) uint32_t stage_all[4][stage_words<T>()];
  __shared__ uint32_t lag_all[4][24 * 64];
  const int lane = threadIdx.x & 63;
  uint32_t* stage = stage_all[threadIdx.x >> 6];
  const uint64_t si = (uint64_t)blockIdx.x * 256u + threadIdx.x;
  G g;
  g.zero();
  g.p = p;
  g.bind(lag_all[threadIdx.x >> 6], lane);
  uint32_t vbeg = 0;
  const bool live = si < n;
  if (live) g.load(state, n, si, vbeg);
  const uint32_t vend = live ? vbeg + draws : vbeg;
  constexpr uint64_t es = DT == F64 ? 8 : 4;
  const uint64_t q = live ? reinterpret_cast<uint64_t>(out) + (si * row_elems + elem_off) * es - 4ull * vbeg : 0;
  lane_loop<G, DT>(g, stage, lane, vbeg, vbeg, vend, q, true, row_elems * es);
  if (live) g.store(state, n, si, vbeg, vend);
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
template <class G, int DT>
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
    // pending skip by starting at local position 24.
    const uint32_t off = j == 0 ? 0u : (requires { g.p; } ? j * S - 24u : j * S);
    gbeg -= off;
    ebeg -= off;
    vend -= off;
    q += 4ull * off;
    wst = rw.wstate;
    wsn = rw.wsn;
    wsi = rw.wsi;
  } else {
    g.zero();
  }
  if constexpr (requires { g.retarget(wst, wsn, wsi); }) g.retarget(last ? wst : nullptr, wsn, wsi);
  wave_sync();
  lane_loop<G, DT>(g, stage, lane, gbeg, ebeg, vend, q, false, 0);
  if (live && last) g.store(wst, wsn, wsi, gbeg, vend);
}

// RANLUX in-kernel consumer with every stream cut into K <= 64 segments: one
// wavefront per stream, lane j working on segment j, positions [j S, (j+1) S)
// of the stream's axis (the first from k, the last to k + draws).  Segments
// j > 0 start from the state jumped ahead from the snapshot `snap` (taken
// before the launch) and run in segment-local coordinates (the pending skip
// at local position 24); the last one writes the final state.  The wavefront
// then adds up its lanes' exact sums and histogram columns, so the results
// are those of one pass over the whole stream.  A few thousand streams thus
// fill the chip instead of a few dozen wavefronts.
constexpr int kFusedSplitT = 144;

template <int P>
__global__ __launch_bounds__(256) void k_lux_fused_split(uint32_t* __restrict__ state, const uint32_t* __restrict__ snap,
                                                         uint64_t n, uint32_t draws, uint32_t p, uint32_t S, uint32_t K,
                                                         const uint32_t* __restrict__ jump,
                                                         const uint32_t* __restrict__ aux, uint64_t* __restrict__ sum,
                                                         uint32_t* __restrict__ hist, int accumulate) {
  __shared__ uint32_t hist_all[4][64 * kPitch];
  using G = Ranlux<kFusedSplitT, P>;
  constexpr uint32_t T = G::T;
  const int lane = threadIdx.x & 63;
  uint32_t* hbase = hist_all[threadIdx.x >> 6];
  uint32_t* hcol = hbase + lane;
#pragma unroll
  for (int b = 0; b < 64; ++b) hcol[b * kPitch] = 0;
  const uint64_t si = (uint64_t)blockIdx.x * 4u + (threadIdx.x >> 6);  // this wavefront's stream
  if (si >= n) return;  // whole wavefront; no block-wide barrier is used
  const uint32_t j = (uint32_t)lane;
  const bool live = j < K, last = j + 1u == K;
  G g;
  g.p = p;
  uint32_t gbeg = 0, vend = 0;
  if (live) {
    uint32_t k0 = 0;
    if (j == 0) {
      g.load(snap, n, si, k0);
      gbeg = k0;
    } else {
      k0 = g.load_jumped(snap, n, si, jump + (j - 1u) * 18u, aux, nullptr);
      gbeg = j * S;
    }
    vend = last ? k0 + draws : (j + 1u) * S;
    const uint32_t off = j == 0 ? 0u : j * S - 24u;  // a multiple of 24: block phases unchanged
    gbeg -= off;
    vend -= off;
  } else {
    g.zero();
  }
  const bool has = vend > gbeg;
  const uint32_t maxb = wave_max(has ? gbeg : 0u);
  const uint32_t minE = wave_min(has ? vend : 0xFFFFFFFFu);
  const uint32_t maxE = wave_max(has ? vend : 0u);
  const uint32_t nchunks = (maxE + T - 1) / T;
  uint64_t total = 0;
  FusedSink<G::BITS> sink{0u, hcol};
  for (uint32_t c = 0; c < nchunks; ++c) {
    const uint32_t lo = c * T;
    sink.acc = 0;
    if (lo >= maxb && lo + T <= minE)
      g.template chunk<false>(lo, gbeg, vend, sink);
    else
      g.template chunk<true>(lo, gbeg, vend, sink);
    total += sink.acc;
  }
  wave_sync();
  for (int o = 32; o > 0; o >>= 1) total += (uint64_t)__shfl_xor((unsigned long long)total, o);
  // bin `lane` summed over the columns of the K live lanes (lanes past K ran
  // the full chunks too, unpredicated, on a zero state)
  uint32_t hb = 0;
  for (uint32_t l = 0; l < K; ++l) hb += hbase[lane * kPitch + l];
  if (lane == 0) sum[si] = (accumulate ? sum[si] : 0ull) + total;
  hist[si * 64u + lane] = (accumulate ? hist[si * 64u + lane] : 0u) + hb;
  if (live && last) g.store(state, n, si, gbeg, vend);
}

template <class G>
__global__ __launch_bounds__(256) void k_lane_fused(uint32_t* __restrict__ state, uint64_t n, uint32_t draws,
                                                    uint32_t p, uint64_t* __restrict__ sum,
                                                    uint32_t* __restrict__ hist, int accumulate) {
  __shared__ uint32_t hist_all[4][64 * kPitch];
  const int lane = threadIdx.x & 63;
  uint32_t* hcol = hist_all[threadIdx.x >> 6] + lane;
#pragma unroll
  for (int b = 0; b < 64; ++b) hcol[b * kPitch] = 0;
  const uint64_t si = (uint64_t)blockIdx.x * 256u + threadIdx.x;
  G g;
  if constexpr (requires { g.p; }) g.p = p;
  uint32_t vbeg = 0;
  const bool live = si < n;
  if (live)
    g.load(state, n, si, vbeg);
  else
    g.zero();
  const uint32_t vend = live ? vbeg + draws : vbeg;
  constexpr uint32_t T = G::T;
  const bool has = vend > vbeg;
  const uint32_t maxb = wave_max(has ? vbeg : 0u);
  const uint32_t minE = wave_min(has ? vend : 0xFFFFFFFFu);
  const uint32_t maxE = wave_max(has ? vend : 0u);
  const uint32_t nchunks = (maxE + T - 1) / T;
  uint64_t total = 0;
  FusedSink<G::BITS> sink{0u, hcol};
  for (uint32_t c = 0; c < nchunks; ++c) {
    const uint32_t lo = c * T;
    sink.acc = 0;
    if (lo >= maxb && lo + T <= minE)
      g.template chunk<false>(lo, vbeg, vend, sink);
    else
      g.template chunk<true>(lo, vbeg, vend, sink);
    total += sink.acc;
  }
  wave_sync();
  if (live) {
    g.store(state, n, si, vbeg, vend);
    sum[si] = (accumulate ? sum[si] : 0ull) + total;
    uint32_t* hp = hist + si * 64u;
#pragma unroll
    for (int b = 0; b < 64; ++b) hp[b] = (accumulate ? hp[b] : 0u) + hcol[b * kPitch];
  }
}

// ============================================================ MT19937
constexpr uint32_t kMtUpper = 0x80000000u, kMtLower = 0x7FFFFFFFu, kMtA = 0x9908B0DFu;

__device__ __forceinline__ uint32_t mt_temper(uint32_t t) {
  t ^= t >> 11;
  t ^= (t << 7) & 0x9D2C5680u;
  t ^= (t << 15) & 0xEFC60000u;
  t ^= t >> 18;
  return t;
}

// Cooperative block twist of one stream by one wavefront: round r updates
// words 64r .. 64r+63 in place.  All reads of a round happen before its
// writes; word i >= 227 reads the new word i - 227 written >= 3 rounds before.
__device__ __forceinline__ void mt_twist(uint32_t* mt, int lane) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const int i = r * 64 + lane;
    const bool act = i < 624;
    uint32_t a = 0, b = 0, x = 0;
    if (act) {
      a = mt[i];
      b = mt[i + 1 == 624 ? 0 : i + 1];
      x = mt[i + 397 >= 624 ? i - 227 : i + 397];
    }
    wave_sync();
    if (act) {
      const uint32_t y = (a & kMtUpper) | (b & kMtLower);
      mt[i] = x ^ (y >> 1) ^ ((y & 1u) ? kMtA : 0u);
    }
    wave_sync();
  }
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

template <int DT>
__device__ __forceinline__ void mt_emit(const uint32_t* st, int lane, uint32_t done, uint32_t m, uint64_t outp) {
  if constexpr (DT != F64) {
    for (uint32_t j = lane; j < m; j += 64) {
      const uint32_t u = st[1 + j];
      if constexpr (DT == U32)
        reinterpret_cast<gu32*>(outp)[done + j] = u;
      else
        reinterpret_cast<gf32*>(outp)[done + j] = mt_f32<DT>(u);
    }
  } else {
    // pairs (2e, 2e+1) of the launch's draws whose second draw is in this block
    const uint32_t first = (done & 1u) ? done : done + 1u;
    for (uint32_t v2 = first + 2u * lane; v2 < done + m; v2 += 128u) {
      const uint32_t s2 = v2 - done + 1u;
      reinterpret_cast<gf64*>(outp)[v2 >> 1] = to_f64<32>(st[s2 - 1u], st[s2]);
    }
  }
}

// One stream of MT19937 by one wavefront: load the table from `src` into
// LDS at position pos0 (skipping `skip` draws of a fresh block when pos0 is
// 624), produce `draws` draws into the output row `outp` (address of element
// 0), and store the table to `sdst` unless it is null.  Used by the plain
// kernel and by the stream-table kernel.
template <int DT>
__device__ __forceinline__ void mt_body(uint32_t* mt, uint32_t* st, int lane, const uint32_t* src, uint32_t pos0,
                                        uint32_t skip, uint32_t draws, uint64_t outp, uint32_t* sdst) {
  constexpr uint64_t es = DT == F64 ? 8 : 4;
  constexpr uint32_t per = DT == F64 ? 2 : 1;
  for (int i = lane; i < 624; i += 64) mt[i] = src[i];
  uint32_t pos = pos0;
  wave_sync();
  if (skip) {
    mt_twist(mt, lane);
    pos = skip;
  }
  uint32_t done = 0;
  while (done < draws) {
    if (pos >= 624u) {
      mt_twist(mt, lane);
      pos = 0;
    }
    const uint32_t m = min(624u - pos, draws - done);
    // byte address of the block's first output; u32/f32 draws and f64 pairs
    // both take 4 bytes per draw, so draw w of the block lands at dst + 4 w
    const uint64_t dst = outp + (uint64_t)(done / per) * es;
    if (pos == 0u && m == 624u && (dst & 15u) == 0u && (DT != F64 || (done & 1u) == 0u)) {
      // whole block, 16-byte aligned: four consecutive words per lane
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const int w0 = q * 256 + 4 * lane;
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
          *reinterpret_cast<__attribute__((address_space(1))) v4u*>(dst + 4ull * (uint64_t)w0) = o;
        }
      }
      if constexpr (DT == F64) {
        if (lane == 0) st[0] = mt_temper(mt[623]);
      }
    } else {
      for (uint32_t j = lane; j < m; j += 64) st[1 + j] = mt_temper(mt[pos + j]);
      wave_sync();
      mt_emit<DT>(st, lane, done, m, outp);
      wave_sync();
      if constexpr (DT == F64) {
        if (lane == 0) st[0] = st[m];
      }
    }
    wave_sync();
    pos += m;
    done += m;
  }
  if (sdst) {
    for (int i = lane; i < 624; i += 64) sdst[i] = mt[i];
    if (lane == 0) sdst[624] = pos;
  }
  wave_sync();
}

template <int DT>
__global__ __launch_bounds__(256) void k_mt_generate(uint32_t* __restrict__ state, uint64_t n, uint32_t draws,
                                                     void* __restrict__ out, uint64_t row_elems, uint64_t elem_off) {
  __shared__ __attribute__((aligned(16))) uint32_t mt_all[4][624];
  __shared__ uint32_t stage_all[4][628];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t s = (uint64_t)blockIdx.x * 4u + w;
  if (s >= n) return;  // whole wavefront; no block-wide barrier is used
  constexpr uint64_t es = DT == F64 ? 8 : 4;
  uint32_t* sp = state + s * kMtStride;
  mt_body<DT>(mt_all[w], stage_all[w], lane, sp, uni(sp[624]), 0u, draws,
              reinterpret_cast<uint64_t>(out) + (s * row_elems + elem_off) * es, sp);
}

__global__ __launch_bounds__(256) void k_mt_fused(uint32_t* __restrict__ state, uint64_t n, uint32_t draws,
                                                  uint64_t* __restrict__ sum, uint32_t* __restrict__ hist,
                                                  int accumulate) {
  __shared__ uint32_t mt_all[4][624];
  __shared__ uint32_t h_all[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t s = (uint64_t)blockIdx.x * 4u + w;
  if (s >= n) return;
  uint32_t* mt = mt_all[w];
  uint32_t* h = h_all[w];
  uint32_t* sp = state + s * kMtStride;
  for (int i = lane; i < 624; i += 64) mt[i] = sp[i];
  h[lane] = 0;
  uint32_t pos = uni(sp[624]);
  wave_sync();
  uint32_t done = 0;
  uint64_t acc = 0;
  while (done < draws) {
    if (pos >= 624u) {
      mt_twist(mt, lane);
      pos = 0;
    }
    const uint32_t m = min(624u - pos, draws - done);
    uint32_t part = 0;
    for (uint32_t j = lane; j < m; j += 64) {
      const uint32_t k = mt_temper(mt[pos + j]) >> 8;
      part += k;
      __hip_atomic_fetch_add(&h[k >> 18], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    }
    acc += part;
    pos += m;
    done += m;
  }
  wave_sync();
  for (int o = 32; o > 0; o >>= 1) acc += (uint64_t)__shfl_xor((unsigned long long)acc, o);
  for (int i = lane; i < 624; i += 64) sp[i] = mt[i];
  if (lane == 0) {
    sp[624] = pos;
    sum[s] = (accumulate ? sum[s] : 0ull) + acc;
  }
  hist[s * 64u + lane] = (accumulate ? hist[s * 64u + lane] : 0u) + h[lane];
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

// Lane-per-stream tasks come in two kernels (classes).  GGL, XOR128, RANECU
// and RANLUX take 64- and 48-draw chunks (a 16.5 KB LDS stage per
// wavefront), so two blocks share a CU; the second wavefront per SIMD hides
// the latency of RANLUX's borrow chain.  RANMAR (97-word window plus a chunk
// of new values in registers, and a 97 x 97 jump) needs most of the register
// file, one wavefront per SIMD.
constexpr int kClassT[2] = {64, 64};

template <int CLASS>
__global__ __launch_bounds__(256) void k_table_lane(const TableTask* __restrict__ tasks, uint32_t ntasks,
                                                    const TableRow* __restrict__ rows,
                                                    const uint32_t* __restrict__ tails, uint32_t* counter,
                                                    const uint32_t* __restrict__ aux) {
  constexpr int TS = kClassT[CLASS];
  // RANMAR's jump also passes 97 values per lane through the stage (stride 64)
  constexpr int SW = CLASS == 1 && stage_words<TS>() < 97 * 64 ? 97 * 64 : stage_words<TS>();
  __shared__ __attribute__((aligned(16))) uint32_t stage_all[4][SW];
  const int lane = threadIdx.x & 63;
  uint32_t* stage = stage_all[threadIdx.x >> 6];
  for (uint32_t t = next_task(counter, lane); t < ntasks; t = next_task(counter, lane)) {
    const TableTask task = tasks[t];
    const uint32_t kind = uni(task.kind), dt = uni(task.dtype), p = uni(task.p);
#define PRNG_TASK(K, G)                                                        \
  case K * 4 + U32: lane_task<G, U32>(stage, lane, rows, tails, task, p, aux); break; \
  case K * 4 + F32: lane_task<G, F32>(stage, lane, rows, tails, task, p, aux); break; \
  case K * 4 + F64: lane_task<G, F64>(stage, lane, rows, tails, task, p, aux); break;
    if constexpr (CLASS == 0) {
      switch (kind * 4 + dt) {
        PRNG_TASK(GGL, Ggl<64>)
        PRNG_TASK(XOR128, Xor128<64>)
        PRNG_TASK(RANECU, Ranecu<64>)
        PRNG_TASK(RANLUX, Ranlux<48>)
        PRNG_TASK(DRAND48, Drand48<64>)
        PRNG_TASK(RANNYU, Rannyu<64>)
        default:
          break;
      }
    } else {
      switch (kind * 4 + dt) {
        PRNG_TASK(RANMAR, Ranmar<64>)
        default:
          break;
      }
    }
#undef PRNG_TASK
    wave_sync();
  }
}

// One task = one MT19937 row or segment of a row.  A row starts at position
// k0 (the stream's block position, 0..624; position 624 m + w is word w of
// the m-th block after the current one).  Segment j > 0 of a row cut at
// seg_len S (a multiple of 624) starts at position j S, from the window of
// the block before it that k_table_mt_jump built; with fp64 output a boundary
// that would split a pair of draws moves one draw later.
__global__ __launch_bounds__(256) void k_table_mt(const TableTask* __restrict__ tasks, uint32_t ntasks,
                                                  const TableRow* __restrict__ rows, uint32_t* counter) {
  __shared__ __attribute__((aligned(16))) uint32_t mt_all[4][624];
  __shared__ uint32_t stage_all[4][628];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (uint32_t t = next_task(counter, lane); t < ntasks; t = next_task(counter, lane)) {
    const TableRow& rw = rows[tasks[t].row0];
    const uint32_t dt = uni(tasks[t].dtype);
    const uint32_t draws = uni(rw.draws), S = uni(rw.seg_len);
    const uint32_t j = uni((uint32_t)tasks[t].g0), last = j + 1u == uni(rw.nseg) ? 1u : 0u;
    const uint32_t* snap = rw.state + rw.si * kMtStride;
    const uint32_t k0 = uni(snap[624]);
    uint32_t beg = k0, end = k0 + draws;
    if (S) {
      const uint32_t par = dt == F64 ? 1u : 0u;
      if (j) beg = j * S + (par & ((j * S - k0) & 1u));
      if (!last) end = (j + 1u) * S + (par & (((j + 1u) * S - k0) & 1u));
    }
    const uint32_t* src = j ? rw.jstate + (j - 1u) * kMtStride : snap;
    const uint32_t pos0 = j ? 624u : k0, skip = j ? beg - j * S : 0u;
    uint32_t* dst = last ? rw.wstate + rw.wsi * kMtStride : nullptr;
    const uint32_t per = dt == F64 ? 2u : 1u;
    const uint64_t outp = reinterpret_cast<uint64_t>(rw.out) + (uint64_t)((beg - k0) / per) * (4ull * per);
    if (dt == U32)
      mt_body<U32>(mt_all[w], stage_all[w], lane, src, pos0, skip, end - beg, outp, dst);
    else if (dt == F32)
      mt_body<F32>(mt_all[w], stage_all[w], lane, src, pos0, skip, end - beg, outp, dst);
    else
      mt_body<F64>(mt_all[w], stage_all[w], lane, src, pos0, skip, end - beg, outp, dst);
  }
}

// Jump-ahead of MT19937 segment starts, one block per segment.  From the
// row's starting window x_0 .. x_623 (the current block), the block extends
// the raw sequence x_n = x_{n-227} ^ twist(x_{n-624}, x_{n-623}) in LDS (227
// words at a time, each chunk reading only earlier chunks), then forms the
// window J words ahead as word k = XOR of x_{i+k} over the set coefficients
// i of x^J mod the characteristic polynomial (the segment's jump data lists
// their exponents).  The low 31 bits of word 0 are not part of the state and
// come out arbitrary; the next twist reads only its top bit.
constexpr int kMtSeqWords = 624 + 19936;
constexpr int kJumpThreads = 1024;  // four groups of 256 split the exponents

__global__ __launch_bounds__(kJumpThreads) void k_table_mt_jump(const uint32_t* __restrict__ list, uint32_t n,
                                                                const TableRow* __restrict__ rows) {
  __shared__ uint32_t seq[kMtSeqWords];
  __shared__ uint32_t part[3][624];  // partial windows of groups 1..3
  const int tid = threadIdx.x;
  const int grp = (int)uni((uint32_t)(tid >> 8)), t = tid & 255;  // a group is whole wavefronts
  // thread t of a group owns words 2t and 2t + 1 (one two-word LDS read per
  // exponent) and, for t < 56, words 512 + 2t and 513 + 2t
  const bool hi = t < 56;
  for (uint32_t r = blockIdx.x; r < n; r += gridDim.x) {
    const TableRow& rw = rows[list[2 * r]];
    const uint32_t j = list[2 * r + 1];  // >= 1
    const uint32_t* src = rw.state + rw.si * kMtStride;
    uint32_t* dst = rw.jstate + (j - 1u) * kMtStride;
    for (int i = tid; i < 624; i += kJumpThreads) seq[i] = src[i];
    __syncthreads();
    for (int n0 = 624; n0 < kMtSeqWords; n0 += 227) {
      const int x = n0 + tid;
      if (tid < 227 && x < kMtSeqWords) {
        const uint32_t y = (seq[x - 624] & kMtUpper) | (seq[x - 623] & kMtLower);
        seq[x] = seq[x - 227] ^ (y >> 1) ^ ((y & 1u) ? kMtA : 0u);
      }
      __syncthreads();
    }
    // group g takes exponents 8 (4m + g) .. 8 (4m + g) + 7; the four words
    // holding the next eight are fetched one round ahead
    const uint32_t* jd = rw.jump + (j - 1u) * rw.jstride;
    const uint32_t nbits = min(uni(jd[0]), 19937u);
    const uint32_t nfull = nbits / 8u;  // complete groups of eight
    uint32_t a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    uint32_t gq = (uint32_t)grp;
    uint32_t w0 = 0, w1 = 0, w2 = 0, w3 = 0;
    // (vector loads: their wait is at the next round's first use, and it
    // does not hold up the LDS reads in between)
    if (gq < nfull) {
      w0 = jd[1 + 4 * gq];
      w1 = jd[2 + 4 * gq];
      w2 = jd[3 + 4 * gq];
      w3 = jd[4 + 4 * gq];
    }
    for (; gq < nfull; gq += 4u) {
      const uint32_t u0 = uni(w0), u1 = uni(w1), u2 = uni(w2), u3 = uni(w3);
      const int ix[8] = {min((int)(u0 & 0xFFFFu), 19936), min((int)(u0 >> 16), 19936),
                         min((int)(u1 & 0xFFFFu), 19936), min((int)(u1 >> 16), 19936),
                         min((int)(u2 & 0xFFFFu), 19936), min((int)(u2 >> 16), 19936),
                         min((int)(u3 & 0xFFFFu), 19936), min((int)(u3 >> 16), 19936)};
      if (gq + 4u < nfull) {
        const uint32_t* nx = jd + 1 + 4 * (gq + 4u);
        w0 = nx[0];
        w1 = nx[1];
        w2 = nx[2];
        w3 = nx[3];
      }
      uint32_t v0[8], v1[8];
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const uint32_t* p = seq + ix[b] + 2 * t;
        v0[b] = p[0];
        v1[b] = p[1];
      }
      if (hi) {
        uint32_t v2[8], v3[8];
#pragma unroll
        for (int b = 0; b < 8; ++b) {
          const uint32_t* p = seq + ix[b] + 2 * t + 512;
          v2[b] = p[0];
          v3[b] = p[1];
        }
#pragma unroll
        for (int b = 0; b < 8; ++b) {
          a2 ^= v2[b];
          a3 ^= v3[b];
        }
      }
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        a0 ^= v0[b];
        a1 ^= v1[b];
      }
    }
    if (grp == 0) {  // the last nbits % 8 exponents
      for (uint32_t q = nfull * 8u; q < nbits; ++q) {
        const int i = min((int)((uni(jd[1 + (q >> 1)]) >> (16u * (q & 1u))) & 0xFFFFu), 19936);
        const uint32_t* p = seq + i + 2 * t;
        a0 ^= p[0];
        a1 ^= p[1];
        if (hi) {
          a2 ^= p[512];
          a3 ^= p[513];
        }
      }
    }
    if (grp > 0) {
      uint32_t* pp = part[grp - 1];
      pp[2 * t] = a0;
      pp[2 * t + 1] = a1;
      if (hi) {
        pp[512 + 2 * t] = a2;
        pp[513 + 2 * t] = a3;
      }
    }
    __syncthreads();
    if (grp == 0) {
#pragma unroll
      for (int g = 0; g < 3; ++g) {
        a0 ^= part[g][2 * t];
        a1 ^= part[g][2 * t + 1];
        if (hi) {
          a2 ^= part[g][512 + 2 * t];
          a3 ^= part[g][513 + 2 * t];
        }
      }
      dst[2 * t] = a0;
      dst[2 * t + 1] = a1;
      if (hi) {
        dst[512 + 2 * t] = a2;
        dst[513 + 2 * t] = a3;
      }
      if (t == 0) dst[624] = 624u;
    }
    __syncthreads();  // seq and part are rebuilt for the next segment
  }
}

// Copies the starting states of split streams (one thread per word).
__global__ void k_table_snapshot(const SnapRow* __restrict__ rows, uint32_t n, uint32_t max_words) {
  const uint64_t total = (uint64_t)n * max_words;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t r = (uint32_t)(t / max_words), w = (uint32_t)(t % max_words);
    const SnapRow& sr = rows[r];
    if (w >= sr.words) continue;
    if (sr.aos)
      sr.dst[sr.di * kMtStride + w] = sr.src[sr.si * kMtStride + w];
    else
      sr.dst[w * sr.dn + sr.di] = sr.src[w * sr.sn + sr.si];
  }
}

// Clears the task counters in-stream (a kernel rather than a memset so that
// the clear is an ordinary node when the run is captured into a graph).
__global__ void k_table_reset(uint32_t* counters, int n) {
  if ((int)threadIdx.x < n) counters[threadIdx.x] = 0u;
}

// ============================================================ init kernels
// Seed tuples arrive as uint64 words, stream by stream.
__global__ void k_init_copy(uint32_t* __restrict__ st, uint64_t n, const uint64_t* __restrict__ seeds, int words) {
  const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  for (int j = 0; j < words; ++j) st[j * n + s] = (uint32_t)seeds[s * words + j];
}

// 48-bit LCGs: the seed is X_0 (low word, high word).
__global__ void k_init_lcg48(uint32_t* __restrict__ st, uint64_t n, const uint64_t* __restrict__ seeds) {
  const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  st[s] = (uint32_t)seeds[s];
  st[n + s] = (uint32_t)(seeds[s] >> 32) & 0xFFFFu;
}

// RMARIN (James' initialiser of RANMAR; run once per instance on the GPU,
// Section 3.5): the 24 bits of each of the 97 lags come, most significant
// first, from a 3-lag multiplicative sequence mod 179 and an LCG mod 169.
// Stored oldest lag first (the initialiser's u[97] down to u[1]), C_0 = 362436.
__global__ void k_init_ranmar(uint32_t* __restrict__ st, uint64_t n, const uint64_t* __restrict__ seeds) {
  const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const uint32_t ij = (uint32_t)seeds[2 * s], kl = (uint32_t)seeds[2 * s + 1];
  uint32_t i = ij / 177u + 2u, j = ij % 177u + 2u, k = kl / 169u + 1u, l = kl % 169u;
  for (uint32_t ii = 1; ii <= 97; ++ii) {
    uint32_t v = 0;
    for (int b = 23; b >= 0; --b) {
      const uint32_t m = ((i * j) % 179u) * k % 179u;
      i = j;
      j = k;
      k = m;
      l = (53u * l + 1u) % 169u;
      v |= (((l * m) & 63u) >= 32u ? 1u : 0u) << b;
    }
    st[(97u - ii) * n + s] = v;
  }
  st[97 * n + s] = 362436u;
}

// RANLUX lag table: 24 successive values of the MLCG (40014, 2^31-85) from v,
// each mod 2^24, oldest first; borrow = (newest lag == 0); k = 0.
__global__ void k_init_ranlux(uint32_t* __restrict__ st, uint64_t n, const uint64_t* __restrict__ seeds) {
  const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  uint32_t x = (uint32_t)seeds[s];
  uint32_t last = 0;
  for (int t = 0; t < 24; ++t) {
    x = mul_mod_2p31<40014u, 85u>(x);
    last = x & 0xFFFFFFu;
    st[t * n + s] = last;
  }
  st[24 * n + s] = last == 0 ? 1u : 0u;
  st[25 * n + s] = 0u;
}

// MT19937 init_genrand: mt[i] = 1812433253 (mt[i-1] ^ (mt[i-1] >> 30)) + i.
__global__ void k_init_mt(uint32_t* __restrict__ st, uint64_t n, const uint64_t* __restrict__ seeds) {
  const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  uint32_t* sp = st + s * kMtStride;
  uint32_t x = (uint32_t)seeds[s];
  sp[0] = x;
  for (uint32_t i = 1; i < 624; ++i) {
    x = 1812433253u * (x ^ (x >> 30)) + i;
    sp[i] = x;
  }
  sp[624] = 624u;
}

template <class G>
hipError_t launch_lane_pack(int dtype, uint32_t p, uint32_t* st, uint64_t n, uint64_t draws, void* out,
                            uint64_t row_elems, uint64_t off, hipStream_t s) {
  const dim3 grid((unsigned)((n + 255) / 256)), block(256);
  const uint32_t d = (uint32_t)draws;
  switch (dtype) {
    case U32:
      hipLaunchKernelGGL((k_lane_generate<G, U32, true>), grid, block, 0, s, st, n, d, p, out, row_elems, off);
      break;
    case F32:
      hipLaunchKernelGGL((k_lane_generate<G, F32, true>), grid, block, 0, s, st, n, d, p, out, row_elems, off);
      break;
    case F32P:
      if constexpr (requires { G::paper_f32(0u); }) {
        hipLaunchKernelGGL((k_lane_generate<G, F32P, true>), grid, block, 0, s, st, n, d, p, out, row_elems, off);
        break;
      }
      return hipErrorInvalidValue;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class G>
hipError_t launch_lane_gen(int dtype, uint32_t p, uint32_t* st, uint64_t n, uint64_t draws, void* out,
                           uint64_t row_elems, uint64_t off, hipStream_t s) {
  const dim3 grid((unsigned)((n + 255) / 256)), block(256);
  const uint32_t d = (uint32_t)draws;
  switch (dtype) {
    case U32:
      hipLaunchKernelGGL((k_lane_generate<G, U32>), grid, block, 0, s, st, n, d, p, out, row_elems, off);
      break;
    case F32:
      hipLaunchKernelGGL((k_lane_generate<G, F32>), grid, block, 0, s, st, n, d, p, out, row_elems, off);
      break;
    case F64:
      hipLaunchKernelGGL((k_lane_generate<G, F64>), grid, block, 0, s, st, n, d, p, out, row_elems, off);
      break;
    case F32P:
      if constexpr (requires { G::paper_f32(0u); }) {
        hipLaunchKernelGGL((k_lane_generate<G, F32P>), grid, block, 0, s, st, n, d, p, out, row_elems, off);
        break;
      }
      return hipErrorInvalidValue;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class G>
hipError_t launch_lane_fused(uint32_t p, uint32_t* st, uint64_t n, uint64_t draws, uint64_t* sum, uint32_t* hist,
                             bool acc, hipStream_t s) {
  const dim3 grid((unsigned)((n + 255) / 256)), block(256);
  hipLaunchKernelGGL((k_lane_fused<G>), grid, block, 0, s, st, n, (uint32_t)draws, p, sum, hist, acc ? 1 : 0);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_init(int kind, uint32_t* state, uint64_t n, const uint64_t* d_seeds, hipStream_t s) {
  const dim3 grid((unsigned)((n + 255) / 256)), block(256);
  switch (kind) {
    case GGL:
    case XOR128:
    case RANECU:
      hipLaunchKernelGGL(k_init_copy, grid, block, 0, s, state, n, d_seeds, kSeedWords[kind]);
      break;
    case RANMAR:
      hipLaunchKernelGGL(k_init_ranmar, grid, block, 0, s, state, n, d_seeds);
      break;
    case RANLUX:
      hipLaunchKernelGGL(k_init_ranlux, grid, block, 0, s, state, n, d_seeds);
      break;
    case MT19937:
      hipLaunchKernelGGL(k_init_mt, grid, block, 0, s, state, n, d_seeds);
      break;
    case DRAND48:
    case RANNYU:
      hipLaunchKernelGGL(k_init_lcg48, grid, block, 0, s, state, n, d_seeds);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_generate(int kind, uint32_t p, uint32_t* st, uint64_t n, uint64_t draws, int dtype, void* out,
                           uint64_t row_elems, uint64_t off, hipStream_t s) {
  switch (kind) {
    case GGL:
      return launch_lane_gen<Ggl<>>(dtype, p, st, n, draws, out, row_elems, off, s);
    case XOR128:
      return launch_lane_gen<Xor128<>>(dtype, p, st, n, draws, out, row_elems, off, s);
    case RANECU:
      return launch_lane_gen<Ranecu<>>(dtype, p, st, n, draws, out, row_elems, off, s);
    case RANMAR:
      return launch_lane_gen<Ranmar<>>(dtype, p, st, n, draws, out, row_elems, off, s);
    case DRAND48:
      return launch_lane_gen<Drand48<>>(dtype, p, st, n, draws, out, row_elems, off, s);
    case RANNYU:
      return launch_lane_gen<Rannyu<>>(dtype, p, st, n, draws, out, row_elems, off, s);
    case RANLUX:  // the luxury levels get a compile-time skip; 96-draw chunks
      switch (p) {
        case 24:
          return launch_lane_gen<Ranlux<96, 24>>(dtype, p, st, n, draws, out, row_elems, off, s);
        case 48:
          return launch_lane_gen<Ranlux<96, 48>>(dtype, p, st, n, draws, out, row_elems, off, s);
        case 97:
          return launch_lane_gen<Ranlux<96, 97>>(dtype, p, st, n, draws, out, row_elems, off, s);
        case 223:
          return launch_lane_gen<Ranlux<96, 223>>(dtype, p, st, n, draws, out, row_elems, off, s);
        case 389:
          return launch_lane_gen<Ranlux<96, 389>>(dtype, p, st, n, draws, out, row_elems, off, s);
        case 120:  // the paper's planar levels discard whole multiples of 24
          return launch_lane_gen<Ranlux<96, 120>>(dtype, p, st, n, draws, out, row_elems, off, s);
        case 240:
          return launch_lane_gen<Ranlux<96, 240>>(dtype, p, st, n, draws, out, row_elems, off, s);
        case 408:
          return launch_lane_gen<Ranlux<96, 408>>(dtype, p, st, n, draws, out, row_elems, off, s);
        default:
          return launch_lane_gen<Ranlux<96>>(dtype, p, st, n, draws, out, row_elems, off, s);
      }
    case MT19937: {
      const dim3 grid((unsigned)((n + 3) / 4)), block(256);
      const uint32_t d = (uint32_t)draws;
      switch (dtype) {
        case U32:
          hipLaunchKernelGGL((k_mt_generate<U32>), grid, block, 0, s, st, n, d, out, row_elems, off);
          break;
        case F32:
          hipLaunchKernelGGL((k_mt_generate<F32>), grid, block, 0, s, st, n, d, out, row_elems, off);
          break;
        case F64:
          hipLaunchKernelGGL((k_mt_generate<F64>), grid, block, 0, s, st, n, d, out, row_elems, off);
          break;
        case F32P:
          hipLaunchKernelGGL((k_mt_generate<F32P>), grid, block, 0, s, st, n, d, out, row_elems, off);
          break;
        default:
          return hipErrorInvalidValue;
      }
      return hipGetLastError();
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_ranlux_variant(int where, uint32_t p, uint32_t* st, uint64_t n, uint64_t draws, int dtype,
                                 void* out, uint64_t row_elems, uint64_t off, hipStream_t s) {
  const dim3 grid((unsigned)((n + 255) / 256)), block(256);
  const uint32_t d = (uint32_t)draws;
#define PRNG_VARIANT(W)                                                                                   \
  switch (dtype) {                                                                                        \
    case U32:                                                                                             \
      hipLaunchKernelGGL((k_ranlux_mem<W, U32>), grid, block, 0, s, st, n, d, p, out, row_elems, off);    \
      break;                                                                                              \
    case F32:                                                                                             \
      hipLaunchKernelGGL((k_ranlux_mem<W, F32>), grid, block, 0, s, st, n, d, p, out, row_elems, off);    \
      break;                                                                                              \
    case F64:                                                                                             \
      hipLaunchKernelGGL((k_ranlux_mem<W, F64>), grid, block, 0, s, st, n, d, p, out, row_elems, off);    \
      break;                                                                                              \
    default:                                                                                              \
      return hipErrorInvalidValue;                                                                        \
  }
  if (where == kLagLds) {
    PRNG_VARIANT(kLagLds)
  } else if (where == kLagHbm) {
    PRNG_VARIANT(kLagHbm)
  } else {
    return hipErrorInvalidValue;
  }
#undef PRNG_VARIANT
  return hipGetLastError();
}

hipError_t launch_generate_packed(int kind, uint32_t p, uint32_t* st, uint64_t n, uint64_t draws, int dtype,
                                  void* out, uint64_t row_elems, uint64_t off, hipStream_t s) {
  switch (kind) {
    case GGL:
      return launch_lane_pack<Ggl<>>(dtype, p, st, n, draws, out, row_elems, off, s);
    case XOR128:
      return launch_lane_pack<Xor128<>>(dtype, p, st, n, draws, out, row_elems, off, s);
    case RANECU:
      return launch_lane_pack<Ranecu<>>(dtype, p, st, n, draws, out, row_elems, off, s);
    case RANMAR:
      return launch_lane_pack<Ranmar<>>(dtype, p, st, n, draws, out, row_elems, off, s);
    case RANLUX:
      return launch_lane_pack<Ranlux<96>>(dtype, p, st, n, draws, out, row_elems, off, s);
    case DRAND48:
      return launch_lane_pack<Drand48<>>(dtype, p, st, n, draws, out, row_elems, off, s);
    case RANNYU:
      return launch_lane_pack<Rannyu<>>(dtype, p, st, n, draws, out, row_elems, off, s);
  }
  return hipErrorInvalidValue;
}

template <int P>
hipError_t launch_lux_fused_split_p(uint32_t p, uint32_t* st, const uint32_t* snap, uint64_t n, uint64_t draws,
                                    uint32_t S, uint32_t K, const uint32_t* jump, const uint32_t* aux, uint64_t* sum,
                                    uint32_t* hist, bool acc, hipStream_t s) {
  const dim3 grid((unsigned)((n + 3) / 4)), block(256);
  hipLaunchKernelGGL((k_lux_fused_split<P>), grid, block, 0, s, st, snap, n, (uint32_t)draws, p, S, K, jump, aux, sum,
                     hist, acc ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_lux_fused_split(uint32_t p, uint32_t* st, const uint32_t* snap, uint64_t n, uint64_t draws,
                                  uint32_t S, uint32_t K, const uint32_t* jump, const uint32_t* aux, uint64_t* sum,
                                  uint32_t* hist, bool acc, hipStream_t s) {
  switch (p) {  // the luxury levels get a compile-time skip
    case 24:
      return launch_lux_fused_split_p<24>(p, st, snap, n, draws, S, K, jump, aux, sum, hist, acc, s);
    case 48:
      return launch_lux_fused_split_p<48>(p, st, snap, n, draws, S, K, jump, aux, sum, hist, acc, s);
    case 97:
      return launch_lux_fused_split_p<97>(p, st, snap, n, draws, S, K, jump, aux, sum, hist, acc, s);
    case 223:
      return launch_lux_fused_split_p<223>(p, st, snap, n, draws, S, K, jump, aux, sum, hist, acc, s);
    case 389:
      return launch_lux_fused_split_p<389>(p, st, snap, n, draws, S, K, jump, aux, sum, hist, acc, s);
    case 120:
      return launch_lux_fused_split_p<120>(p, st, snap, n, draws, S, K, jump, aux, sum, hist, acc, s);
    case 240:
      return launch_lux_fused_split_p<240>(p, st, snap, n, draws, S, K, jump, aux, sum, hist, acc, s);
    case 408:
      return launch_lux_fused_split_p<408>(p, st, snap, n, draws, S, K, jump, aux, sum, hist, acc, s);
    default:
      return launch_lux_fused_split_p<0>(p, st, snap, n, draws, S, K, jump, aux, sum, hist, acc, s);
  }
}

hipError_t launch_fused(int kind, uint32_t p, uint32_t* st, uint64_t n, uint64_t draws, uint64_t* sum,
                        uint32_t* hist, bool acc, hipStream_t s) {
  switch (kind) {
    case GGL:
      return launch_lane_fused<Ggl<>>(p, st, n, draws, sum, hist, acc, s);
    case XOR128:
      return launch_lane_fused<Xor128<>>(p, st, n, draws, sum, hist, acc, s);
    case RANECU:
      return launch_lane_fused<Ranecu<>>(p, st, n, draws, sum, hist, acc, s);
    case RANMAR:
      return launch_lane_fused<Ranmar<>>(p, st, n, draws, sum, hist, acc, s);
    case RANLUX:
      return launch_lane_fused<Ranlux<>>(p, st, n, draws, sum, hist, acc, s);
    case DRAND48:
      return launch_lane_fused<Drand48<>>(p, st, n, draws, sum, hist, acc, s);
    case RANNYU:
      return launch_lane_fused<Rannyu<>>(p, st, n, draws, sum, hist, acc, s);
    case MT19937: {
      const dim3 grid((unsigned)((n + 3) / 4)), block(256);
      hipLaunchKernelGGL(k_mt_fused, grid, block, 0, s, st, n, (uint32_t)draws, sum, hist, acc ? 1 : 0);
      return hipGetLastError();
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_table_reset(uint32_t* counters, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_table_reset, dim3(1), dim3(64), 0, s, counters, n);
  return hipGetLastError();
}

hipError_t launch_table_lane(int cls, const TableTask* tasks, uint32_t ntasks, const TableRow* rows,
                             const uint32_t* tails, uint32_t* counter, const uint32_t* aux, int grid, hipStream_t s) {
  if (cls == 0)
    hipLaunchKernelGGL((k_table_lane<0>), dim3(grid), dim3(256), 0, s, tasks, ntasks, rows, tails, counter, aux);
  else
    hipLaunchKernelGGL((k_table_lane<1>), dim3(grid), dim3(256), 0, s, tasks, ntasks, rows, tails, counter, aux);
  return hipGetLastError();
}

hipError_t launch_table_snapshot(const SnapRow* rows, uint32_t n, uint32_t max_words, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint64_t threads = (uint64_t)n * max_words;
  const unsigned grid = (unsigned)std::min<uint64_t>((threads + 255) / 256, 4096);
  hipLaunchKernelGGL(k_table_snapshot, dim3(grid), dim3(256), 0, s, rows, n, max_words);
  return hipGetLastError();
}

hipError_t launch_table_mt_jump(const uint32_t* list, uint32_t n, const TableRow* rows, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const unsigned grid = std::min<uint32_t>(n, 1024u);
  hipLaunchKernelGGL(k_table_mt_jump, dim3(grid), dim3(kJumpThreads), 0, s, list, n, rows);
  return hipGetLastError();
}

hipError_t launch_table_mt(const TableTask* tasks, uint32_t ntasks, const TableRow* rows, uint32_t* counter, int grid,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_table_mt, dim3(grid), dim3(256), 0, s, tasks, ntasks, rows, counter);
  return hipGetLastError();
}

}  // namespace prng
