// Plain bulk generation: leapfrog kernels (GGL, RANECU, DRAND48, RANNYU), lane-per-stream kernels
// (XOR128, RANMAR; and every lane kind for four-way interleaved output) and MT19937.
#include <array>

#include "device.h"

namespace prng {
namespace {

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

// XOR128 plain generation with every stream cut into K segments of S
// positions: block b works on segment j = b / nb of the 256 streams
// (b mod nb) of that range, nb = ceil(n / 256).  Every segment starts from
// the snapshot `snap` taken before the launch, segment j > 0 jumped j S
// positions ahead; the last segment writes the final state.  XOR128's draws
// carry no position structure, so segments run in the stream's own
// coordinates; S is even, so fp64 pairs never straddle a boundary.
template <int DT>
__global__ __launch_bounds__(256) void k_xor128_split(uint32_t* __restrict__ state, const uint32_t* __restrict__ snap,
                                                      uint64_t n, uint32_t draws, uint32_t S, uint32_t K,
                                                      const uint32_t* __restrict__ pow2, void* __restrict__ out,
                                                      uint64_t row_elems, uint64_t elem_off) {
  using G = Xor128<>;
  constexpr uint32_t T = G::T;
  __shared__ __attribute__((aligned(16))) uint32_t stage_all[4][stage_words<T>()];
  const int lane = threadIdx.x & 63;
  uint32_t* stage = stage_all[threadIdx.x >> 6];
  const uint32_t nb = (uint32_t)((n + 255) / 256);
  const uint32_t j = blockIdx.x / nb;
  const uint64_t si = (uint64_t)(blockIdx.x - j * nb) * 256u + threadIdx.x;
  const bool live = si < n;
  G g;
  const uint32_t beg = j * S, end = j + 1u == K ? draws : min((j + 1u) * S, draws);
  if (live) {
    if (j == 0) {
      uint32_t v0;
      g.load(snap, n, si, v0);
    } else {
      g.load_jumped_pow2(snap, n, si, beg, pow2);
    }
  } else {
    g.zero();
  }
  constexpr uint64_t es = DT == F64 ? 8 : 4;
  const uint64_t q = live ? reinterpret_cast<uint64_t>(out) + (si * row_elems + elem_off) * es : 0;
  lane_loop<G, DT>(g, stage, lane, beg, beg, live ? end : beg, q, true, row_elems * es);
  if (live && j + 1u == K) g.store(state, n, si, beg, end);
}

// One stream at a time per workgroup: its four wavefronts twist and store
// each block together, so that the chip writes few rows at a time, each in
// bursts.  A workgroup takes streams 2b and 2b + 1 and fetches the second
// one's table into registers before it generates the first, so that only
// the first table's load is waited for.
template <int DT>
__global__ __launch_bounds__(256) void k_mt_generate(uint32_t* __restrict__ state, uint64_t n, uint32_t draws,
                                                     void* __restrict__ out, uint64_t row_elems, uint64_t elem_off) {
  __shared__ __attribute__((aligned(16))) uint32_t mt[624];
  __shared__ __attribute__((aligned(16))) uint32_t stage[628];
  const int tid = (int)threadIdx.x;
  const uint64_t s0 = 2ull * blockIdx.x;
  if (s0 >= n) return;  // the whole workgroup
  const bool two = s0 + 1 < n;
  constexpr uint64_t es = DT == F64 ? 8 : 4;
  uint32_t* const sp0 = state + s0 * kMtStride;
  uint32_t* const sp1 = sp0 + kMtStride;
  uint32_t nxt[3] = {0u, 0u, 0u}, nxt_pos = 0u;
  if (two) {
#pragma unroll
    for (int q = 0; q < 3; ++q)
      if (tid + 256 * q < 624) nxt[q] = sp1[tid + 256 * q];
    nxt_pos = sp1[624];
  }
  mt_body<DT>(mt, stage, tid, sp0, uni(sp0[624]), 0u, draws,
              reinterpret_cast<uint64_t>(out) + (s0 * row_elems + elem_off) * es, sp0);
  if (!two) return;
#pragma unroll
  for (int q = 0; q < 3; ++q)
    if (tid + 256 * q < 624) mt[tid + 256 * q] = nxt[q];
  __syncthreads();
  mt_body<DT>(mt, stage, tid, nullptr, uni(nxt_pos), 0u, draws,
              reinterpret_cast<uint64_t>(out) + ((s0 + 1) * row_elems + elem_off) * es, sp1);
}

// ============================================================ leapfrog kernels
// Multiplicative and affine generators (GGL, RANECU, DRAND48, RANNYU): one
// wavefront per stream; lane l produces positions 4 l .. 4 l + 3 of every
// block of 256, so that each store instruction writes 256 consecutive
// elements of the row (1 KB for u32/f32, four per lane) with no LDS
// transpose, and the stream's row is written front to back.  Within its four
// positions a lane steps the recurrence; to its next four it leaps by a^253
// from the last (the affine map of 253 steps for the 48-bit LCGs), so every
// position still costs one multiplication.

constexpr uint64_t cpowmod(uint64_t a, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  a %= m;
  while (e) {
    if (e & 1) r = r * a % m;
    a = a * a % m;
    e >>= 1;
  }
  return r;
}

struct Affine48 {
  uint64_t a, c;
};
// J steps of X -> a X + c mod 2^48 as one affine map
constexpr Affine48 caffine_pow(uint64_t a, uint64_t c, uint64_t J) {
  constexpr uint64_t M = (1ull << 48) - 1;
  Affine48 r{1, 0}, b{a & M, c & M};
  while (J) {
    if (J & 1) r = Affine48{(b.a * r.a) & M, (b.a * r.c + b.c) & M};
    b = Affine48{(b.a * b.a) & M, (b.a * b.c + b.c) & M};
    J >>= 1;
  }
  return r;
}

constexpr uint32_t kLeapQuad = 4, kLeapBlock = 64 * kLeapQuad;

// a^(4 l + 1) mod m for the 64 lanes: each lane's first position in one multiplication
template <uint64_t A, uint64_t Mod>
struct LaneStart {
  static constexpr std::array<uint32_t, 64> table() {
    std::array<uint32_t, 64> t{};
    for (uint32_t l = 0; l < 64; ++l) t[l] = (uint32_t)cpowmod(A, kLeapQuad * l + 1, Mod);
    return t;
  }
  static constexpr std::array<uint32_t, 64> kPow = table();
};

// GGL: the output of position v is X_{v+1} = a^{v+1} X_0.
struct LeapGgl {
  static constexpr int BITS = 31;
  static constexpr bool kNtOut = false;
  static constexpr uint32_t A = 16807u, AL = (uint32_t)cpowmod(A, kLeapBlock - 3, 2147483647u);
  uint32_t x;  // X of the lane's first position in the current block
  __device__ void load(const uint32_t* st, uint64_t, uint64_t si) { x = st[si]; }
  // lane l: X_{4l+1}, the state of its first position
  __device__ void start(int lane) { x = mulmod_2p31<1u>(x, LaneStart<A, 2147483647u>::kPow[lane]); }
  // draws of the lane's four positions; leaves x at the last one
  __device__ __forceinline__ void quad(uint32_t* u) {
    u[0] = x;
#pragma unroll
    for (int j = 1; j < 4; ++j) {
      x = mul_mod_2p31<A, 1u>(x);
      u[j] = x;
    }
  }
  __device__ __forceinline__ void leap() { x = mulmod_2p31<1u>(x, AL); }
  // state after the position at offset j of the quad (x at the quad's first position)
  __device__ void store_at(uint32_t j, uint32_t* st, uint64_t, uint64_t si) const {
    uint32_t y = x;
    for (uint32_t i = 0; i < j; ++i) y = mul_mod_2p31<A, 1u>(y);
    st[si] = y;
  }
  static __device__ float paper_f32(uint32_t u) { return Ggl<>::paper_f32(u); }
  // the map of q steps, for the host (j0, j1), and its w-fold application
  static void q_map(uint64_t q, uint64_t& j0, uint64_t& j1) {
    j0 = cpowmod(A, q, 2147483647u);
    j1 = 0;
  }
  __device__ void advance_q(uint64_t j0, uint64_t, uint32_t w) {
    for (uint32_t i = 0; i < w; ++i) x = mulmod_2p31<1u>(x, (uint32_t)j0);
  }
};

// RANECU: both MLCGs leap; the draw combines the two states.
struct LeapRanecu {
  static constexpr int BITS = 31;
  static constexpr bool kNtOut = true;  // two MLCG steps per draw between the stores
  static constexpr uint32_t A1 = 40014u, A2 = 40692u;
  static constexpr uint32_t B1 = (uint32_t)cpowmod(A1, kLeapBlock - 3, 2147483563u),
                            B2 = (uint32_t)cpowmod(A2, kLeapBlock - 3, 2147483399u);
  uint32_t s1, s2;
  __device__ void load(const uint32_t* st, uint64_t sn, uint64_t si) {
    s1 = st[si];
    s2 = st[sn + si];
  }
  __device__ void start(int lane) {
    s1 = mulmod_2p31<85u>(s1, LaneStart<A1, 2147483563u>::kPow[lane]);
    s2 = mulmod_2p31<249u>(s2, LaneStart<A2, 2147483399u>::kPow[lane]);
  }
  static __device__ __forceinline__ uint32_t combine(uint32_t a, uint32_t b) {
    int32_t z = (int32_t)a - (int32_t)b;
    z += (z <= 0) ? 2147483562 : 0;
    return (uint32_t)z;
  }
  __device__ __forceinline__ void quad(uint32_t* u) {
    u[0] = combine(s1, s2);
#pragma unroll
    for (int j = 1; j < 4; ++j) {
      s1 = mul_mod_2p31<A1, 85u>(s1);
      s2 = mul_mod_2p31<A2, 249u>(s2);
      u[j] = combine(s1, s2);
    }
  }
  __device__ __forceinline__ void leap() {
    s1 = mulmod_2p31<85u>(s1, B1);
    s2 = mulmod_2p31<249u>(s2, B2);
  }
  __device__ void store_at(uint32_t j, uint32_t* st, uint64_t sn, uint64_t si) const {
    uint32_t a = s1, b = s2;
    for (uint32_t i = 0; i < j; ++i) {
      a = mul_mod_2p31<A1, 85u>(a);
      b = mul_mod_2p31<A2, 249u>(b);
    }
    st[si] = a;
    st[sn + si] = b;
  }
  static __device__ float paper_f32(uint32_t u) { return Ranecu<>::paper_f32(u); }
  static void q_map(uint64_t q, uint64_t& j0, uint64_t& j1) {
    j0 = cpowmod(A1, q, 2147483563u);
    j1 = cpowmod(A2, q, 2147483399u);
  }
  __device__ void advance_q(uint64_t j0, uint64_t j1, uint32_t w) {
    for (uint32_t i = 0; i < w; ++i) {
      s1 = mulmod_2p31<85u>(s1, (uint32_t)j0);
      s2 = mulmod_2p31<249u>(s2, (uint32_t)j1);
    }
  }
};

// DRAND48 / RANNYU: the draw is X >> 16 of the 48-bit state.
template <uint64_t A, uint64_t C>
struct LeapLcg48 {
  static constexpr int BITS = 32;
  static constexpr bool kNtOut = false;
  static constexpr uint64_t M = (1ull << 48) - 1;
  static constexpr Affine48 PL = caffine_pow(A, C, kLeapBlock - 3);
  uint64_t x;
  __device__ void load(const uint32_t* st, uint64_t sn, uint64_t si) {
    x = (uint64_t)st[si] | ((uint64_t)st[sn + si] << 32);
  }
  static constexpr std::array<Affine48, 64> starts() {
    std::array<Affine48, 64> t{};
    for (uint32_t l = 0; l < 64; ++l) t[l] = caffine_pow(A, C, kLeapQuad * l + 1);
    return t;
  }
  static constexpr std::array<Affine48, 64> kStart = starts();
  // lane l: X_{4l+1}, the state of its first position
  __device__ void start(int lane) {
    const Affine48 f = kStart[lane];
    x = (f.a * x + f.c) & M;
  }
  __device__ __forceinline__ void quad(uint32_t* u) {
    u[0] = (uint32_t)(x >> 16);
#pragma unroll
    for (int j = 1; j < 4; ++j) {
      x = (A * x + C) & M;
      u[j] = (uint32_t)(x >> 16);
    }
  }
  __device__ __forceinline__ void leap() { x = (PL.a * x + PL.c) & M; }
  __device__ void store_at(uint32_t j, uint32_t* st, uint64_t sn, uint64_t si) const {
    uint64_t y = x;
    for (uint32_t i = 0; i < j; ++i) y = (A * y + C) & M;
    st[si] = (uint32_t)y;
    st[sn + si] = (uint32_t)(y >> 32);
  }
  static void q_map(uint64_t q, uint64_t& j0, uint64_t& j1) {
    const Affine48 f = caffine_pow(A, C, q);
    j0 = f.a;
    j1 = f.c;
  }
  __device__ void advance_q(uint64_t j0, uint64_t j1, uint32_t w) {
    for (uint32_t i = 0; i < w; ++i) x = (j0 * x + j1) & M;
  }
};

template <class L, int DT>
__device__ __forceinline__ float leap_f32(uint32_t u) {
  if constexpr (DT == F32P)
    return L::paper_f32(u);
  else
    return to_f32<L::BITS>(u);
}

// Stores the four draws of positions v .. v+3 (v a multiple of 4): one
// 16-byte store when all are valid and `vec` (the row is 16-byte aligned),
// element by element otherwise.  fp64: elements v/2 and v/2 + 1.
template <class L, int DT>
__device__ __forceinline__ void leap_emit(uint64_t row, uint32_t v, const uint32_t* u, uint32_t draws, bool vec) {
  if constexpr (DT == F64) {
    const double d0 = to_f64<L::BITS>(u[0], u[1]), d1 = to_f64<L::BITS>(u[2], u[3]);
    const uint64_t p = row + 4ull * v;
    if (vec && v + 4u <= draws) {
      const uint64_t b0 = (uint64_t)__double_as_longlong(d0), b1 = (uint64_t)__double_as_longlong(d1);
      put<v4u, L::kNtOut>(p, v4u{(uint32_t)b0, (uint32_t)(b0 >> 32), (uint32_t)b1, (uint32_t)(b1 >> 32)});
    } else {  // draws is even: pairs are whole
      if (v + 2u <= draws) put<double, L::kNtOut>(p, d0);
      if (v + 4u <= draws) put<double, L::kNtOut>(p + 8u, d1);
    }
  } else {
    uint32_t o[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) o[j] = DT == U32 ? u[j] : __float_as_uint(leap_f32<L, DT>(u[j]));
    const uint64_t p = row + 4ull * v;
    if (vec && v + 4u <= draws) {
      put<v4u, L::kNtOut>(p, v4u{o[0], o[1], o[2], o[3]});
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (v + (uint32_t)j < draws) put<uint32_t, L::kNtOut>(p + 4ull * j, o[j]);
    }
  }
}

template <class L, int DT>
__global__ __launch_bounds__(256) void k_leap_generate(uint32_t* __restrict__ state, uint64_t n, uint32_t draws,
                                                       void* __restrict__ out, uint64_t row_elems, uint64_t elem_off) {
  const int lane = threadIdx.x & 63;
  const uint64_t s = (uint64_t)blockIdx.x * 4u + (threadIdx.x >> 6);
  if (s >= n || draws == 0) return;  // whole wavefront
  L g;
  g.load(state, n, s);
  g.start(lane);  // X of position 4 l
  constexpr uint64_t es = DT == F64 ? 8 : 4;
  // position v's element at byte row + 4 v (an fp64 element per pair of draws)
  const uint64_t row = reinterpret_cast<uint64_t>(out) + (s * row_elems + elem_off) * es;
  const bool vec = (row & 15u) == 0u;
  // blocks k with 256 (k + 2) <= draws: every lane fills its four positions and leaps
  const uint32_t full = draws / kLeapBlock;
  uint32_t k = 0;
  uint32_t u[4];
#pragma unroll 2
  for (; k + 1u < full; ++k) {
    g.quad(u);
    leap_emit<L, DT>(row, k * kLeapBlock + kLeapQuad * (uint32_t)lane, u, draws, vec);
    g.leap();
  }
  // the last one or two blocks: a lane leaps only if it has a later position;
  // the lane of the last position stores the state after it
  const uint32_t last = draws - 1u;
  for (; k * kLeapBlock < draws; ++k) {
    const uint32_t v = k * kLeapBlock + kLeapQuad * (uint32_t)lane;
    if (v < draws) {
      L h = g;  // quad() moves the state to the quad's last position
      h.quad(u);
      leap_emit<L, DT>(row, v, u, draws, vec);
      if (v + kLeapBlock < draws) {
        h.leap();
        g = h;
      } else if (last - v < kLeapQuad) {
        g.store_at(last - v, state, n, s);
      }
    }
  }
}

// Plain generation by quarters of rows: the four wavefronts of a workgroup
// share its four streams, wavefront w generating positions [w Q, (w + 1) Q)
// (Q a multiple of 256) of each row in turn, from the stream's state advanced
// w Q positions (the map of Q steps, j0/j1, applied w times).  At any moment a
// workgroup's stores fall in four contiguous stretches of adjacent rows; this
// store order measured 4-5% faster than one wavefront per row.  Every
// wavefront reads the four states before the barrier; the wavefront of a
// row's last position writes its new state after it.
template <class L, int DT>
__global__ __launch_bounds__(256) void k_leap_quarters(uint32_t* __restrict__ state, uint64_t n, uint32_t draws,
                                                       uint32_t Q, uint64_t j0, uint64_t j1, void* __restrict__ out,
                                                       uint64_t row_elems, uint64_t elem_off) {
  const int lane = threadIdx.x & 63;
  const uint32_t w = uni(threadIdx.x >> 6);
  const uint64_t s0 = (uint64_t)blockIdx.x * 4u;
  L g[4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
    if (s0 + r < n) g[r].load(state, n, s0 + r);
  __syncthreads();
  const uint32_t beg = w * Q, end = min(beg + Q, draws);
  if (beg >= end) return;  // whole wavefront, after the barrier
  constexpr uint64_t es = DT == F64 ? 8 : 4;
  const uint32_t last = draws - 1u;
  for (int r = 0; r < 4; ++r) {
    const uint64_t s = s0 + r;
    if (s >= n) break;
    L h = g[r];
    h.advance_q(j0, j1, w);  // X of position w Q
    h.start(lane);           // X of position w Q + 4 l
    const uint64_t row = reinterpret_cast<uint64_t>(out) + (s * row_elems + elem_off) * es;
    const bool vec = (row & 15u) == 0u;
    uint32_t u[4];
    uint32_t v = beg + kLeapQuad * (uint32_t)lane;
    // blocks whose next block is still inside the quarter: fill, then leap
    for (; v + kLeapBlock + (kLeapBlock - kLeapQuad * (uint32_t)lane) <= end; v += kLeapBlock) {
      h.quad(u);
      leap_emit<L, DT>(row, v, u, end, vec);
      h.leap();
    }
    // the remaining one or two blocks: leap only towards a later position
    for (; v - kLeapQuad * (uint32_t)lane < end; v += kLeapBlock) {
      if (v < end) {
        L q = h;
        q.quad(u);
        leap_emit<L, DT>(row, v, u, end, vec);
        if (v + kLeapBlock < end) {
          q.leap();
          h = q;
        } else if (end == draws && last - v < kLeapQuad) {
          h.store_at(last - v, state, n, s);
        }
      }
    }
  }
}

template <class L>
hipError_t launch_leap_quarters(int dtype, uint32_t* st, uint64_t n, uint64_t draws, void* out, uint64_t row_elems,
                                uint64_t off, hipStream_t s) {
  const uint64_t Q = ((draws + 3) / 4 + kLeapBlock - 1) / kLeapBlock * kLeapBlock;
  uint64_t j0 = 0, j1 = 0;
  L::q_map(Q, j0, j1);
  const dim3 grid((unsigned)((n + 3) / 4)), block(256);
  const uint32_t d = (uint32_t)draws, q = (uint32_t)Q;
  switch (dtype) {
    case U32:
      hipLaunchKernelGGL((k_leap_quarters<L, U32>), grid, block, 0, s, st, n, d, q, j0, j1, out, row_elems, off);
      break;
    case F32:
      hipLaunchKernelGGL((k_leap_quarters<L, F32>), grid, block, 0, s, st, n, d, q, j0, j1, out, row_elems, off);
      break;
    case F64:
      hipLaunchKernelGGL((k_leap_quarters<L, F64>), grid, block, 0, s, st, n, d, q, j0, j1, out, row_elems, off);
      break;
    case F32P:
      if constexpr (requires { L::paper_f32(0u); }) {
        hipLaunchKernelGGL((k_leap_quarters<L, F32P>), grid, block, 0, s, st, n, d, q, j0, j1, out, row_elems,
                           off);
        break;
      }
      return hipErrorInvalidValue;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class L>
hipError_t launch_leap(int dtype, uint32_t* st, uint64_t n, uint64_t draws, void* out, uint64_t row_elems,
                       uint64_t off, hipStream_t s) {
  // rows of at least four blocks per wavefront go by quarters
  if (draws >= 16 * kLeapBlock) return launch_leap_quarters<L>(dtype, st, n, draws, out, row_elems, off, s);
  const dim3 grid((unsigned)((n + 3) / 4)), block(256);
  const uint32_t d = (uint32_t)draws;
  switch (dtype) {
    case U32:
      hipLaunchKernelGGL((k_leap_generate<L, U32>), grid, block, 0, s, st, n, d, out, row_elems, off);
      break;
    case F32:
      hipLaunchKernelGGL((k_leap_generate<L, F32>), grid, block, 0, s, st, n, d, out, row_elems, off);
      break;
    case F64:
      hipLaunchKernelGGL((k_leap_generate<L, F64>), grid, block, 0, s, st, n, d, out, row_elems, off);
      break;
    case F32P:
      if constexpr (requires { L::paper_f32(0u); }) {
        hipLaunchKernelGGL((k_leap_generate<L, F32P>), grid, block, 0, s, st, n, d, out, row_elems, off);
        break;
      }
      return hipErrorInvalidValue;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
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


}  // namespace

hipError_t launch_generate(int kind, uint32_t p, uint32_t* st, uint64_t n, uint64_t draws, int dtype, void* out,
                           uint64_t row_elems, uint64_t off, hipStream_t s) {
  switch (kind) {
    case GGL:
      return launch_leap<LeapGgl>(dtype, st, n, draws, out, row_elems, off, s);
    case XOR128:
      return launch_lane_gen<Xor128<>>(dtype, p, st, n, draws, out, row_elems, off, s);
    case RANECU:
      return launch_leap<LeapRanecu>(dtype, st, n, draws, out, row_elems, off, s);
    case RANMAR:
      return launch_lane_gen<Ranmar<>>(dtype, p, st, n, draws, out, row_elems, off, s);
    case DRAND48:
      return launch_leap<LeapLcg48<25214903917ull, 11u>>(dtype, st, n, draws, out, row_elems, off, s);
    case RANNYU:
      return launch_leap<LeapLcg48<31167285ull, 0u>>(dtype, st, n, draws, out, row_elems, off, s);
    case RANLUX:  // prng_generate runs RANLUX through launch_lux_plain
      return hipErrorInvalidValue;
    case MT19937: {
      const dim3 grid((unsigned)((n + 1) / 2)), block(256);
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

hipError_t launch_xor128_split(uint32_t* st, const uint32_t* snap, uint64_t n, uint64_t draws, int dtype, uint32_t S,
                               uint32_t K, const uint32_t* pow2, void* out, uint64_t row_elems, uint64_t off,
                               hipStream_t s) {
  const dim3 grid((unsigned)((n + 255) / 256 * K)), block(256);
  const uint32_t d = (uint32_t)draws;
  switch (dtype) {
    case U32:
      hipLaunchKernelGGL((k_xor128_split<U32>), grid, block, 0, s, st, snap, n, d, S, K, pow2, out, row_elems, off);
      break;
    case F32:
      hipLaunchKernelGGL((k_xor128_split<F32>), grid, block, 0, s, st, snap, n, d, S, K, pow2, out, row_elems, off);
      break;
    case F64:
      hipLaunchKernelGGL((k_xor128_split<F64>), grid, block, 0, s, st, snap, n, d, S, K, pow2, out, row_elems, off);
      break;
    case F32P:
      hipLaunchKernelGGL((k_xor128_split<F32P>), grid, block, 0, s, st, snap, n, d, S, K, pow2, out, row_elems,
                         off);
      break;
    default:
      return hipErrorInvalidValue;
  }
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


}  // namespace prng
