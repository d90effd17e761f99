// Split plain RANLUX generation: the kernel and its per-luxury launcher,
// instantiated for groups of luxury levels in k_lux_plain_a.hip,
// k_lux_plain_b.hip and k_lux_plain_c.hip.
#pragma once
#include "device.h"

namespace prng {
namespace {

// Plain RANLUX generation with every stream cut into K segments of S
// positions (S a multiple of 24): block b works on segment b / nb of the 256
// streams (b mod nb) of that range, nb = ceil(n / 256).  Segment 0 starts
// from the state, segment j > 0 from the state jumped ahead from the snapshot
// `snap` (taken before the launch; equal to `state` when K = 1) to the block
// boundary j S, j S / 24 - 1 blocks past the end of the stream's current one
// (multiplier from the object's block-jump table); the last segment writes
// the final state.  Draws are staged in
// three bytes (StageSplit24), so that the 96-draw chunks that keep each row's
// stores 128-byte aligned leave room for two wavefronts per SIMD: the borrow
// chain of one wavefront then overlaps the stores of the other.  Positions,
// fp64 pairing at segment boundaries and the output rows are as in
// k_lux_fused_split and the stream table.
template <int P, int DT>
__global__ __launch_bounds__(256) void k_lux_plain(uint32_t* __restrict__ state, const uint32_t* __restrict__ snap,
                                                   uint64_t n, uint32_t draws, uint32_t p, uint32_t S, uint32_t K,
                                                   const uint32_t* __restrict__ digits,
                                                   const uint32_t* __restrict__ aux, void* __restrict__ out,
                                                   uint64_t row_elems, uint64_t elem_off) {
  using G = Ranlux<96, P>;
  constexpr uint32_t T = G::T;
  __shared__ __attribute__((aligned(16))) uint32_t stage_all[4][(StageSplit24<T>::kBytes + 3) / 4];
  const int lane = threadIdx.x & 63;
  uint32_t* stage = stage_all[threadIdx.x >> 6];
  const uint32_t nb = (uint32_t)((n + 255) / 256);
  const uint32_t j = blockIdx.x / nb;
  const uint64_t si = (uint64_t)(blockIdx.x - j * nb) * 256u + threadIdx.x;
  const bool live = si < n;
  const bool last = j + 1u == K;
  G g;
  g.p = p;
  uint32_t k0 = 0, gbeg = 0, ebeg = 0, vend = 0;
  uint64_t q = 0;
  constexpr uint64_t es = DT == F64 ? 8 : 4;
  if (live) {
    constexpr bool f64 = DT == F64;
    if (j == 0) {
      g.load(snap, n, si, k0);
      gbeg = k0;
    } else {
      k0 = g.load_jumped_blocks(snap, n, si, j * S / 24u - 1u, digits, aux);
      gbeg = j * S;
    }
    vend = last ? k0 + draws : (j + 1u) * S + ((f64 && (((j + 1u) * S - k0) & 1u)) ? 1u : 0u);
    ebeg = j == 0 ? k0 : j * S + ((f64 && ((j * S - k0) & 1u)) ? 1u : 0u);
    q = reinterpret_cast<uint64_t>(out) + (si * row_elems + elem_off) * es - 4ull * k0;
    // Segment-local coordinates, local = global - off, off a multiple of 24 so
    // that ring slots and block boundaries stay where they are (a skip is due
    // at local block starts >= 24, segment j > 0 starting at local 24 u with
    // its skip pending).  When k0 is a multiple of 8, off is also congruent to
    // k0 mod 32: chunks (multiples of 96 local) then start at output elements
    // that are multiples of 32, and every row store covers whole 128-byte lines.
    int32_t off;
    if (k0 % 8u == 0u) {
      const uint32_t w = (k0 / 8u) & 3u;
      off = j == 0 ? -24 * (int32_t)w : (int32_t)(j * S) - 24 * (int32_t)(((w + 3u) & 3u) + 1u);
    } else {
      off = j == 0 ? 0 : (int32_t)(j * S) - 24;
    }
    gbeg = (uint32_t)((int32_t)gbeg - off);
    ebeg = (uint32_t)((int32_t)ebeg - off);
    vend = (uint32_t)((int32_t)vend - off);
    q += (uint64_t)(4ll * off);
  } else {
    g.zero();
  }
  lane_loop<G, DT, false, true>(g, stage, lane, gbeg, ebeg, vend, q, true, row_elems * es);
  if (live && last) g.store(state, n, si, gbeg, vend);
}


template <int P>
hipError_t launch_lux_plain_p(uint32_t p, uint32_t* st, const uint32_t* snap, uint64_t n, uint64_t draws, int dtype,
                              uint32_t S, uint32_t K, const uint32_t* digits, const uint32_t* aux, void* out,
                              uint64_t row_elems, uint64_t off, hipStream_t s) {
  const dim3 grid((unsigned)((n + 255) / 256 * K)), block(256);
  const uint32_t d = (uint32_t)draws;
  switch (dtype) {
    case U32:
      hipLaunchKernelGGL((k_lux_plain<P, U32>), grid, block, 0, s, st, snap, n, d, p, S, K, digits, aux, out, row_elems,
                         off);
      break;
    case F32:
      hipLaunchKernelGGL((k_lux_plain<P, F32>), grid, block, 0, s, st, snap, n, d, p, S, K, digits, aux, out, row_elems,
                         off);
      break;
    case F64:
      hipLaunchKernelGGL((k_lux_plain<P, F64>), grid, block, 0, s, st, snap, n, d, p, S, K, digits, aux, out, row_elems,
                         off);
      break;
    case F32P:
      hipLaunchKernelGGL((k_lux_plain<P, F32P>), grid, block, 0, s, st, snap, n, d, p, S, K, digits, aux, out,
                         row_elems, off);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}


}  // namespace

// One group of luxury levels each (false when p is not in the group).
bool launch_lux_plain_group_a(uint32_t p, uint32_t* st, const uint32_t* snap, uint64_t n, uint64_t draws, int dtype,
                              uint32_t S, uint32_t K, const uint32_t* digits, const uint32_t* aux, void* out,
                              uint64_t row_elems, uint64_t off, hipStream_t s, hipError_t* err);
bool launch_lux_plain_group_b(uint32_t p, uint32_t* st, const uint32_t* snap, uint64_t n, uint64_t draws, int dtype,
                              uint32_t S, uint32_t K, const uint32_t* digits, const uint32_t* aux, void* out,
                              uint64_t row_elems, uint64_t off, hipStream_t s, hipError_t* err);
bool launch_lux_plain_group_c(uint32_t p, uint32_t* st, const uint32_t* snap, uint64_t n, uint64_t draws, int dtype,
                              uint32_t S, uint32_t K, const uint32_t* digits, const uint32_t* aux, void* out,
                              uint64_t row_elems, uint64_t off, hipStream_t s, hipError_t* err);

}  // namespace prng
