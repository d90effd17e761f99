// RANLUX: the lag-table variants of Table 3, the split in-kernel consumer, and
// the dispatch of split plain generation over the luxury groups.
#include "lux_plain.h"

namespace prng {
namespace {

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
                                                         const uint32_t* __restrict__ digits,
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
      k0 = g.load_jumped_blocks(snap, n, si, j * S / 24u - 1u, digits, aux);
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


}  // namespace

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

hipError_t launch_lux_plain(uint32_t p, uint32_t* st, const uint32_t* snap, uint64_t n, uint64_t draws, int dtype,
                            uint32_t S, uint32_t K, const uint32_t* digits, const uint32_t* aux, void* out,
                            uint64_t row_elems, uint64_t off, hipStream_t s) {
  // the luxury levels get a compile-time skip, spread over three translation units
  hipError_t err = hipErrorInvalidValue;
  if (launch_lux_plain_group_a(p, st, snap, n, draws, dtype, S, K, digits, aux, out, row_elems, off, s, &err) ||
      launch_lux_plain_group_c(p, st, snap, n, draws, dtype, S, K, digits, aux, out, row_elems, off, s, &err) ||
      launch_lux_plain_group_b(p, st, snap, n, draws, dtype, S, K, digits, aux, out, row_elems, off, s, &err))
    return err;
  return hipErrorInvalidValue;
}
template <int P>
hipError_t launch_lux_fused_split_p(uint32_t p, uint32_t* st, const uint32_t* snap, uint64_t n, uint64_t draws,
                                    uint32_t S, uint32_t K, const uint32_t* digits, const uint32_t* aux, uint64_t* sum,
                                    uint32_t* hist, bool acc, hipStream_t s) {
  const dim3 grid((unsigned)((n + 3) / 4)), block(256);
  hipLaunchKernelGGL((k_lux_fused_split<P>), grid, block, 0, s, st, snap, n, (uint32_t)draws, p, S, K, digits, aux, sum,
                     hist, acc ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_lux_fused_split(uint32_t p, uint32_t* st, const uint32_t* snap, uint64_t n, uint64_t draws,
                                  uint32_t S, uint32_t K, const uint32_t* digits, const uint32_t* aux, uint64_t* sum,
                                  uint32_t* hist, bool acc, hipStream_t s) {
  switch (p) {  // the luxury levels get a compile-time skip
    case 24:
      return launch_lux_fused_split_p<24>(p, st, snap, n, draws, S, K, digits, aux, sum, hist, acc, s);
    case 48:
      return launch_lux_fused_split_p<48>(p, st, snap, n, draws, S, K, digits, aux, sum, hist, acc, s);
    case 97:
      return launch_lux_fused_split_p<97>(p, st, snap, n, draws, S, K, digits, aux, sum, hist, acc, s);
    case 223:
      return launch_lux_fused_split_p<223>(p, st, snap, n, draws, S, K, digits, aux, sum, hist, acc, s);
    case 389:
      return launch_lux_fused_split_p<389>(p, st, snap, n, draws, S, K, digits, aux, sum, hist, acc, s);
    case 120:
      return launch_lux_fused_split_p<120>(p, st, snap, n, draws, S, K, digits, aux, sum, hist, acc, s);
    case 240:
      return launch_lux_fused_split_p<240>(p, st, snap, n, draws, S, K, digits, aux, sum, hist, acc, s);
    case 408:
      return launch_lux_fused_split_p<408>(p, st, snap, n, draws, S, K, digits, aux, sum, hist, acc, s);
    default:
      return launch_lux_fused_split_p<0>(p, st, snap, n, draws, S, K, digits, aux, sum, hist, acc, s);
  }
}


}  // namespace prng
