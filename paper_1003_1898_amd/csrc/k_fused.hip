// In-kernel consumers: exact mantissa sums and 64-bin histograms per stream.
#include "device.h"

namespace prng {
namespace {

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

// Emitter of mt_twist_emit for the fused consumer: the draw's top 24 bits
// (the f32 value times 2^24) into the lane's sum and the wave's histogram.
struct MtFusedEmit {
  uint32_t* h;
  uint32_t part;
  __device__ __forceinline__ void operator()(int, uint32_t w) {
    const uint32_t k = mt_temper(w) >> 8;
    part += k;
    __hip_atomic_fetch_add(&h[k >> 18], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
  }
};

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
    if (pos == 0u && draws - done > 624u) {
      // a whole block with draws after it: consumed during the twist that
      // makes the next block
      MtFusedEmit emit{h, 0u};
      mt_twist_emit(mt, lane, emit);
      acc += emit.part;
      done += 624u;
      continue;
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

template <class G>
hipError_t launch_lane_fused(uint32_t p, uint32_t* st, uint64_t n, uint64_t draws, uint64_t* sum, uint32_t* hist,
                             bool acc, hipStream_t s) {
  const dim3 grid((unsigned)((n + 255) / 256)), block(256);
  hipLaunchKernelGGL((k_lane_fused<G>), grid, block, 0, s, st, n, (uint32_t)draws, p, sum, hist, acc ? 1 : 0);
  return hipGetLastError();
}


}  // namespace

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


}  // namespace prng
