// Plain bulk generation: lane-per-stream kernels (stream-major and four-way interleaved output) and MT19937.
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
    case RANLUX:  // prng_generate runs RANLUX through launch_lux_plain
      return hipErrorInvalidValue;
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
