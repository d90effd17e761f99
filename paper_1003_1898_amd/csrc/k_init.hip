// Initialisation: seed tuples to canonical device states.
#include "device.h"

namespace prng {
namespace {

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


}  // namespace prng
