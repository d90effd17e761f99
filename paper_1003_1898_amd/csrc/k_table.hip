// Stream table: persistent lane and MT19937 kernels, MT19937 jump windows, snapshots, counters.
#include "device.h"

namespace prng {
namespace {

template <int CLASS>
__global__ __launch_bounds__(256) void k_table_lane(const TableTask* __restrict__ tasks, uint32_t ntasks,
                                                    const TableRow* __restrict__ rows,
                                                    const uint32_t* __restrict__ tails, uint32_t* counter,
                                                    const uint32_t* __restrict__ aux) {
  constexpr int TS = kClassT[CLASS];
  // RANMAR's jump also passes 97 values per lane through the stage (stride
  // 64), which its 128-draw stage holds; RANLUX, in class 0, stages its
  // 24-bit draws of 96-draw chunks in three bytes, which takes a little more
  // than the 64-draw word stage
  constexpr int SW = CLASS == 0 ? std::max(stage_words<TS>(), (StageSplit24<kLuxTableT>::kBytes + 3) / 4)
                     : stage_words<TS>() < 97 * 64 ? 97 * 64
                                                   : stage_words<TS>();
  __shared__ __attribute__((aligned(16))) uint32_t stage_all[4][SW];
  const int lane = threadIdx.x & 63;
  uint32_t* stage = stage_all[threadIdx.x >> 6];
  for (uint32_t t = next_task(counter, lane); t < ntasks; t = next_task(counter, lane)) {
    const TableTask task = tasks[t];
    const uint32_t kind = uni(task.kind), dt = uni(task.dtype), p = uni(task.p);
#define PRNG_TASK(K, G, SPLIT)                                                              \
  case K * 4 + U32: lane_task<G, U32, SPLIT>(stage, lane, rows, tails, task, p, aux); break; \
  case K * 4 + F32: lane_task<G, F32, SPLIT>(stage, lane, rows, tails, task, p, aux); break; \
  case K * 4 + F64: lane_task<G, F64, SPLIT>(stage, lane, rows, tails, task, p, aux); break;
    if constexpr (CLASS == 0) {
      switch (kind * 4 + dt) {
        PRNG_TASK(GGL, Ggl<64>, false)
        PRNG_TASK(XOR128, Xor128<64>, false)
        PRNG_TASK(RANECU, Ranecu<64>, false)
        PRNG_TASK(DRAND48, Drand48<64>, false)
        PRNG_TASK(RANNYU, Rannyu<64>, false)
        PRNG_TASK(RANLUX, Ranlux<kLuxTableT>, true)
        default:
          break;
      }
    } else {
      switch (kind * 4 + dt) {
        PRNG_TASK(RANMAR, Ranmar<kClassT[1]>, false)
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
// that would split a pair of draws moves one draw later.  One task per
// workgroup, its four wavefronts sharing the stream (a segment's chain runs
// about four times as wide as on one wavefront).
__global__ __launch_bounds__(256) void k_table_mt(const TableTask* __restrict__ tasks, uint32_t ntasks,
                                                  const TableRow* __restrict__ rows, uint32_t* counter) {
  __shared__ __attribute__((aligned(16))) uint32_t mt[624];
  __shared__ __attribute__((aligned(16))) uint32_t stage[628];
  __shared__ uint32_t task_slot;
  const int tid = (int)threadIdx.x;
  // the next task index, uniform over the workgroup
  auto fetch = [&]() -> uint32_t {
    __syncthreads();  // every thread has read the previous index
    if (tid == 0) task_slot = atomicAdd(counter, 1u);
    __syncthreads();
    return task_slot;
  };
  for (uint32_t t = fetch(); t < ntasks; t = fetch()) {
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
      mt_body<U32>(mt, stage, tid, src, pos0, skip, end - beg, outp, dst);
    else if (dt == F32)
      mt_body<F32>(mt, stage, tid, src, pos0, skip, end - beg, outp, dst);
    else
      mt_body<F64>(mt, stage, tid, src, pos0, skip, end - beg, outp, dst);
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
  // thread t of a group owns words t, t + 256 and, for t < 112, t + 512, so
  // that the 64 lanes of every LDS read take 64 consecutive words (no bank
  // conflicts: two words per lane at stride two halved the LDS rate)
  const bool hi = t < 112;
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
    uint32_t a0 = 0, a1 = 0, a2 = 0;
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
        const uint32_t* p = seq + ix[b] + t;
        v0[b] = p[0];
        v1[b] = p[256];
      }
      if (hi) {
        uint32_t v2[8];
#pragma unroll
        for (int b = 0; b < 8; ++b) v2[b] = seq[ix[b] + t + 512];
#pragma unroll
        for (int b = 0; b < 8; ++b) a2 ^= v2[b];
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
        const uint32_t* p = seq + i + t;
        a0 ^= p[0];
        a1 ^= p[256];
        if (hi) a2 ^= p[512];
      }
    }
    if (grp > 0) {
      uint32_t* pp = part[grp - 1];
      pp[t] = a0;
      pp[t + 256] = a1;
      if (hi) pp[t + 512] = a2;
    }
    __syncthreads();
    if (grp == 0) {
#pragma unroll
      for (int g = 0; g < 3; ++g) {
        a0 ^= part[g][t];
        a1 ^= part[g][t + 256];
        if (hi) a2 ^= part[g][t + 512];
      }
      dst[t] = a0;
      dst[t + 256] = a1;
      if (hi) dst[t + 512] = a2;
      if (t == 0) dst[624] = 624u;
    }
    __syncthreads();  // seq and part are rebuilt for the next segment
  }
}

// Copies the starting states of split streams (one thread per word).
// Start of a run: clears the task counters (block 0) and copies the starting
// states of the cut streams (a kernel rather than a memset and a copy, so
// that both are one ordinary node when the run is captured into a graph).
__global__ void k_table_prepare(uint32_t* counters, int n_counters, const SnapRow* __restrict__ rows, uint32_t n,
                                uint32_t max_words) {
  if (blockIdx.x == 0 && (int)threadIdx.x < n_counters) counters[threadIdx.x] = 0u;
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


}  // namespace

hipError_t launch_table_lane(int cls, const TableTask* tasks, uint32_t ntasks, const TableRow* rows,
                             const uint32_t* tails, uint32_t* counter, const uint32_t* aux, int grid, hipStream_t s) {
  if (cls == 0)
    hipLaunchKernelGGL((k_table_lane<0>), dim3(grid), dim3(256), 0, s, tasks, ntasks, rows, tails, counter, aux);
  else
    hipLaunchKernelGGL((k_table_lane<1>), dim3(grid), dim3(256), 0, s, tasks, ntasks, rows, tails, counter, aux);
  return hipGetLastError();
}

hipError_t launch_table_prepare(uint32_t* counters, int n_counters, const SnapRow* rows, uint32_t n,
                                uint32_t max_words, hipStream_t s) {
  if (n_counters > 256) return hipErrorInvalidValue;
  const uint64_t threads = (uint64_t)n * max_words;
  const unsigned grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((threads + 255) / 256, 4096));
  hipLaunchKernelGGL(k_table_prepare, dim3(grid), dim3(256), 0, s, counters, n_counters, rows, n, max_words);
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
