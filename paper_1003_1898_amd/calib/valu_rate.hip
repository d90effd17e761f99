// VALU issue-rate calibration for gfx950: kernels made of a known number of
// one vector instruction, so that the time of a launch (and the SQ_INSTS_VALU
// and GRBM_GUI_ACTIVE counters of a profiled run) give the chip's measured
// issue rate per SIMD and clock.  This is the peak that VALU utilisation
// figures of the generator kernels are set against.  Not part of libprng.
//
// Each thread runs `iters` iterations of 8 independent chains x 8 steps of
// the chosen instruction (64 per iteration, written in inline assembly so the
// compiler can neither fuse nor drop them); the loop adds a few scalar
// instructions per iteration.  One store per thread keeps the chains live.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace {

enum Op : int {
  kXor = 0,      // v_xor_b32: plain 32-bit logic
  kSubCo = 1,    // v_sub_co_u32: subtract with carry out (the SWB step's first half)
  kSubb = 2,     // v_subb_co_u32 chained through VCC: the SWB borrow chain, one step after another
  kBitop3 = 3,   // v_bitop3_b32: gfx950's three-input bitwise operation
  kShl = 4,      // v_lshlrev_b32
  kMulLo = 5,    // v_mul_lo_u32: 32-bit integer multiply
  kCvt = 6,      // v_cvt_f32_u32
  kAnd = 7,      // v_and_b32
  kMad64 = 8,    // v_mad_u64_u32: 32 x 32 + 64-bit multiply-add (the MLCG product)
  kAlign = 9,    // v_alignbit_b32: funnel shift (the 64-bit product's bits 31..62)
  kMad24 = 10,   // v_mad_u32_u24: 24-bit multiply-add (the MLCG fold)
  kMin = 11,     // v_min_u32 (the MLCG's conditional subtraction)
  kAdd = 12,     // v_add_u32
};

#define STEP8(ASM) ASM(b0) ASM(b1) ASM(b2) ASM(b3) ASM(b4) ASM(b5) ASM(b6) ASM(b7)

template <int OP>
__global__ __launch_bounds__(256) void k_valu(uint32_t* __restrict__ out, uint32_t iters, uint32_t seed) {
  const uint32_t t = blockIdx.x * 256u + threadIdx.x;
  uint32_t a0 = seed ^ t, a1 = a0 * 3u + 1u, a2 = a0 * 5u + 2u, a3 = a0 * 7u + 3u, a4 = a0 * 11u + 4u,
           a5 = a0 * 13u + 5u, a6 = a0 * 17u + 6u, a7 = a0 * 19u + 7u;
  const uint32_t k = seed | 1u, k2 = seed * 7u + 3u;
  using Acc = std::conditional_t<OP == kMad64, uint64_t, uint32_t>;
  Acc b0 = a0, b1 = a1, b2 = a2, b3 = a3, b4 = a4, b5 = a5, b6 = a6, b7 = a7;
  for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      if constexpr (OP == kXor) {
#define A(x) asm volatile("v_xor_b32 %0, %1, %0" : "+v"(x) : "v"(k));
        STEP8(A)
#undef A
      } else if constexpr (OP == kSubCo) {
        // carry out of each chain to an SGPR pair of its own (no VCC hazard between chains)
        uint64_t c0, c1, c2, c3, c4, c5, c6, c7;
#define A(x, c) asm volatile("v_sub_co_u32 %0, %1, %0, %2" : "+v"(x), "=s"(c) : "v"(k));
        A(b0, c0) A(b1, c1) A(b2, c2) A(b3, c3) A(b4, c4) A(b5, c5) A(b6, c6) A(b7, c7)
#undef A
        (void)c0; (void)c1; (void)c2; (void)c3; (void)c4; (void)c5; (void)c6; (void)c7;
      } else if constexpr (OP == kSubb) {
#define A(x) asm volatile("v_subb_co_u32 %0, vcc, %0, %1, vcc" : "+v"(x) : "v"(k) : "vcc");
        STEP8(A)
#undef A
      } else if constexpr (OP == kBitop3) {
#define A(x) asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x6a" : "+v"(x) : "v"(k), "v"(a0));
        STEP8(A)
#undef A
      } else if constexpr (OP == kShl) {
#define A(x) asm volatile("v_lshlrev_b32 %0, 1, %0" : "+v"(x));
        STEP8(A)
#undef A
      } else if constexpr (OP == kMulLo) {
#define A(x) asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(x) : "v"(k));
        STEP8(A)
#undef A
      } else if constexpr (OP == kCvt) {
#define A(x) asm volatile("v_cvt_f32_u32 %0, %0" : "+v"(x));
        STEP8(A)
#undef A
      } else if constexpr (OP == kAnd) {
#define A(x) asm volatile("v_and_b32 %0, %0, %1" : "+v"(x) : "v"(k));
        STEP8(A)
#undef A
      } else if constexpr (OP == kMad64) {
        // eight 64-bit accumulators, each x <- k * k2 + x (carry out to an SGPR pair)
        uint64_t c;
#define A(x) asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(x), "=s"(c) : "v"(k), "v"(k2));
        STEP8(A)
#undef A
        (void)c;
      } else if constexpr (OP == kAlign) {
#define A(x) asm volatile("v_alignbit_b32 %0, %1, %0, 31" : "+v"(x) : "v"(k));
        STEP8(A)
#undef A
      } else if constexpr (OP == kMad24) {
#define A(x) asm volatile("v_mad_u32_u24 %0, %0, %1, %2" : "+v"(x) : "v"(k), "v"(k2));
        STEP8(A)
#undef A
      } else if constexpr (OP == kMin) {
#define A(x) asm volatile("v_min_u32 %0, %0, %1" : "+v"(x) : "v"(k));
        STEP8(A)
#undef A
      } else {
#define A(x) asm volatile("v_add_u32 %0, %0, %1" : "+v"(x) : "v"(k));
        STEP8(A)
#undef A
      }
    }
  }
  out[t] = (uint32_t)(b0 ^ b1 ^ b2 ^ b3 ^ b4 ^ b5 ^ b6 ^ b7);
}

}  // namespace

extern "C" __attribute__((visibility("default"))) int calib_valu_launch(int op, uint32_t iters, uint32_t blocks,
                                                                          void* out, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  uint32_t* o = static_cast<uint32_t*>(out);
  const dim3 grid(blocks), block(256);
  switch (op) {
    case kXor: hipLaunchKernelGGL((k_valu<kXor>), grid, block, 0, s, o, iters, 12345u); break;
    case kSubCo: hipLaunchKernelGGL((k_valu<kSubCo>), grid, block, 0, s, o, iters, 12345u); break;
    case kSubb: hipLaunchKernelGGL((k_valu<kSubb>), grid, block, 0, s, o, iters, 12345u); break;
    case kBitop3: hipLaunchKernelGGL((k_valu<kBitop3>), grid, block, 0, s, o, iters, 12345u); break;
    case kShl: hipLaunchKernelGGL((k_valu<kShl>), grid, block, 0, s, o, iters, 12345u); break;
    case kMulLo: hipLaunchKernelGGL((k_valu<kMulLo>), grid, block, 0, s, o, iters, 12345u); break;
    case kCvt: hipLaunchKernelGGL((k_valu<kCvt>), grid, block, 0, s, o, iters, 12345u); break;
    case kAnd: hipLaunchKernelGGL((k_valu<kAnd>), grid, block, 0, s, o, iters, 12345u); break;
    case kMad64: hipLaunchKernelGGL((k_valu<kMad64>), grid, block, 0, s, o, iters, 12345u); break;
    case kAlign: hipLaunchKernelGGL((k_valu<kAlign>), grid, block, 0, s, o, iters, 12345u); break;
    case kMad24: hipLaunchKernelGGL((k_valu<kMad24>), grid, block, 0, s, o, iters, 12345u); break;
    case kMin: hipLaunchKernelGGL((k_valu<kMin>), grid, block, 0, s, o, iters, 12345u); break;
    case kAdd: hipLaunchKernelGGL((k_valu<kAdd>), grid, block, 0, s, o, iters, 12345u); break;
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

// VALU instructions per thread and iteration of every op's kernel.
extern "C" __attribute__((visibility("default"))) int calib_valu_per_iter(void) { return 64; }
