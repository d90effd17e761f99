// Arithmetic modulo m = 2^576 - 2^240 + 1 on 18 little-endian 32-bit limbs,
// for jump-ahead of the RANLUX core.
//
// The subtract-with-borrow recurrence x_n = x_{n-10} - x_{n-24} - c mod 2^24
// (Appendix A.4.5) is an LCG in disguise: with b = 2^24, R = sum_j x_{n-24+j} b^j
// (the 24 lags, oldest least significant) and c the borrow, the number
// S = R - floor(R / b^14) + c satisfies S_{n+1} = b^{-1} S_n mod m for
// m = b^24 - b^10 + 1.  (Multiply the definition of S_{n+1} by b and use the
// recurrence: b S_{n+1} = S_n + x_n m.)  Jumping J steps is therefore one
// multiplication by b^{-J} mod m.  Used by the host (jump tables) and by the
// device (applying them), so the functions are plain loops over limbs.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__) || defined(__HIP__)
#define PRNG_HD __host__ __device__
#else
#define PRNG_HD
#endif

namespace prng {

constexpr int kL576 = 18;

// m = 2^576 - 2^240 + 1: limbs 8..17 all ones, limb 7 = 0xFFFF0000, limb 0 = 1.
PRNG_HD inline uint32_t m576_limb(int k) {
  return k == 0 ? 1u : (k < 7 ? 0u : (k == 7 ? 0xFFFF0000u : 0xFFFFFFFFu));
}

// out (nout limbs) = L + (H << 240) - H for v = H 2^576 + L (n limbs, n > 18):
// the same residue mod m, since 2^576 = 2^240 - 1 (mod m).  The result is
// non-negative because 2^240 > 1.
template <int N, int NOUT>
PRNG_HD inline void fold576(const uint32_t* v, uint32_t* out) {
  constexpr int NH = N - 18;
  int64_t acc = 0;
#pragma unroll
  for (int k = 0; k < NOUT; ++k) {
    if (k < 18) acc += (int64_t)v[k];
    uint32_t sh = 0;
    if (k - 7 >= 0 && k - 7 < NH) sh |= v[18 + k - 7] << 16;
    if (k - 8 >= 0 && k - 8 < NH) sh |= v[18 + k - 8] >> 16;
    acc += (int64_t)sh;
    if (k < NH) acc -= (int64_t)v[18 + k];
    out[k] = (uint32_t)acc;
    acc >>= 32;  // arithmetic: carries and borrows
  }
}

// v (19 limbs, v < 2^577) -> v mod m in 18 limbs.
PRNG_HD inline void finish576(uint32_t* v, uint32_t* r) {
#pragma unroll
  for (int it = 0; it < 3; ++it) {
    // subtract m while v >= m
    bool ge = v[18] != 0;
    if (!ge) {
      ge = true;  // equal counts as >=
      for (int k = 17; k >= 0; --k) {
        const uint32_t mk = m576_limb(k);
        if (v[k] != mk) {
          ge = v[k] > mk;
          break;
        }
      }
    }
    if (ge) {
      int64_t acc = 0;
      for (int k = 0; k < 19; ++k) {
        acc += (int64_t)v[k] - (int64_t)(k < 18 ? m576_limb(k) : 0u);
        v[k] = (uint32_t)acc;
        acc >>= 32;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 18; ++k) r[k] = v[k];
}

// r = x * y mod m  (x, y in [0, m)); r may alias x or y.
PRNG_HD inline void mulmod576(const uint32_t* x, const uint32_t* y, uint32_t* r) {
  uint32_t p[36];
#pragma unroll
  for (int i = 0; i < 36; ++i) p[i] = 0;
#pragma unroll
  for (int i = 0; i < 18; ++i) {
    uint64_t carry = 0;
#pragma unroll
    for (int j = 0; j < 18; ++j) {
      const uint64_t t = (uint64_t)x[i] * y[j] + p[i + j] + carry;
      p[i + j] = (uint32_t)t;
      carry = t >> 32;
    }
    p[i + 18] = (uint32_t)carry;
  }
  uint32_t a[27], b[19], c[19];
  fold576<36, 27>(p, a);
  fold576<27, 19>(a, b);
  fold576<19, 19>(b, c);
  fold576<19, 19>(c, b);
  finish576(b, r);
}

// 24 lags (oldest first, 24-bit each) and borrow -> S = R - floor(R / 2^336) + c.
PRNG_HD inline void swb_to_lcg(const uint32_t* lag, uint32_t c, uint32_t* s) {
  uint32_t R[18];
#pragma unroll
  for (int k = 0; k < 18; ++k) R[k] = 0;
#pragma unroll
  for (int j = 0; j < 24; ++j) {  // lag j at bit 24 j
    const int bit = 24 * j, k = bit >> 5, o = bit & 31;
    R[k] |= lag[j] << o;
    if (o > 8) R[k + 1] |= lag[j] >> (32 - o);
  }
  // Q = R >> 336 = lags 14..23 packed the same way (240 bits, limbs 0..7)
  uint32_t Q[18];
#pragma unroll
  for (int k = 0; k < 18; ++k) Q[k] = 0;
#pragma unroll
  for (int j = 14; j < 24; ++j) {
    const int bit = 24 * (j - 14), k = bit >> 5, o = bit & 31;
    Q[k] |= lag[j] << o;
    if (o > 8) Q[k + 1] |= lag[j] >> (32 - o);
  }
  int64_t acc = (int64_t)c;
#pragma unroll
  for (int k = 0; k < 18; ++k) {
    acc += (int64_t)R[k] - (int64_t)Q[k];
    s[k] = (uint32_t)acc;
    acc >>= 32;
  }
}

// S in [0, m) -> 24 lags with R - floor(R / 2^336) = S (borrow 0).  Any such
// preimage yields the same future outputs as the true state (the outputs are
// digits of S), and after 24 steps the same lags and borrow.
PRNG_HD inline void lcg_to_swb(const uint32_t* s, uint32_t* lag) {
  uint32_t R[18];
#pragma unroll
  for (int k = 0; k < 18; ++k) R[k] = s[k];
#pragma unroll
  for (int it = 0; it < 3; ++it) {  // R = S + (R >> 336): a fixed point in <= 2 steps
    // R >> 336: bit 336 = limb 10 bit 16
    int64_t acc = 0;
    uint32_t nr[18];
#pragma unroll
    for (int k = 0; k < 18; ++k) {
      uint32_t q = 0;
      if (k + 10 < 18) q |= R[k + 10] >> 16;
      if (k + 11 < 18) q |= R[k + 11] << 16;
      acc += (int64_t)s[k] + (int64_t)q;
      nr[k] = (uint32_t)acc;
      acc >>= 32;
    }
#pragma unroll
    for (int k = 0; k < 18; ++k) R[k] = nr[k];
  }
#pragma unroll
  for (int j = 0; j < 24; ++j) {
    const int bit = 24 * j, k = bit >> 5, o = bit & 31;
    uint32_t v = R[k] >> o;
    if (o > 8) v |= R[k + 1] << (32 - o);
    lag[j] = v & 0xFFFFFFu;
  }
}

}  // namespace prng
