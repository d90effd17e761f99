/*
 * CPU oracle for the uniform generators of Demchik, "Pseudo-random number
 * generators for Monte Carlo simulations on Graphics Processing Units"
 * (arXiv:1003.1898).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file.  It is used by the tests, by the smoke check and by the
 * CPU-baseline leg of the benchmark, and nowhere else.  It shares no code,
 * header, table or constant with the HIP implementation.
 *
 * Style: plain, slow, obviously correct.  Every generator keeps its state in
 * the canonical per-stream layout (32-bit words):
 *
 *   GGL      [x]                                   1 word
 *   XOR128   [x, y, z, w] = (X_{n-4}..X_{n-1})     4 words
 *   RANECU   [s1, s2]                              2 words
 *   RANMAR   [Y_{n-97} .. Y_{n-1}, C]             98 words (lags oldest first)
 *   RANLUX   [X_{n-24} .. X_{n-1}, c, k]          26 words (k = kept values
 *                                                   already taken from the
 *                                                   current luxury block)
 *   MT19937  [mt[0..623], index]                 625 words (block form)
 *   DRAND48  [x mod 2^32, x >> 32]                 2 words (48-bit LCG)
 *   RANNYU   [x mod 2^32, x >> 32]                 2 words (48-bit MLCG)
 *
 * Lag tables are kept as plain arrays with the oldest value first and are
 * shifted by one after every step, so that every recurrence reads exactly the
 * lags written in the paper's equations.
 *
 * Native integer draw u and its bit width b:
 *   GGL 31 (u in [1, 2^31-2]), XOR128 32, RANECU 31 (u in [1, 2147483562]),
 *   RANMAR 24, RANLUX 24, MT19937 32, DRAND48 and RANNYU 32 (the top 32 of the
 *   48 bits, u = x >> 16).
 * Conversions (the paper asks for exact use of several draws for double
 * precision, Section 3.1; the single-precision rule is this project's reading):
 *   f32 = (u >> (b-24)) * 2^-24                       exact, in [0, 1)
 *   f64 = ((u1 >> (b-27)) * 2^26 + (u2 >> (b-26))) * 2^-53   for b >= 27
 *       = (u1 * 2^24 + u2) * 2^-48                             for b == 24
 * A second single-precision rule, "paper", repeats the scalings written in
 * the paper's kernels (Sections 3.2-3.7) in fp32 arithmetic; see
 * orc_to_f32_paper.
 * Seeding procedures the paper omits (RANMAR, RANLUX, MT19937 lag tables) are
 * the published initialisers of those generators, written out below.
 *
 * Parity pins (tests/): known-answer values, brute-force periods, GF(2)
 * matrix identities for XOR128, the RANLUX/SWB sampling identity and
 * cross-checks against independently compiled library engines.
 */
#include <stdint.h>
#include <string.h>

enum {
  ORC_GGL = 1, ORC_XOR128 = 2, ORC_RANECU = 3, ORC_RANMAR = 4, ORC_RANLUX = 5, ORC_MT19937 = 6,
  ORC_DRAND48 = 7, ORC_RANNYU = 8
};
enum { ORC_U32 = 1, ORC_F32 = 2, ORC_F64 = 3, ORC_F32_PAPER = 4 };

int orc_state_words(int kind) {
  switch (kind) {
    case ORC_GGL: return 1;
    case ORC_XOR128: return 4;
    case ORC_RANECU: return 2;
    case ORC_RANMAR: return 98;
    case ORC_RANLUX: return 26;
    case ORC_MT19937: return 625;
    case ORC_DRAND48: return 2;
    case ORC_RANNYU: return 2;
  }
  return -1;
}

int orc_seed_words(int kind) {
  switch (kind) {
    case ORC_GGL: return 1;
    case ORC_XOR128: return 4;
    case ORC_RANECU: return 2;
    case ORC_RANMAR: return 2;
    case ORC_RANLUX: return 1;
    case ORC_MT19937: return 1;
    case ORC_DRAND48: return 1;
    case ORC_RANNYU: return 1;
  }
  return -1;
}

int orc_bits(int kind) {
  switch (kind) {
    case ORC_GGL: return 31;
    case ORC_XOR128: return 32;
    case ORC_RANECU: return 31;
    case ORC_RANMAR: return 24;
    case ORC_RANLUX: return 24;
    case ORC_MT19937: return 32;
    case ORC_DRAND48: return 32;
    case ORC_RANNYU: return 32;
  }
  return -1;
}

/* ------------------------------------------------------------------ GGL
 * Appendix A.1 (linear congruential generators): the minimal standard
 * multiplicative LCG, X_n = 16807 X_{n-1} mod (2^31 - 1).  Written as the plain
 * definition in 64-bit arithmetic. */
static uint32_t ggl_next(uint32_t *st) {
  uint64_t x = st[0];
  x = (16807u * x) % 2147483647u;
  st[0] = (uint32_t)x;
  return st[0];
}

/* --------------------------------------------------------------- XOR128
 * Appendix A.4.2 (XORShift), the component form of Marsaglia's XOR128:
 *   t = X_{n-4} ^ (X_{n-4} << 11)
 *   X_n = (X_{n-1} ^ (X_{n-1} >> 19)) ^ (t ^ (t >> 8)),
 * and the window moves by one.  The draw is the new X_n. */
static uint32_t xor128_next(uint32_t *st) {
  uint32_t x4 = st[0], x1 = st[3];
  uint32_t t = x4 ^ (x4 << 11);
  uint32_t xn = (x1 ^ (x1 >> 19)) ^ (t ^ (t >> 8));
  st[0] = st[1];
  st[1] = st[2];
  st[2] = st[3];
  st[3] = xn;
  return xn;
}

/* --------------------------------------------------------------- RANECU
 * Appendix A.4.1 (multiple recursive generators): two MLCGs
 * (a1 = 40014, m1 = 2147483563) and (a2 = 40692, m2 = 2147483399), each advanced
 * once, combined as X = X_1 - X_2 mod (m1 - 1), with m1 - 1 added when the
 * difference is <= 0.  Each MLCG is written as its plain definition. */
static uint32_t ranecu_next(uint32_t *st) {
  uint64_t s1 = st[0], s2 = st[1];
  s1 = (40014u * s1) % 2147483563u;
  s2 = (40692u * s2) % 2147483399u;
  st[0] = (uint32_t)s1;
  st[1] = (uint32_t)s2;
  int64_t z = (int64_t)s1 - (int64_t)s2;
  if (z <= 0) z += 2147483562;
  return (uint32_t)z;
}

/* --------------------------------------------------------------- RANMAR
 * Appendix A.4.4: Y_n = (Y_{n-97} - Y_{n-33}) mod 2^24,
 * C_n = (C_{n-1} - D) mod M with D = 7654321, M = 2^24 - 3,
 * X_n = (Y_n - C_n) mod 2^24.  All values are 24-bit integers (the paper's
 * floating-point version holds the same integers scaled by 2^-24). */
static uint32_t ranmar_next(uint32_t *st) {
  uint32_t *lag = st;        /* lag[t] = Y_{n-97+t} */
  int64_t y = (int64_t)lag[0] - (int64_t)lag[64];
  if (y < 0) y += 16777216;
  memmove(lag, lag + 1, 96 * sizeof(uint32_t));
  lag[96] = (uint32_t)y;
  int64_t c = (int64_t)st[97] - 7654321;
  if (c < 0) c += 16777213;
  st[97] = (uint32_t)c;
  int64_t x = y - c;
  if (x < 0) x += 16777216;
  return (uint32_t)x;
}

/* RMARIN (James' initialiser, which the paper runs once per instance and does
 * not print, Section 3.5): two seeds ij in [0, 31328], kl in [0, 30081] fill
 * 97 lag values of 24 bits each, most significant bit first; C_0 = 362436. */
static void ranmar_init(uint32_t ij, uint32_t kl, uint32_t *st) {
  uint32_t u[98];
  int64_t i = (ij / 177) % 177 + 2;
  int64_t j = ij % 177 + 2;
  int64_t k = (kl / 169) % 178 + 1;
  int64_t l = kl % 169;
  for (int ii = 1; ii <= 97; ++ii) {
    uint32_t s = 0;
    for (int jj = 1; jj <= 24; ++jj) {
      int64_t m = (((i * j) % 179) * k) % 179;
      i = j;
      j = k;
      k = m;
      l = (53 * l + 1) % 169;
      if ((l * m) % 64 >= 32) s |= 1u << (24 - jj);
    }
    u[ii] = s;
  }
  /* James' generator starts with u[97] as Y_{n-97} and u[33] as Y_{n-33}, and
   * steps both indices downwards: the oldest lag is u[97], the newest u[1]. */
  for (int t = 0; t < 97; ++t) st[t] = u[97 - t];
  st[97] = 362436;
}

/* --------------------------------------------------------------- RANLUX
 * Appendix A.4.5-A.4.6.  The subtract-with-borrow core RCARRY with m = 2^24,
 * r = 24, s = 10 in the variant X_n = (X_{n-10} - X_{n-24} - c) mod 2^24,
 * c = 1 when the difference is negative (the paper notes both operand orders
 * of SWB; this is the order of James' RCARRY and of the published check
 * values).  RANLUX keeps `r` values and then discards the next p - r. */
static uint32_t swb_step(uint32_t *st) {
  uint32_t *lag = st;        /* lag[t] = X_{n-24+t} */
  int64_t d = (int64_t)lag[14] - (int64_t)lag[0] - (int64_t)st[24];
  uint32_t c = d < 0 ? 1u : 0u;
  if (d < 0) d += 16777216;
  memmove(lag, lag + 1, 23 * sizeof(uint32_t));
  lag[23] = (uint32_t)d;
  st[24] = c;
  return (uint32_t)d;
}

static uint32_t ranlux_next(uint32_t *st, uint32_t p, uint32_t r) {
  if (st[25] == r) {                 /* block of r kept values done: discard */
    for (uint32_t i = 0; i < p - r; ++i) swb_step(st);
    st[25] = 0;
  }
  st[25] += 1;
  return swb_step(st);
}

/* Seeding of the lag table (not given in the paper, Section 3.6): the
 * initialiser of the ISO C++ subtract_with_carry_engine, i.e. 24 successive
 * draws of the MLCG (40014, 2147483563) started at v, each reduced mod 2^24,
 * oldest first, and the borrow set when the newest lag is zero. */
static void ranlux_init(uint32_t v, uint32_t *st) {
  uint64_t x = v;
  for (int t = 0; t < 24; ++t) {
    x = (40014u * x) % 2147483563u;
    st[t] = (uint32_t)(x % 16777216u);
  }
  st[24] = st[23] == 0 ? 1u : 0u;
  st[25] = 0;
}

/* -------------------------------------------------------------- MT19937
 * Appendix A.4.3: TGFSR recurrence
 *   X_{n+624} = X_{n+397} ^ ((X_n & upper) | (X_{n+1} & lower)) A
 * with w = 32, u = 31, a = 0x9908B0DF, and tempering (m, d/b, e/c, l) =
 * (11, 7/0x9D2C5680, 15/0xEFC60000, 18).  The 624 values are updated in place
 * in index order when a block is used up, so X_{n+1} and X_{n+397} are already
 * new for the last entries, exactly as the recurrence requires. */
static void mt_twist(uint32_t *mt) {
  for (int n = 0; n < 624; ++n) {
    uint32_t y = (mt[n] & 0x80000000u) | (mt[(n + 1) % 624] & 0x7FFFFFFFu);
    uint32_t ya = (y >> 1) ^ ((y & 1u) ? 0x9908B0DFu : 0u);
    mt[n] = mt[(n + 397) % 624] ^ ya;
  }
}

static uint32_t mt_next(uint32_t *st) {
  if (st[624] >= 624) {
    mt_twist(st);
    st[624] = 0;
  }
  uint32_t t = st[st[624]];
  st[624] += 1;
  t ^= t >> 11;
  t ^= (t << 7) & 0x9D2C5680u;
  t ^= (t << 15) & 0xEFC60000u;
  t ^= t >> 18;
  return t;
}

/* Seeding (not given in the paper, Section 3.7): Matsumoto-Nishimura
 * init_genrand, mt[i] = 1812433253 (mt[i-1] ^ (mt[i-1] >> 30)) + i. */
static void mt_init(uint32_t s, uint32_t *st) {
  st[0] = s;
  for (uint32_t i = 1; i < 624; ++i) st[i] = 1812433253u * (st[i - 1] ^ (st[i - 1] >> 30)) + i;
  st[624] = 624;
}

/* ------------------------------------------------------- 48-bit LCGs
 * Appendix A.1, the LCG of equation (LCG) with modulus 2^48:
 *   DRAND48  X_n = (25214903917 X_{n-1} + 11) mod 2^48   (equation DRAND48)
 *   RANNYU   X_n = 31167285 X_{n-1} mod 2^48            (Section 2, Chroma;
 *            no increment is given, so c = 0: an MLCG, equation MLCG)
 * The state is X as two words (low 32 bits, high 16 bits).  The product is
 * formed in 64-bit unsigned arithmetic, which is exact modulo 2^64 and hence
 * modulo 2^48 after the mask.  The draw is the top 32 bits, X >> 16: the low
 * bits of a power-of-two-modulus LCG have short periods (bit k repeats after
 * 2^(k+1) steps) and are dropped, as the C library's jrand48 does. */
static uint32_t lcg48_next(uint32_t *st, uint64_t a, uint64_t c) {
  uint64_t x = (uint64_t)st[0] | ((uint64_t)st[1] << 32);
  x = (a * x + c) & 0xFFFFFFFFFFFFull;
  st[0] = (uint32_t)x;
  st[1] = (uint32_t)(x >> 32);
  return (uint32_t)(x >> 16);
}

/* ------------------------------------------------------------ interface */

/* One draw of the native integer sequence; advances the canonical state. */
uint32_t orc_next(int kind, uint32_t p, uint32_t r, uint32_t *st) {
  switch (kind) {
    case ORC_GGL: return ggl_next(st);
    case ORC_XOR128: return xor128_next(st);
    case ORC_RANECU: return ranecu_next(st);
    case ORC_RANMAR: return ranmar_next(st);
    case ORC_RANLUX: return ranlux_next(st, p, r);
    case ORC_MT19937: return mt_next(st);
    case ORC_DRAND48: return lcg48_next(st, 25214903917ull, 11u);
    case ORC_RANNYU: return lcg48_next(st, 31167285u, 0u);
  }
  return 0;
}

/* Canonical state from one stream's mapped seed tuple.  Returns 0, or -1 when
 * a seed word lies outside the generator's valid range. */
int orc_init(int kind, const uint64_t *seed, uint32_t *st) {
  switch (kind) {
    case ORC_GGL:
      if (seed[0] < 1 || seed[0] > 2147483646u) return -1;
      st[0] = (uint32_t)seed[0];
      return 0;
    case ORC_XOR128:
      for (int i = 0; i < 4; ++i)
        if (seed[i] > 0xFFFFFFFFu) return -1;
      if ((seed[0] | seed[1] | seed[2] | seed[3]) == 0) return -1;
      for (int i = 0; i < 4; ++i) st[i] = (uint32_t)seed[i];
      return 0;
    case ORC_RANECU:
      if (seed[0] < 1 || seed[0] > 2147483562u) return -1;
      if (seed[1] < 1 || seed[1] > 2147483398u) return -1;
      st[0] = (uint32_t)seed[0];
      st[1] = (uint32_t)seed[1];
      return 0;
    case ORC_RANMAR:
      if (seed[0] > 31328 || seed[1] > 30081) return -1;
      ranmar_init((uint32_t)seed[0], (uint32_t)seed[1], st);
      return 0;
    case ORC_RANLUX:
      if (seed[0] < 1 || seed[0] > 2147483562u) return -1;
      ranlux_init((uint32_t)seed[0], st);
      return 0;
    case ORC_MT19937:
      if (seed[0] > 0xFFFFFFFFu) return -1;
      mt_init((uint32_t)seed[0], st);
      return 0;
    case ORC_DRAND48:
    case ORC_RANNYU:
      /* the seed is X_0 itself; the multiplicative generator takes odd seeds
       * only (an even X_0 shortens its period modulo a power of two) */
      if (seed[0] > 0xFFFFFFFFFFFFull) return -1;
      if (kind == ORC_RANNYU && (seed[0] & 1u) == 0) return -1;
      st[0] = (uint32_t)seed[0];
      st[1] = (uint32_t)(seed[0] >> 32);
      return 0;
  }
  return -1;
}

float orc_to_f32(int kind, uint32_t u) {
  int b = orc_bits(kind);
  uint32_t k = u >> (b - 24);
  return (float)k * 0x1p-24f;
}

/* The paper's own single-precision scalings, evaluated as written in fp32
 * (the integer converted to float with rounding to nearest, then the stated
 * operation with the stated constant rounded to float):
 *   GGL      x / 2147483647.0            (Section 3.2, constant PM_m_FP)
 *   XOR128   w / 4294967295.0            (Section 3.3, XR_m)
 *   RANECU   Z * (1.0 / 2147483648.0)    (Section 3.4, RETWOM31)
 *   RANMAR   X * 2^-24: the paper works on floats that are multiples of
 *            2^-24 throughout (RM_CD, RM_CM), so its output is exact
 *   RANLUX   X * 2^-24                   (Section 3.6, RLTWOM24)
 *   MT19937  (y + 0.5) / 4294967296.0    (Section 3.7, MTSEEDP4, MTSEEDP5)
 * Rounding reaches 1.0 for GGL, XOR128 and MT19937 (not RANECU, whose
 * largest value 2^31 - 86 rounds down).  The paper
 * gives no float rule for DRAND48 and RANNYU; -1 is returned for them. */
float orc_to_f32_paper(int kind, uint32_t u) {
  switch (kind) {
    case ORC_GGL: return (float)u / 2147483647.0f;
    case ORC_XOR128: return (float)u / 4294967295.0f;
    case ORC_RANECU: return (float)u * (1.0f / 2147483648.0f);
    case ORC_RANMAR: return (float)u / 16777216.0f;
    case ORC_RANLUX: return (float)u * 0x1p-24f;
    case ORC_MT19937: return ((float)u + 0.5f) / 4294967296.0f;
  }
  return -1.0f;
}

double orc_to_f64(int kind, uint32_t u1, uint32_t u2) {
  int b = orc_bits(kind);
  if (b == 24) return (double)(((uint64_t)u1 << 24) | u2) * 0x1p-48;
  uint64_t m = ((uint64_t)(u1 >> (b - 27)) << 26) | (uint64_t)(u2 >> (b - 26));
  return (double)m * 0x1p-53;
}

/* Plain bulk generation: for each of n streams (states at st + s*W), the next
 * `count` elements, stream-major (out[s*count + i]).  f64 elements take two
 * consecutive draws each. */
void orc_generate(int kind, uint32_t p, uint32_t r, uint64_t n, uint32_t *states, uint64_t count,
                  int dtype, void *out) {
  int W = orc_state_words(kind);
  for (uint64_t s = 0; s < n; ++s) {
    uint32_t *st = states + s * (uint64_t)W;
    for (uint64_t i = 0; i < count; ++i) {
      uint64_t o = s * count + i;
      if (dtype == ORC_U32) {
        ((uint32_t *)out)[o] = orc_next(kind, p, r, st);
      } else if (dtype == ORC_F32) {
        ((float *)out)[o] = orc_to_f32(kind, orc_next(kind, p, r, st));
      } else if (dtype == ORC_F32_PAPER) {
        ((float *)out)[o] = orc_to_f32_paper(kind, orc_next(kind, p, r, st));
      } else {
        uint32_t u1 = orc_next(kind, p, r, st);
        uint32_t u2 = orc_next(kind, p, r, st);
        ((double *)out)[o] = orc_to_f64(kind, u1, u2);
      }
    }
  }
}

/* The in-kernel consumer (Section 3.1: numbers used where they are produced,
 * never stored): per stream, the exact integer sum of the 24-bit mantissas
 * k = u >> (b-24) of `draws` single-precision uniforms, and a 64-bin histogram
 * with bin = k >> 18, i.e. [j/64, (j+1)/64). */
void orc_fused(int kind, uint32_t p, uint32_t r, uint64_t n, uint32_t *states, uint64_t draws,
               uint64_t *sum, uint32_t *hist) {
  int W = orc_state_words(kind);
  int b = orc_bits(kind);
  for (uint64_t s = 0; s < n; ++s) {
    uint32_t *st = states + s * (uint64_t)W;
    uint64_t acc = 0;
    uint32_t *h = hist + s * 64;
    for (int j = 0; j < 64; ++j) h[j] = 0;
    for (uint64_t i = 0; i < draws; ++i) {
      uint32_t k = orc_next(kind, p, r, st) >> (b - 24);
      acc += k;
      h[k >> 18] += 1;
    }
    sum[s] = acc;
  }
}

/* The paper's CPU benchmark shape (Section 4): one stream, one number per
 * call, the single-precision values summed.  Returns the sum; advances st. */
double orc_sum_f32(int kind, uint32_t p, uint32_t r, uint32_t *st, uint64_t count) {
  double acc = 0.0;
  for (uint64_t i = 0; i < count; ++i) acc += orc_to_f32(kind, orc_next(kind, p, r, st));
  return acc;
}

/* Brute-force period of GGL from x0 (Appendix A.1 gives 2^31 - 2). */
uint64_t orc_ggl_period(uint32_t x0) {
  uint32_t st = x0;
  uint64_t n = 0;
  do {
    ggl_next(&st);
    ++n;
  } while (st != x0 && n < (1ull << 32));
  return n;
}

/* Brute-force period of the RANMAR arithmetic sequence C_n (Appendix A.4.4:
 * modulus M = 2^24 - 3, step D = 7654321). */
uint64_t orc_ranmar_c_period(uint32_t c0) {
  int64_t c = c0;
  uint64_t n = 0;
  do {
    c -= 7654321;
    if (c < 0) c += 16777213;
    ++n;
  } while (c != (int64_t)c0 && n < (1ull << 32));
  return n;
}
