// Host check of the jump-ahead data of libprng's jump.cpp.
//
// MT19937: prints "weight W" (nonzero coefficients of the characteristic polynomial),
// then one line per jump distance J: "J ok" when the window J words ahead
// built from x^J mod phi equals (a) the window reached by running the
// recurrence J more steps and, for J a multiple of 624, (b) the oracle's
// state after J draws.  The top bit is the only one of the window's first
// word that belongs to the state, so its low 31 bits are not compared.
//
// 48-bit LCGs: "lcg K ok" when, for kind K (7 DRAND48, 8 RANNYU), the map
// X -> A X + C of segment j (j L steps) applied to the oracle's starting state
// gives the oracle's state after j L draws, for several L and j.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "jump.h"

extern "C" {
uint32_t orc_next(int kind, uint32_t p, uint32_t r, uint32_t* st);
int orc_init(int kind, const uint64_t* seed, uint32_t* st);
}

static uint32_t step(const std::vector<uint32_t>& x, size_t n) {
  const uint32_t y = (x[n - 624] & 0x80000000u) | (x[n - 623] & 0x7FFFFFFFu);
  return x[n - 227] ^ (y >> 1) ^ ((y & 1u) ? 0x9908B0DFu : 0u);
}

static bool same_window(const uint32_t* a, const uint32_t* b) {
  if ((a[0] ^ b[0]) & 0x80000000u) return false;
  return memcmp(a + 1, b + 1, 623 * 4) == 0;
}

int main() {
  printf("weight %d\n", prng::mt_phi_weight());
  // window 0: the array init_genrand(19650218) leaves, before its first twist
  uint32_t st0[625];
  const uint64_t seed = 19650218u;
  if (orc_init(6, &seed, st0) != 0) return 1;
  const uint64_t Js[] = {1, 2, 3, 623, 624, 625, 1000, 19936, 19937, 19938, 62400, 624 * 255, 624 * 767};
  for (uint64_t J : Js) {
    std::vector<uint32_t> x(st0, st0 + 624);
    const size_t need = std::max<size_t>(J + 624, 624 + 19936 + 624);
    x.resize(need);
    for (size_t n = 624; n < need; ++n) x[n] = step(x, n);
    uint32_t poly[624];
    if (!prng::mt_jump_poly(J, poly)) {
      printf("%llu nopoly\n", (unsigned long long)J);
      continue;
    }
    uint32_t acc[624] = {0};
    for (int i = 0; i < 19937; ++i)
      if ((poly[i >> 5] >> (i & 31)) & 1u)
        for (int k = 0; k < 624; ++k) acc[k] ^= x[i + k];
    bool ok = same_window(acc, x.data() + J);
    if (J % 624 == 0) {
      uint32_t st[625];
      memcpy(st, st0, sizeof st);
      for (uint64_t d = 0; d < J; ++d) orc_next(6, 0, 24, st);
      ok = ok && st[624] == 624 && same_window(acc, st);
    }
    printf("%llu %s\n", (unsigned long long)J, ok ? "ok" : "FAIL");
  }
  // the segment table: slot j - 1 lists the exponents of x^(j L - 624)
  const uint64_t L = 624 * 256;
  std::vector<uint32_t> tab(3 * prng::jump_slot_words(6));
  bool ok = prng::fill_jumps(6, 0, L, 3, tab.data());
  for (uint32_t j = 1; j <= 3 && ok; ++j) {
    uint32_t poly[624], back[624] = {0};
    const uint32_t* slot = tab.data() + (j - 1) * prng::jump_slot_words(6);
    ok = prng::mt_jump_poly(j * L - 624, poly);
    uint32_t prev = 0;
    for (uint32_t q = 0; q < slot[0] && ok; ++q) {
      const uint32_t e = (slot[1 + q / 2] >> (16 * (q & 1))) & 0xFFFFu;
      ok = e < 19937 && (q == 0 || e > prev);  // ascending, in range
      back[e >> 5] |= 1u << (e & 31);
      prev = e;
    }
    ok = ok && memcmp(poly, back, sizeof poly) == 0;
  }
  printf("table %s\n", ok ? "ok" : "FAIL");
  for (int kind = 7; kind <= 8; ++kind) {
    bool good = true;
    const uint64_t seeds[] = {1, 0x330F, 0xFFFFFFFFFFFFull, 0x9E3779B97F4Bull};  // odd: valid for both
    for (uint64_t seed : seeds) {
      for (uint64_t L : {1ull, 384ull, 1000ull, 65536ull * 3}) {
        const uint32_t nj = 5, stride = prng::jump_slot_words(kind);
        std::vector<uint32_t> jd(nj * stride);
        good = good && prng::fill_jumps(kind, 0, L, nj, jd.data());
        uint32_t st0[2], st[2];
        if (orc_init(kind, &seed, st0) != 0) return 1;
        memcpy(st, st0, sizeof st);
        const uint64_t x0 = st0[0] | ((uint64_t)st0[1] << 32);
        for (uint32_t j = 1; j <= nj; ++j) {
          for (uint64_t d = 0; d < L; ++d) orc_next(kind, 0, 24, st);
          const uint32_t* w = jd.data() + (j - 1) * stride;
          const uint64_t A = w[0] | ((uint64_t)w[1] << 32), C = w[2] | ((uint64_t)w[3] << 32);
          const uint64_t x = (A * x0 + C) & 0xFFFFFFFFFFFFull;
          good = good && A < (1ull << 48) && C < (1ull << 48) && x == (st[0] | ((uint64_t)st[1] << 32));
        }
      }
    }
    printf("lcg%d %s\n", kind, good ? "ok" : "FAIL");
  }
  return 0;
}
