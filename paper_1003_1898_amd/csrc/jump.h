// Host-side jump-ahead parameters (see jump.cpp).
#pragma once

#include <stdint.h>

#include "internal.h"

namespace prng {

// a^e mod m for moduli below 2^32.
uint32_t powmod31(uint64_t a, uint64_t e, uint64_t m);
// T^J of the XOR128 transition as 128 rows of 4 words (row i: image of bit i).
void xor128_power(uint64_t J, uint32_t* out512);
// T^(2^k) for k = 0..kXorPow2-1, 512 words each (matrix k at out + 512 k).
void fill_xor128_pow2(uint32_t* out);
// out = A after B for two such matrices (out may alias).
void xor128_compose(const uint32_t* A, const uint32_t* B, uint32_t* out512);
// x^J mod (x^97 + x^64 - 1) over Z / 2^24: 97 coefficients.
void ranmar_power(uint64_t J, uint32_t* out97);
void ranmar_polymul(const uint32_t* a, const uint32_t* b, uint32_t* out97);
// J * 7654321 mod (2^24 - 3): how far C_n moves back in J steps.
uint32_t ranmar_c_shift(uint64_t J);
// J steps of X -> a X + c mod 2^48 as one map X -> A X + C.
void lcg48_power(uint64_t a, uint64_t c, uint64_t J, uint64_t* A, uint64_t* C);
// (2^-24)^e mod 2^576 - 2^240 + 1: the RANLUX core after e SWB steps.
void ranlux_power(uint64_t e, uint32_t* out18);
// b * b^-1 = 1 for the constants above.
bool ranlux_selfcheck();

// Words per jump slot of a kind (its jump data rounded up to 16 bytes).
inline uint32_t jump_slot_words(int kind) { return (uint32_t)((kJumpWords[kind] + 3) & ~3); }
// Jump data of segments j = 1..nj for segment length L (slot j - 1 at
// dst + (j - 1) * jump_slot_words(kind)).  RANLUX uses luxury level p;
// MT19937 needs L to be a multiple of 624, at least 1248, and stores the
// exponents of the set coefficients of x^J mod phi (word 0 their number,
// then 16-bit exponents two per word, low half first).  False if it cannot
// be built.
bool fill_jumps(int kind, uint32_t p, uint64_t L, uint32_t nj, uint32_t* dst);
// MT19937: x^J mod the characteristic polynomial of its 19937-bit state
// transition, as 624 words (coefficient i is bit i % 32 of word i / 32).
// Results are cached for the life of the process.
bool mt_jump_poly(uint64_t J, uint32_t* out624);
// Number of nonzero coefficients of that characteristic polynomial.
int mt_phi_weight();
// The 25 RANLUX core multipliers (2^-24)^d, d = 0..24, 18 words each.
void fill_ranlux_aux(uint32_t* dst);
// The block-jump table of luxury p (kLuxDigitWords words): entry (d, v) at
// dst + (d * 256 + v) * 18 is (2^-24)^(p v 256^d).
void fill_ranlux_digits(uint32_t p, uint32_t* dst);

}  // namespace prng
