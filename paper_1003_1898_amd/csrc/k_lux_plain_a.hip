// Split plain RANLUX generation for luxury levels 24, 48, 97.
#include "lux_plain.h"

namespace prng {

bool launch_lux_plain_group_a(uint32_t p, uint32_t* st, const uint32_t* snap, uint64_t n, uint64_t draws, int dtype,
                              uint32_t S, uint32_t K, const uint32_t* digits, const uint32_t* aux, void* out,
                              uint64_t row_elems, uint64_t off, hipStream_t s, hipError_t* err) {
  switch (p) {
    case 24:
      *err = launch_lux_plain_p<24>(p, st, snap, n, draws, dtype, S, K, digits, aux, out, row_elems, off, s);
      return true;
    case 48:
      *err = launch_lux_plain_p<48>(p, st, snap, n, draws, dtype, S, K, digits, aux, out, row_elems, off, s);
      return true;
    case 97:
      *err = launch_lux_plain_p<97>(p, st, snap, n, draws, dtype, S, K, digits, aux, out, row_elems, off, s);
      return true;
    default:
      return false;
  }
}

}  // namespace prng
