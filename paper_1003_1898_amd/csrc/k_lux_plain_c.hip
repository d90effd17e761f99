// Split plain RANLUX generation for luxury levels 120, 240, 408.
#include "lux_plain.h"

namespace prng {

bool launch_lux_plain_group_c(uint32_t p, uint32_t* st, const uint32_t* snap, uint64_t n, uint64_t draws, int dtype,
                              uint32_t S, uint32_t K, const uint32_t* digits, const uint32_t* aux, void* out,
                              uint64_t row_elems, uint64_t off, hipStream_t s, hipError_t* err) {
  switch (p) {
    case 120:
      *err = launch_lux_plain_p<120>(p, st, snap, n, draws, dtype, S, K, digits, aux, out, row_elems, off, s);
      return true;
    case 240:
      *err = launch_lux_plain_p<240>(p, st, snap, n, draws, dtype, S, K, digits, aux, out, row_elems, off, s);
      return true;
    case 408:
      *err = launch_lux_plain_p<408>(p, st, snap, n, draws, dtype, S, K, digits, aux, out, row_elems, off, s);
      return true;
    default:
      return false;
  }
}

}  // namespace prng
