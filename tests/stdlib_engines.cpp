// Independent reference sequences from the C++ standard library's predefined
// engines, compiled and run by tests/test_oracle_pins.py at test time (the
// library is run, never read).  Prints one line per engine:
//   <name> <seed> <first N outputs, space separated>
#include <cstdint>
#include <cstdio>
#include <random>

template <class E>
void dump(const char* name, unsigned long seed, int n) {
  E e(seed);
  std::printf("%s %lu", name, seed);
  for (int i = 0; i < n; ++i) std::printf(" %llu", (unsigned long long)e());
  std::printf("\n");
}

int main() {
  const unsigned long seeds[] = {1ul, 12345ul, 19780503ul, 2147483562ul, 987654321ul};
  const int n = 3000;
  for (unsigned long s : seeds) {
    dump<std::minstd_rand0>("minstd_rand0", s, n);
    dump<std::mt19937>("mt19937", s, n);
    dump<std::ranlux24_base>("ranlux24_base", s, n);
    dump<std::discard_block_engine<std::ranlux24_base, 48, 24>>("ranlux_p48", s, n);
    dump<std::discard_block_engine<std::ranlux24_base, 97, 24>>("ranlux_p97", s, n);
    dump<std::discard_block_engine<std::ranlux24_base, 223, 24>>("ranlux_p223", s, n);
    dump<std::discard_block_engine<std::ranlux24_base, 389, 24>>("ranlux_p389", s, n);
    dump<std::ranlux24>("ranlux24", s, n);
    dump<std::linear_congruential_engine<std::uint_fast32_t, 40014, 0, 2147483563>>("lcg40014", s, n);
    dump<std::linear_congruential_engine<std::uint_fast32_t, 40692, 0, 2147483399>>("lcg40692", s, n);
  }
  return 0;
}
