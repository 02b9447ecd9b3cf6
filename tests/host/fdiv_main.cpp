// Host check of the launch-time divisor (gp_fdiv.hpp) against the hardware division:
// every divisor up to 5000 (and the powers of two and their neighbours up to 2^30) with
// numerators 0..2^16, the top of the range, and seeded numerators below 2^31.
// Prints "ok <checks>" or the first mismatch; exit status 1 on a mismatch.
#include <stdio.h>
#include <stdint.h>

#include "gp_fdiv.hpp"

using gpdbec::FDiv;

static uint64_t state = 0x9e3779b97f4a7c15ull;
static uint32_t next31() {  // splitmix64, top 31 bits
  state += 0x9e3779b97f4a7c15ull;
  uint64_t z = state;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return (uint32_t)((z ^ (z >> 31)) >> 33);
}

static long long checks = 0;
static int check(uint32_t d) {
  const FDiv f = gpdbec::fdiv_make(d);
  const uint32_t top = 0x7fffffffu;
  for (uint32_t n = 0; n <= 65536; ++n) {
    if (gpdbec::fdiv(n, f) != n / d) { printf("bad %u / %u\n", n, d); return 1; }
  }
  for (uint32_t k = 0; k < 4096; ++k) {
    const uint32_t n = top - k;
    if (gpdbec::fdiv(n, f) != n / d) { printf("bad %u / %u\n", n, d); return 1; }
    const uint32_t r = next31();
    if (gpdbec::fdiv(r, f) != r / d) { printf("bad %u / %u\n", r, d); return 1; }
    // multiples of d and their neighbours
    const uint64_t q = r / d;
    for (int64_t o = -1; o <= 1; ++o) {
      const int64_t n2 = (int64_t)(q * d) + o;
      if (n2 < 0 || n2 > (int64_t)top) continue;
      if (gpdbec::fdiv((uint32_t)n2, f) != (uint32_t)n2 / d) {
        printf("bad %lld / %u\n", (long long)n2, d);
        return 1;
      }
    }
  }
  checks += 65537 + 4096 * 5;
  return 0;
}

int main() {
  for (uint32_t d = 1; d <= 5000; ++d)
    if (check(d)) return 1;
  for (int b = 13; b <= 30; ++b)
    for (int64_t o = -1; o <= 1; ++o)
      if (check((uint32_t)((1ll << b) + o))) return 1;
  printf("ok %lld\n", checks);
  return 0;
}
