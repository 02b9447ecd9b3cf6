// Division by a divisor fixed at launch, by a multiply-high and a shift.
//
// For 0 <= n < 2^31 and a divisor d >= 1: with s = ceil(log2 d) and
// m = floor(2^32 (2^s - d) / d) + 1, the quotient is n / d = (mulhi(n, m) + n) >> s
// (Granlund and Montgomery, "Division by invariant integers using multiplication",
// PLDI 1994, the round-up multiplier with a 33-bit intermediate; mulhi(n, m) <= n keeps
// the sum below 2^32 for n < 2^31).  The run-time-length kernels index lines, butterflies
// and grid points with it instead of the integer division sequence.
//
// Plain C++ apart from the __host__ __device__ qualifiers, which a HIP translation unit
// defines before including this header.
#pragma once
#include <stdint.h>

namespace gpdbec {

struct FDiv {
  uint32_t d, m, s;
};

__host__ __device__ inline FDiv fdiv_make(uint32_t d) {
  FDiv f{d, 0u, 0u};
  if (d == 0) return f;  // never divided by: callers pass divisors >= 1
  uint32_t s = 0;
  while ((1ull << s) < (uint64_t)d) ++s;
  f.s = s;
  f.m = (uint32_t)((((1ull << 32) * ((1ull << s) - d)) / d) + 1);
  return f;
}

// n / d for 0 <= n < 2^31
__host__ __device__ inline uint32_t fdiv(uint32_t n, FDiv f) {
  const uint32_t hi = (uint32_t)(((uint64_t)n * f.m) >> 32);
  return (hi + n) >> f.s;
}

}  // namespace gpdbec
