// Reference Philox4x32-10 from PyTorch's header-only engine
// (ATen/core/PhiloxRNGEngine.h), used to cross-check the oracle's
// independent implementation.  Reads "c0 c1 c2 c3 k0 k1" per line (decimal
// uint32) and prints the four output words.  The engine's counter is
// (offset_lo, offset_hi, subsequence_lo, subsequence_hi) and its key is the
// 64-bit seed, so any counter/key pair maps onto its constructor.
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdint>
#include <cstdio>

int main() {
  unsigned long long c0, c1, c2, c3, k0, k1;
  while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint64_t seed = (uint64_t)k0 | ((uint64_t)k1 << 32);
    uint64_t sub = (uint64_t)c2 | ((uint64_t)c3 << 32);
    uint64_t off = (uint64_t)c0 | ((uint64_t)c1 << 32);
    at::Philox4_32 eng(seed, sub, off);
    uint32_t a = eng(), b = eng(), c = eng(), d = eng();
    std::printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
