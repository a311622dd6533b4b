// Third, independent Philox4x32-10: PyTorch's header-only engine.
// Reads lines "seed c0 c1 c2 c3" (decimal) from stdin and prints the four
// output words.  The engine's counter is (offset lo, offset hi, subsequence lo,
// subsequence hi) and its key is the 64-bit seed.
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cinttypes>

int main() {
  unsigned long long seed, c0, c1, c2, c3;
  while (std::scanf("%llu %llu %llu %llu %llu", &seed, &c0, &c1, &c2, &c3) == 5) {
    const uint64_t offset = c0 | (c1 << 32);
    const uint64_t subseq = c2 | (c3 << 32);
    at::Philox4_32 engine(seed, subseq, offset);
    const uint32_t a = engine(), b = engine(), c = engine(), d = engine();
    std::printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
