// Test-only harness: prints raw Philox4x32-10 blocks computed by PyTorch's
// own header-only engine (ATen/core/PhiloxRNGEngine.h), an implementation
// independent of the oracle.  Reads lines "c0 c1 c2 c3 k0 k1" (decimal) on
// stdin and prints "o0 o1 o2 o3".
//
// The engine's constructor takes (seed, subsequence, offset) and forms the
// key (lo32(seed), hi32(seed)) and counter (lo32(offset), hi32(offset),
// lo32(subsequence), hi32(subsequence)); its first four outputs are the four
// words of one block.
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cstdint>

int main() {
  unsigned long long c0, c1, c2, c3, k0, k1;
  while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint64_t seed = (uint64_t)k0 | ((uint64_t)k1 << 32);
    uint64_t sub = (uint64_t)c2 | ((uint64_t)c3 << 32);
    uint64_t off = (uint64_t)c0 | ((uint64_t)c1 << 32);
    at::philox_engine eng(seed, sub, off);
    uint32_t o[4];
    for (int i = 0; i < 4; ++i) o[i] = eng();
    std::printf("%u %u %u %u\n", o[0], o[1], o[2], o[3]);
  }
  return 0;
}
