// Known-answer generator for Philox4x32-10 built from rocRAND's header.
// The test-suite compiles this host program (hipcc, host code only) and
// compares its output with the oracle's Philox for random counters and keys,
// so the oracle's generator is pinned to an independent library
// implementation.  Input lines: c0 c1 c2 c3 k0 k1 (hex); output: the four
// result words.  rocRAND addresses the counter as (offset/4 in words 0-1,
// subsequence in words 2-3) with the key taken from the 64-bit seed, so
// counter word 1 must stay below 2^30 for offset*4 to fit 64 bits.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main() {
  unsigned c[4], k[2];
  while (std::scanf("%x %x %x %x %x %x", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
    unsigned long long seed = ((unsigned long long)k[1] << 32) | k[0];
    unsigned long long sub = ((unsigned long long)c[3] << 32) | c[2];
    unsigned long long off = (((unsigned long long)c[1] << 32) | c[0]) * 4ULL;
    rocrand_device::philox4x32_10_engine e(seed, sub, off);
    unsigned a = e(), b = e(), d = e(), f = e();
    std::printf("%08x %08x %08x %08x\n", a, b, d, f);
  }
  return 0;
}
