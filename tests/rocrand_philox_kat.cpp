// Host-side known-answer helper: reads "c0 c1 c2 c3 k0 k1" (hex) lines and
// prints the first output block of rocRAND's open-source Philox4x32-10
// engine positioned at that counter (c1 must be below 2^30 so that the
// engine's 64-bit offset, 4 * (c1:c0), does not overflow).
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
    unsigned long long subsequence = ((unsigned long long)c3 << 32) | c2;
    unsigned long long offset = 4ull * (((unsigned long long)c1 << 32) | c0);
    rocrand_device::philox4x32_10_engine engine(seed, subsequence, offset);
    uint4 r = engine.next4();
    std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
