// Host-side driver around rocRAND's philox4x32_10 engine, used only as an independent
// reference for the oracle's Philox4x32-10 (the rocRAND engine is callable on the host).
// Input lines: key(64-bit) counter_lo64 counter_hi64  ->  output: four 32-bit words.
// The engine's state maps seed -> key, subsequence -> counter words (z, w) and
// offset/4 -> counter words (x, y).
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main() {
  unsigned long long key, lo, hi;
  while (std::scanf("%llu %llu %llu", &key, &lo, &hi) == 3) {
    rocrand_device::philox4x32_10_engine eng(key, hi, 4ull * lo);
    uint4 r = eng.next4();
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
