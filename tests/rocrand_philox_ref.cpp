// Third-party reference for the Philox4x32-10 pin: rocRAND's engine, built
// for the host.  Reads lines "w0 w1 w2 w3 k0 k1" (decimal counter words and
// key words) and prints the four output words of that counter.  rocRAND's
// engine keeps counter words (0,1) as a 64-bit offset in units of four
// outputs and words (2,3) as the subsequence, so counter (w0,w1,w2,w3) is
// reached with offset 4*(w0 + 2^32 w1) and subsequence w2 + 2^32 w3.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
  unsigned long long w0, w1, w2, w3, k0, k1;
  while (std::scanf("%llu %llu %llu %llu %llu %llu", &w0, &w1, &w2, &w3, &k0, &k1) == 6) {
    rocrand_device::philox4x32_10_engine e(k0 | (k1 << 32), w2 | (w3 << 32),
                                           4ull * (w0 | (w1 << 32)));
    unsigned a = e(), b = e(), c = e(), d = e();
    std::printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
