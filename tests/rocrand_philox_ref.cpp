// Independent Philox4x32-10 reference for the oracle's generator: calls the
// ten-round block function of the rocRAND library on the host.  Reads lines of
// "c0 c1 c2 c3 k0 k1" (decimal) from stdin, prints the four output words.
#include <rocrand/rocrand_kernel.h>

#include <cstdio>

struct Philox : rocrand_device::philox4x32_10_engine {
  using rocrand_device::philox4x32_10_engine::ten_rounds;
};

int main() {
  Philox e;
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint4 r = e.ten_rounds(uint4{c0, c1, c2, c3}, uint2{k0, k1});
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
