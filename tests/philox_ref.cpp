// Philox4x32-10 outputs from rocRAND's implementation of the generator
// (Salmon et al., SC'11), an implementation independent of the oracle's: reads
// lines "c0 c1 c2 c3 k0 k1" (hex) and prints the four output words.  Host code
// only; used by the oracle tests.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

// the ten-round function is a protected member of the engine
struct Engine : rocrand_device::philox4x32_10_engine {
  using rocrand_device::philox4x32_10_engine::ten_rounds;
};

int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  Engine eng;
  while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    const uint4 r = eng.ten_rounds(uint4{c0, c1, c2, c3}, uint2{k0, k1});
    std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
