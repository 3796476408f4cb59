// Host-side cross-check of Philox4x32-10: reads "c0 c1 c2 c3 k0 k1" lines,
// prints the four output words from rocRAND's independent implementation.
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_kernel.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char** argv) {
  struct X : rocrand_device::philox4x32_10_engine { using rocrand_device::philox4x32_10_engine::ten_rounds; } e;
  unsigned v[6];
  while (scanf("%u %u %u %u %u %u", &v[0],&v[1],&v[2],&v[3],&v[4],&v[5]) == 6) {
    uint4 c = {v[0], v[1], v[2], v[3]}; uint2 k = {v[4], v[5]};
    uint4 r = e.ten_rounds(c, k);
    printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
