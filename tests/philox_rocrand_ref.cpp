// Independent Philox4x32-10 for the oracle's pin: rocRAND's host/device
// implementation, driven through its public API.  Reads lines
// "c0 c1 c2 c3 k0 k1" and prints the four output words of the block at that
// counter and key.  rocRAND addresses the counter as (offset / 4) in the low
// two words and the subsequence in the high two words; offsets must stay
// below 2**64, so c1 < 2**30.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char** argv) {
  unsigned c0,c1,c2,c3,k0,k1;
  while (scanf("%u %u %u %u %u %u", &c0,&c1,&c2,&c3,&k0,&k1) == 6) {
    rocrand_state_philox4x32_10 st;
    unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
    unsigned long long off = (((unsigned long long)c1 << 32) | c0) * 4ull;
    unsigned long long sub = ((unsigned long long)c3 << 32) | c2;
    rocrand_init(seed, sub, off, &st);
    uint4 r = rocrand4(&st);
    printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
