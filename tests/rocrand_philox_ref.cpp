// Independent Philox4x32-10 reference for the oracle pin: rocRAND's public
// host-callable generator.  Reads "c0 c1 c2 c3 k0 k1" lines (hex) on stdin and
// prints the four output words of the block at that counter and key.
//
// rocRAND's layout: key = seed; counter words 2,3 = subsequence; counter words
// 0,1 = offset / 4.  Offsets are 64-bit, so the two top bits of counter word
// 1 are added with extra skips of 2^63 numbers (= 2^61 blocks) each.
#include <rocrand/rocrand_kernel.h>

#include <cstdio>

int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    rocrand_state_philox4x32_10 st;
    unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
    unsigned long long sub = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
    unsigned long long off =
        4ull * ((unsigned long long)c0 | ((unsigned long long)(c1 & 0x3FFFFFFFu) << 32));
    rocrand_init(seed, sub, off, &st);
    for (unsigned i = 0; i < 2u * (c1 >> 30); ++i) skipahead(1ull << 63, &st);
    uint4 r = rocrand4(&st);
    std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
