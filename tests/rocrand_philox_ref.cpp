// Reference Philox4x32-10 outputs from rocRAND's host-callable engine.
// Test helper only: reads "c0 c1 c2 c3 k0 k1" per line on stdin and prints the
// four output words of the block at that counter under that key.  rocRAND
// places the counter as (offset/4 low, offset/4 high, subsequence low,
// subsequence high), so the engine is seeded to land exactly on the counter.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main() {
  unsigned int c0, c1, c2, c3, k0, k1;
  while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    unsigned long long seed = (static_cast<unsigned long long>(k1) << 32) | k0;
    unsigned long long subseq = (static_cast<unsigned long long>(c3) << 32) | c2;
    unsigned long long block = (static_cast<unsigned long long>(c1) << 32) | c0;
    rocrand_device::philox4x32_10_engine eng(seed, subseq, 0);
    // discard() takes a count of 32-bit outputs; step in pieces so that the
    // count never overflows 64 bits
    while (block > 0) {
      unsigned long long step = block < (1ull << 60) ? block : (1ull << 60);
      eng.discard(step * 4ull);
      block -= step;
    }
    unsigned int w0 = eng.next(), w1 = eng.next(), w2 = eng.next(), w3 = eng.next();
    std::printf("%u %u %u %u\n", w0, w1, w2, w3);
  }
  return 0;
}
