// Prints Philox4x32-10(counter, key) as computed by rocRAND's host-callable
// engine, one 32-bit word per line.  Used only by the oracle pin tests as an
// independent library implementation of the generator.
//   usage: rocrand_philox_ref c0 c1 c2 c3 k0 k1     (c1 < 2^30)
// rocRAND's engine takes (seed, subsequence, offset): key = seed, counter
// words 2-3 = subsequence, counter words 0-1 = offset / 4.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>
#include <cstdlib>

int main(int argc, char** argv) {
  if (argc != 7) return 2;
  unsigned long long c[4], k[2];
  for (int i = 0; i < 4; ++i) c[i] = strtoull(argv[1 + i], nullptr, 0);
  for (int i = 0; i < 2; ++i) k[i] = strtoull(argv[5 + i], nullptr, 0);
  if (c[1] >= (1ull << 30)) return 3;
  unsigned long long seed = k[0] | (k[1] << 32);
  unsigned long long sub = c[2] | (c[3] << 32);
  unsigned long long off = (c[0] | (c[1] << 32)) * 4ull;
  rocrand_device::philox4x32_10_engine e(seed, sub, off);
  for (int i = 0; i < 4; ++i) printf("%u\n", e.next());
  return 0;
}
