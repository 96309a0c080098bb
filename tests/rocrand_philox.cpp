// rocRAND's own Philox4x32-10 engine (the header-only engine its generators
// run), called on the host: an implementation independent of the oracle's
// and the library's, against which tests check the oracle's Philox.  Test
// infrastructure; built by the test that uses it.
#include <rocrand/rocrand_kernel.h>
#include <stdint.h>

// n successive 32-bit outputs of the engine seeded with `seed`, started at
// `subsequence` and `offset` (in outputs), into out[0..n).
extern "C" void rr_philox(unsigned long long seed, unsigned long long subsequence,
                          unsigned long long offset, uint32_t n, uint32_t *out) {
  rocrand_state_philox4x32_10 st;
  rocrand_init(seed, subsequence, offset, &st);
  for (uint32_t i = 0; i < n; ++i) out[i] = rocrand(&st);
}
