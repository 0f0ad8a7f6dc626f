// Prints the first 4 * BLOCKS outputs of rocRAND's Philox4x32-10 engine
// (rocrand_device::philox4x32_10_engine, the library's open-source header)
// for a seed, one 32-bit word per line: an implementation independent of the
// oracle's, used as a known-answer source by the tests.
#include <cstdio>
#include <cstdlib>

#include <rocrand/rocrand_philox4x32_10.h>

int main(int argc, char **argv)
{
    const unsigned long long seed = argc > 1 ? strtoull(argv[1], nullptr, 0) : 0ull;
    const int blocks = argc > 2 ? atoi(argv[2]) : 16;
    rocrand_device::philox4x32_10_engine eng(seed, 0, 0);
    for (int k = 0; k < 4 * blocks; ++k) printf("%u\n", eng());
    return 0;
}
