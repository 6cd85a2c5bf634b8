// Reference Philox-4x32-10 outputs from rocRAND's engine (host side).
// Reads "seed subsequence offset" triples from stdin and prints the four
// 32-bit outputs that start at that position of the stream.  Used only by
// the tests, to pin the two independent Philox implementations of the
// project (oracle and GPU library) to a published library.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
    unsigned long long seed, sub, off;
    while (std::scanf("%llu %llu %llu", &seed, &sub, &off) == 3) {
        rocrand_device::philox4x32_10_engine eng(seed, sub, off);
        unsigned a = eng.next(), b = eng.next(), c = eng.next(), d = eng.next();
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
