// Independent Philox4x32-10 word generator used to pin the oracle's Philox.
// It calls rocRAND's open-source header engine through its public API:
// engine(seed, subsequence, offset) then next().  With
// subsequence = stream | (realization << 32) and offset = e, the engine's
// counter is (e >> 2, stream, realization) and next() returns word e & 3,
// which is the counter map the oracle documents.
// Usage: rocrand_philox_words SEED STREAM REALIZATION E0 COUNT
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdlib>

int main(int argc, char** argv) {
    if (argc != 6) return 2;
    unsigned long long seed = std::strtoull(argv[1], nullptr, 10);
    unsigned long long stream = std::strtoull(argv[2], nullptr, 10);
    unsigned long long real = std::strtoull(argv[3], nullptr, 10);
    unsigned long long e0 = std::strtoull(argv[4], nullptr, 10);
    long long count = std::strtoll(argv[5], nullptr, 10);
    rocrand_device::philox4x32_10_engine eng(seed, stream | (real << 32), e0);
    for (long long i = 0; i < count; ++i) std::printf("%u\n", eng.next());
    return 0;
}
