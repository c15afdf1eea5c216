// Sanitizer driver for the library's host-side plan compiler (decoding-tree
// classification, operation schedule, codeword-domain CRC table): random
// frozen masks of every length, every list size and mode, so that an
// address or undefined-behaviour sanitizer build of schedule.cpp exercises
// every code path.  Exits 0 when no sanitizer reports (reports abort).
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

#include "schedule.h"

int main() {
    std::mt19937_64 rng(12345);
    int built = 0;
    for (int n = 1; n <= 12; ++n) {
        const int N = 1 << n;
        for (int trial = 0; trial < 12; ++trial) {
            std::vector<uint8_t> frozen(N);
            const double p = (trial % 4) / 3.0;
            int K = 0;
            for (int i = 0; i < N; ++i) {
                frozen[i] = (uint8_t)(std::uniform_real_distribution<double>(0, 1)(rng) < p);
                K += frozen[i] ? 0 : 1;
            }
            for (int L : {1, 2, 4, 8, 16, 32, 64, 128}) {
                for (int mode : {0, 1}) {
                    for (int spc : {4, N}) {
                        std::vector<pscl::SchedOp> ops;
                        if (!pscl::build_schedule(N, frozen.data(), L, spc, mode, ops)) return 2;
                        ++built;
                    }
                }
            }
            for (int r : {1, 8, 32, 64}) {
                if (K >= r) {
                    auto t = pscl::crc_codeword_table(N, frozen.data(), 0x04C11DB7ull & ((r == 64) ? ~0ull : ((1ull << r) - 1)), r);
                    if ((int)t.size() != N) return 3;
                }
            }
        }
    }
    std::printf("schedule sanitizer driver: %d schedules\n", built);
    return 0;
}
