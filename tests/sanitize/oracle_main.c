/* Sanitizer driver for the oracle (test infrastructure): decodes random
 * frames of random small codes with decoders A, B and C in every dtype and
 * tree mode, so that an address or undefined-behaviour sanitizer build of
 * polar_oracle.c exercises every code path.  Exits 0 when every call
 * returns without a sanitizer report (reports abort the process). */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;

static uint64_t next_u64(void) { /* splitmix64 */
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static double uniform(void) { return (double)(next_u64() >> 11) * (1.0 / 9007199254740992.0); }

int main(void) {
    const int Ns[] = {2, 4, 8, 16, 32, 64, 128};
    const int Ls[] = {1, 2, 4, 8, 32};
    const int F = 3;
    int calls = 0;
    for (int trial = 0; trial < 40; ++trial) {
        const int N = Ns[next_u64() % 7];
        uint8_t* frozen = (uint8_t*)malloc((size_t)N);
        int K = 0;
        for (int i = 0; i < N; ++i) {
            frozen[i] = (uint8_t)(uniform() < 0.5);
            K += frozen[i] ? 0 : 1;
        }
        if (K == 0) {
            frozen[N - 1] = 0;
            K = 1;
        }
        const int r = K > 3 ? 3 : 0;
        const uint64_t poly = 0x3;
        for (int dtype = 0; dtype < 3; ++dtype) {
            const int es = dtype == 0 ? 4 : (dtype == 1 ? 2 : 1);
            uint8_t* llr = (uint8_t*)malloc((size_t)F * N * es);
            for (int i = 0; i < F * N; ++i) {
                const double v = (uniform() - 0.5) * 20.0;
                if (dtype == 0) ((float*)llr)[i] = (float)v;
                else if (dtype == 1) ((int16_t*)llr)[i] = (int16_t)(v * 3000.0);
                else ((int8_t*)llr)[i] = (int8_t)(next_u64() % 256 - 128); /* -128 too */
            }
            uint8_t* u = (uint8_t*)calloc((size_t)F * K, 1);
            uint8_t ok[3], nt[3];
            double pm[3], dist[3];
            for (int li = 0; li < 5; ++li) {
                const int L = Ls[li];
                for (int mode = 0; mode < 3; ++mode) {
                    if (orc_decode_tree(N, K, frozen, poly, r, L, dtype, (mode == 0 && li & 1) ? N : 4,
                                        mode, llr, F, u, ok, pm, nt, 1) < 0)
                        return 2;
                    ++calls;
                }
                if (orc_decode_scl(N, K, frozen, poly, r, L, dtype, llr, F, u, ok, pm, nt, 2) < 0)
                    return 3;
                int np = 0;
                uint8_t* cw = (uint8_t*)malloc((size_t)L * N);
                double* pms = (double*)malloc(sizeof(double) * (size_t)L);
                if (orc_decode_tree_list(N, K, frozen, L, dtype, 4, 0, llr, &np, cw, pms) < 0) return 4;
                free(cw);
                free(pms);
                calls += 2;
            }
            if (K - r <= 12) {
                if (orc_decode_ml(N, K, frozen, poly, r, dtype, llr, F, u, dist) < 0) return 5;
                ++calls;
            }
            free(u);
            free(llr);
        }
        free(frozen);
    }
    uint8_t bits[40];
    uint64_t rem = 0;
    for (int i = 0; i < 40; ++i) bits[i] = (uint8_t)(next_u64() & 1);
    if (orc_crc(bits, 40, 0x04C11DB7ull, 32, &rem) < 0) return 6;
    double m[9] = {0, -1, -1, -2, -0.5, -3, -1, 0, -2};
    int keep[9];
    if (orc_select(m, 9, 4, keep) < 0) return 7;
    printf("oracle sanitizer driver: %d decoder calls\n", calls);
    return 0;
}
