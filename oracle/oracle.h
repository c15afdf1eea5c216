/*
 * Test-infrastructure oracle for CRC-aided list decoding of polar codes
 * ("Fast List Decoders for Polar Codes", Sarkis, Giard, Vardy, Thibeault,
 * Gross).
 *
 * THIS IS TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It shares
 * no code, headers or tables with the HIP decoder.
 *
 * Three independent decoders are provided, all plain scalar C:
 *   A  orc_decode_tree  list decoding on the decoding tree with the
 *                       specialised constituent decoders (Sec. III; Rate-0,
 *                       Rate-1, repetition and SPC nodes), or with size-1
 *                       leaves only ("unrolled SC-list", Sec. VII-C, Table 1);
 *   B  orc_decode_scl   plain bit-by-bit LLR SC-list decoding (Sec. II-B,
 *                       eq. (sc-list:info)), a per-phase loop over stage
 *                       arrays with full path copies;
 *   C  orc_decode_ml    brute-force maximum-likelihood decoding over all
 *                       CRC-valid codewords (tiny codes only).
 *
 * Arithmetic domains (dtype):
 *   ORC_F32  LLRs are IEEE float32; F is exact, G is one float32 add, the
 *            penalty a node subtracts from a path metric is summed in double
 *            and rounded once to float32, the path-metric update is one
 *            float32 subtraction.
 *   ORC_I16  LLRs are int16 in [-32767, 32767]; G saturates to that range.
 *   ORC_I8   LLRs are int8 in [-127, 127]; G saturates to that range.
 *   Integer path metrics are exact integers.
 *
 * Conventions shared with the rest of the project (and stated again in each
 * function): a frozen_mask byte is 1 for a frozen position; the K unfrozen
 * positions carry, in increasing position order, the K-r payload bits followed
 * by the r CRC bits; the CRC register starts at zero, is fed MSB-first, is not
 * reflected and has no final XOR; poly is given in normal form without the
 * x^r term.
 *
 * Every entry point returns 0 on success and a negative value on invalid
 * arguments.  No entry point keeps state between calls.
 */
#ifndef POLAR_ORACLE_H
#define POLAR_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_F32 = 0, ORC_I16 = 1, ORC_I8 = 2 };
/* Tree modes: all four node classes; size-1 leaves only (plain SC-list on the
 * tree); Rate-0 and repetition nodes only (every other node split to size 1). */
enum { ORC_MODE_TREE = 0, ORC_MODE_SCL_LEAVES = 1, ORC_MODE_R0_REP = 2 };

/* CRC remainder of nbits bits (one bit per byte, values 0/1) under the
 * generator x^r + poly, register initialised to zero, fed MSB-first.
 * r in [1, 64].  Result in *rem. */
int orc_crc(const uint8_t* bits, int nbits, uint64_t poly, int r, uint64_t* rem);

/* In-place polar transform v <- v * F^{(x)n}, F = [[1,0],[1,1]], natural
 * order (Sec. II-A, Fig. 1).  N a power of two. The transform is an
 * involution over GF(2). */
int orc_polar_transform(uint8_t* v, int N);

/* Select the L best of n candidates (Alg. 1): best = larger metric, ties go to
 * the smaller enumeration index.  keep[] receives the survivors' enumeration
 * indices in slot order: best first when candidates were dropped (n > L),
 * enumeration order when all are kept.  Returns the number kept (min(n, L)). */
int orc_select(const double* pm, int n, int L, int* keep);

/*
 * Decoder A.  llr: F x N row-major in the dtype's storage type (float, int16_t,
 * int8_t).  Outputs (each nullable except u_hat):
 *   u_hat[F*K]   decided bits at the unfrozen positions, increasing order;
 *   crc_ok[F]    1 if the output path satisfies the CRC (always 1 if r == 0);
 *   pm[F]        path metric of the output path;
 *   near_tie[F]  1 if a float32 selection or the final pick was decided by a
 *                metric gap <= 1e-5 * |metric| (always 0 for integer dtypes).
 * spc_max: largest SPC node (4 = "Dec-SPC-4"; 0 disables SPC nodes).
 * mode: ORC_MODE_TREE, ORC_MODE_SCL_LEAVES or ORC_MODE_R0_REP.  threads: worker threads (<=0 =
 * one).
 */
int orc_decode_tree(int N, int K, const uint8_t* frozen_mask, uint64_t poly,
                    int r, int L, int dtype, int spc_max, int mode,
                    const void* llr, int64_t F, uint8_t* u_hat,
                    uint8_t* crc_ok, double* pm, uint8_t* near_tie,
                    int threads);

/* Decoder A on one frame, returning the whole final list: *n_paths paths, the
 * codeword (root output, N bytes each) and metric of each, in slot order. */
int orc_decode_tree_list(int N, int K, const uint8_t* frozen_mask, int L,
                         int dtype, int spc_max, int mode, const void* llr,
                         int* n_paths, uint8_t* codewords, double* pms);

/* Decoder B, same interface as decoder A. */
int orc_decode_scl(int N, int K, const uint8_t* frozen_mask, uint64_t poly,
                   int r, int L, int dtype, const void* llr, int64_t F,
                   uint8_t* u_hat, uint8_t* crc_ok, double* pm,
                   uint8_t* near_tie, int threads);

/* Decoder C.  Requires K - r <= 20.  dist[F] receives the minimum of
 * sum_i |llr_i| [x_i != h(llr_i)] over CRC-valid codewords (exact in double),
 * u_hat the first minimiser in payload enumeration order. */
int orc_decode_ml(int N, int K, const uint8_t* frozen_mask, uint64_t poly,
                  int r, int dtype, const void* llr, int64_t F,
                  uint8_t* u_hat, double* dist);

#ifdef __cplusplus
}
#endif

#endif
