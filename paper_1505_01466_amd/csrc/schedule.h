// Host-side plan compiler for the list decoder: decoding-tree classification,
// the unrolled operation schedule, and the CRC syndrome table.
#pragma once

#include <cstdint>
#include <vector>

namespace pscl {

enum OpType : uint8_t {
    OP_F = 0,
    OP_G = 1,
    OP_COMB = 2,
    OP_R0 = 3,
    OP_REP = 4,
    OP_R1 = 5,
    OP_SPC = 6,
};

// One operation of the unrolled decoder (Listing 2 shows the (8, 4) case).
//   k:     log2 of the node size N_v the operation belongs to.
//   side:  0 if the node is a left child (its output feeds G and Combine of
//          its parent), 1 if it is a right child or the root.
//   cand:  candidates generated per source path (leaf operations).
//   paths: active paths after the operation.
struct SchedOp {
    uint8_t type;
    uint8_t k;
    uint8_t side;
    uint8_t cand;
    int paths;
};

// Decoding-tree modes: see pscl_mode in pscl.h.
constexpr int MODE_TREE = 0;
constexpr int MODE_SCL_LEAVES = 1;

// Builds the schedule for a code of length N = 2^n; returns false on invalid
// input.  The tree is walked depth first; a node is replaced by a list
// decoder when its frozen pattern makes it a Rate-0, Rate-1, repetition or
// (4 <= N_v <= spc_max) SPC constituent code (Sec. II-C, Sec. II-D).
bool build_schedule(int N, const uint8_t* frozen, int L, int spc_max, int mode,
                    std::vector<SchedOp>& out);

// Candidates per source path for a leaf operation (Sec. III): Rate-0 keeps
// its one word, repetition has two, a single information bit two, Rate-1
// (N_v >= 2) four, SPC eight (two when L = 2).
int leaf_candidates(int type, int k, int L);

// CRC check in the codeword domain.  With u = x G_N and the CRC of the K
// unfrozen bits linear in u, the check is linear in x: the register value
// after feeding all K bits (payload then CRC field) equals the XOR of
// table[i] over the positions i where x_i = 1, and the CRC holds iff that
// XOR is zero.  Requires 1 <= r <= 64.
std::vector<uint64_t> crc_codeword_table(int N, const uint8_t* frozen, uint64_t poly, int r);

}  // namespace pscl
