// Host-side plan compiler: decoding-tree classification (Sec. II-C/II-D), the
// unrolled operation sequence (Listing 2), and the codeword-domain CRC table.
#include "schedule.h"

#include <algorithm>

namespace pscl {

namespace {

struct Walker {
    const uint8_t* frozen;
    int L;
    int spc_max;
    int mode;
    std::vector<SchedOp>* out;

    // Node class of the constituent code at [off, off + 2^k).
    int classify(int off, int k) const {
        const int nv = 1 << k;
        int nf = 0;
        for (int i = 0; i < nv; ++i) nf += frozen[off + i] ? 1 : 0;
        if (nv == 1) return nf ? OP_R0 : OP_R1;
        if (mode == MODE_SCL_LEAVES) return -1;
        if (nf == nv) return OP_R0;
        if (nf == 0) return OP_R1;
        if (nf == nv - 1 && !frozen[off + nv - 1]) return OP_REP;
        if (nf == 1 && frozen[off] && nv >= 4 && nv <= spc_max) return OP_SPC;
        return -1;
    }

    int visit(int off, int k, int side, int paths) {
        const int cls = classify(off, k);
        if (cls >= 0) {
            const int c = leaf_candidates(cls, k, L);
            const int np = std::min(L, paths * c);
            out->push_back(SchedOp{(uint8_t)cls, (uint8_t)k, (uint8_t)side, (uint8_t)c, np});
            return np;
        }
        const int h = 1 << (k - 1);
        out->push_back(SchedOp{OP_F, (uint8_t)k, (uint8_t)side, 0, paths});
        const int p1 = visit(off, k - 1, 0, paths);
        out->push_back(SchedOp{OP_G, (uint8_t)k, (uint8_t)side, 0, p1});
        const int p2 = visit(off + h, k - 1, 1, p1);
        out->push_back(SchedOp{OP_COMB, (uint8_t)k, (uint8_t)side, 0, p2});
        return p2;
    }
};

bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

}  // namespace

int leaf_candidates(int type, int k, int L) {
    switch (type) {
        case OP_R0:
            return 1;
        case OP_REP:
            return 2;
        case OP_R1:
            return k == 0 ? 2 : 4;
        case OP_SPC:
            return L == 2 ? 2 : 8;
        default:
            return 0;
    }
}

bool build_schedule(int N, const uint8_t* frozen, int L, int spc_max, int mode,
                    std::vector<SchedOp>& out) {
    if (!is_pow2(N) || N < 2 || N > (1 << 12) || !frozen || L < 1) return false;
    if (mode != MODE_TREE && mode != MODE_SCL_LEAVES) return false;
    int n = 0;
    while ((1 << n) < N) ++n;
    out.clear();
    Walker w{frozen, L, spc_max, mode, &out};
    w.visit(0, n, 1, 1);
    return true;
}

std::vector<uint64_t> crc_codeword_table(int N, const uint8_t* frozen, uint64_t poly, int r) {
    const uint64_t mask = (r >= 64) ? ~0ull : ((1ull << r) - 1);
    const uint64_t top = 1ull << (r - 1);
    std::vector<int> pos;
    for (int i = 0; i < N; ++i)
        if (!frozen[i]) pos.push_back(i);
    const int K = (int)pos.size();
    // Register contribution of message bit t after all K bits are fed: the
    // last bit adds poly (x^r mod g), each earlier bit is one more
    // multiplication by x modulo g.
    std::vector<uint64_t> tab(N, 0);
    uint64_t v = poly & mask;
    for (int t = K - 1; t >= 0; --t) {
        tab[pos[t]] = v;
        const bool carry = (v & top) != 0;
        v = (v << 1) & mask;
        if (carry) v ^= poly & mask;
    }
    // u_p = XOR of x_i over the i that contain p as a sub-mask (G_N is its own
    // inverse and row i of G_N covers the sub-masks of i), so position i of x
    // carries the XOR of the contributions of its sub-masks: a zeta transform.
    for (int s = 1; s < N; s <<= 1)
        for (int i = 0; i < N; ++i)
            if (i & s) tab[i] ^= tab[i ^ s];
    return tab;
}

}  // namespace pscl
