// CRC-aided list decoding of polar codes on gfx950 (MI355X).
//
// One workgroup decodes FW frames of the same code in lockstep: every
// operation of the unrolled schedule (Listing 2 generalised to the list
// decoder of Sec. III) is applied to all frames, all active paths and all
// elements at once, spread over the workgroup's threads, with one barrier
// between operations.  The list-decoder state of a frame lives in LDS:
//   - LLR stages S_k (Sec. V-A): L buffers of 2^k values per stage; stage n is
//     the channel row itself, read straight from the input.  Stages too large
//     for the LDS budget live in a per-workgroup global workspace instead.
//   - Partial-sum (beta) stages (Sec. V-B) as bit-packed words, separate for
//     left and right children.
//   - Per-stage path -> buffer indices: a fork shares its source's buffers by
//     copying indices, never data (the pointer sharing of Sec. V-A); every
//     write goes to the writer's own slot, which is always dead data at that
//     point of the depth-first walk.
// Leaves score candidates with eq. (pm) and keep the L best (Alg. 1) by
// ranking (larger metric first, ties to the smaller enumeration index).
// After the last operation each path's codeword is checked against the CRC
// through a codeword-domain syndrome table, the best passing path is chosen
// (Sec. II-B), and its bits are mapped back to u = x G_N.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "pscl.h"
#include "schedule.h"

namespace pscl {

constexpr int MAXLVL = 13;  // tree levels 0..12 (N <= 4096)
constexpr int SP_LDS = 0;   // operand in LDS
constexpr int SP_WS = 1;    // operand in the global workspace
constexpr int SP_CH = 2;    // operand is the channel row

#define DEV __device__ __forceinline__

// ---------------------------------------------------------------------------
// Arithmetic of one LLR domain.
// ---------------------------------------------------------------------------

template <typename T>
struct Dom;

// float32: F exact, G one IEEE add, node penalties accumulated in double and
// rounded once to float, path-metric update one float subtraction.
template <>
struct Dom<float> {
    using A = float;   // LLR arithmetic
    using S = double;  // penalty accumulation
    using M = float;   // path metric
    static DEV A load(float v) { return v; }
    static DEV A f(A a, A b) {
        const float m = fminf(fabsf(a), fabsf(b));
        return ((a < 0.f) != (b < 0.f)) ? -m : m;
    }
    static DEV A g(A a, A b, int beta) { return beta ? __fsub_rn(b, a) : __fadd_rn(b, a); }
    static DEV uint32_t mag_key(A a) { return __float_as_uint(fabsf(a)); }
    static DEV S mag_from_key(uint32_t k) { return (double)__uint_as_float(k); }
    static DEV S widen_abs(A a) { return (double)fabsf(a); }
    static DEV M round_pen(S s) { return __double2float_rn(s); }
    static DEV M sub(M pm, M pen) { return __fsub_rn(pm, pen); }
    static DEV uint32_t order(M pm) {
        const uint32_t b = __float_as_uint(__fadd_rn(pm, 0.0f));  // -0 -> +0
        return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
    }
    static DEV uint32_t bits(M pm) { return __float_as_uint(pm); }
};

// Integers: F exact, G saturated to [-Q, Q], exact int32 metrics.
template <int Q>
struct DomI {
    using A = int;
    using S = int;
    using M = int;
    static DEV A load(int v) { return max(-Q, min(Q, v)); }
    static DEV A f(A a, A b) {
        const int m = min(abs(a), abs(b));
        return ((a ^ b) < 0) ? -m : m;
    }
    static DEV A g(A a, A b, int beta) {
        const int v = beta ? b - a : b + a;
        return max(-Q, min(Q, v));
    }
    static DEV uint32_t mag_key(A a) { return (uint32_t)abs(a); }
    static DEV S mag_from_key(uint32_t k) { return (int)k; }
    static DEV S widen_abs(A a) { return abs(a); }
    static DEV M round_pen(S s) { return s; }
    static DEV M sub(M pm, M pen) { return pm - pen; }
    static DEV uint32_t order(M pm) { return (uint32_t)pm ^ 0x80000000u; }
    static DEV uint32_t bits(M pm) { return (uint32_t)pm; }
};
template <>
struct Dom<int16_t> : DomI<32767> {};
template <>
struct Dom<int8_t> : DomI<127> {};

// ---------------------------------------------------------------------------
// Kernel arguments and per-workgroup context.
// ---------------------------------------------------------------------------

struct KArgs {
    const uint32_t* ops;  // type | k << 8 | side << 16 | cand << 24
    const int32_t* tab;   // [a_off | bl_off | br_off], MAXLVL entries each
    const uint64_t* syn;  // N codeword-domain CRC syndromes
    const uint16_t* info_pos;
    uint8_t* ws;
    int64_t ws_frame;
    int n_ops, N, n, K, L, lL, FW, k_glob, lds_frame, has_crc;
    int ptrA_off, ptrB_off, pm_off, cpm_off, surv_off, sinfo_off;
};

DEV int words_of(int k) { return k >= 5 ? (1 << (k - 5)) : 1; }
DEV int ilog2u(unsigned v) { return 31 - __clz(v); }

template <typename T>
struct Ctx {
    unsigned char* lds;
    uint8_t* wsb;
    const T* llr;
    const int32_t* tab;
    int64_t f0, F, ws_frame;
    int lds_frame, N, n, L, lL, FW, k_glob, tid, NT, lane;
    int ptrA_off, ptrB_off, pm_off, cpm_off, surv_off, sinfo_off;
    int cur;

    DEV unsigned char* fl(int fi) const { return lds + fi * lds_frame; }
    DEV uint8_t* ptrA(int fi, int buf, int k) const {
        return fl(fi) + ptrA_off + (buf * MAXLVL + k) * L;
    }
    DEV uint8_t* ptrB(int fi, int buf, int k) const {
        return fl(fi) + ptrB_off + (buf * MAXLVL + k) * L;
    }
    DEV typename Dom<T>::M* pm(int fi) const {
        return (typename Dom<T>::M*)(fl(fi) + pm_off);
    }
    DEV typename Dom<T>::M* cpm(int fi) const {
        return (typename Dom<T>::M*)(fl(fi) + cpm_off);
    }
    DEV uint16_t* surv(int fi) const { return (uint16_t*)(fl(fi) + surv_off); }
    DEV uint16_t* sinfo(int fi) const { return (uint16_t*)(fl(fi) + sinfo_off); }
    DEV uint32_t* bl(int fi, int k, int slot) const {
        return (uint32_t*)(fl(fi) + tab[MAXLVL + k]) + slot * words_of(k);
    }
    DEV uint32_t* br(int fi, int k, int slot) const {
        return (uint32_t*)(fl(fi) + tab[2 * MAXLVL + k]) + slot * words_of(k);
    }
    DEV T* st_lds(int fi, int k, int slot) const {
        return (T*)(fl(fi) + tab[k]) + (slot << k);
    }
    DEV T* st_ws(int fi, int k, int slot) const {
        return (T*)(wsb + fi * ws_frame + tab[k]) + (slot << k);
    }
    DEV const T* chan(int fi) const {
        int64_t f = f0 + fi;
        if (f >= F) f = F - 1;
        return llr + f * N;
    }
    // Input of a leaf node of size 2^k (the channel row when the root itself
    // is a leaf).
    DEV const T* leaf_in(int fi, int k, int slot) const {
        if (k == n) return chan(fi);
        if (k >= k_glob) return st_ws(fi, k, slot);
        return st_lds(fi, k, slot);
    }
    template <int SP>
    DEV const T* in_stage(int fi, int k, int slot) const {
        if constexpr (SP == SP_CH) return chan(fi);
        else if constexpr (SP == SP_WS) return st_ws(fi, k, slot);
        else return st_lds(fi, k, slot);
    }
    template <int SP>
    DEV T* out_stage(int fi, int k, int slot) const {
        if constexpr (SP == SP_WS) return st_ws(fi, k, slot);
        else return st_lds(fi, k, slot);
    }
};

// ---------------------------------------------------------------------------
// F and G over all frames, paths and elements of a level-k node.
// ---------------------------------------------------------------------------

template <typename T, bool IS_G, int ISP, int OSP>
DEV void op_fg(const Ctx<T>& c, int k, int P) {
    using D = Dom<T>;
    using A = typename D::A;
    const int lm = k - 1;
    const int M = 1 << lm;
    const int lP = ilog2u(P);
    const int lpm = lP + lm;
    const int total = c.FW << lpm;
    for (int it = c.tid; it < total; it += c.NT) {
        const int fi = it >> lpm;
        const int rem = it & ((1 << lpm) - 1);
        const int p = rem >> lm;
        const int i = rem & (M - 1);
        const int src = (ISP == SP_CH) ? 0 : c.ptrA(fi, c.cur, k)[p];
        const T* in = c.template in_stage<ISP>(fi, k, src);
        T* out = c.template out_stage<OSP>(fi, k - 1, p);
        const A x = D::load(in[i]);
        const A y = D::load(in[i + M]);
        A v;
        if constexpr (IS_G) {
            const uint32_t* b = c.bl(fi, k - 1, c.ptrB(fi, c.cur, k - 1)[p]);
            const int beta = (b[i >> 5] >> (i & 31)) & 1;
            v = D::g(x, y, beta);
        } else {
            v = D::f(x, y);
        }
        out[i] = (T)v;
    }
    const int tp = c.FW << lP;
    for (int it = c.tid; it < tp; it += c.NT) {
        const int fi = it >> lP;
        const int p = it & (P - 1);
        c.ptrA(fi, c.cur, k - 1)[p] = (uint8_t)p;
    }
}

template <typename T, bool IS_G>
DEV void op_fg_dispatch(const Ctx<T>& c, int k, int P) {
    const bool in_ch = (k == c.n);
    const bool in_ws = !in_ch && k >= c.k_glob;
    const bool out_ws = (k - 1) >= c.k_glob;
    if (in_ch) {
        if (out_ws) op_fg<T, IS_G, SP_CH, SP_WS>(c, k, P);
        else op_fg<T, IS_G, SP_CH, SP_LDS>(c, k, P);
    } else if (in_ws) {
        if (out_ws) op_fg<T, IS_G, SP_WS, SP_WS>(c, k, P);
        else op_fg<T, IS_G, SP_WS, SP_LDS>(c, k, P);
    } else {
        op_fg<T, IS_G, SP_LDS, SP_LDS>(c, k, P);
    }
}

// Combine, eq. (combine), on bit-packed words: beta_v = (beta_l ^ beta_r, beta_r).
template <typename T>
DEV void op_comb(const Ctx<T>& c, int k, int side, int P) {
    const int W = words_of(k);
    const int lw = ilog2u(W);
    const int lP = ilog2u(P);
    const int total = c.FW << (lP + lw);
    for (int it = c.tid; it < total; it += c.NT) {
        const int fi = it >> (lP + lw);
        const int p = (it >> lw) & (P - 1);
        const int w = it & (W - 1);
        const uint32_t* l = c.bl(fi, k - 1, c.ptrB(fi, c.cur, k - 1)[p]);
        const uint32_t* r = c.br(fi, k - 1, p);
        uint32_t v;
        if (k >= 6) {
            const int hw = W >> 1;
            v = (w < hw) ? (l[w] ^ r[w]) : r[w - hw];
        } else {
            const int h = 1 << (k - 1);
            const uint32_t m = (1u << h) - 1u;
            const uint32_t lv = l[0] & m, rv = r[0] & m;
            v = (lv ^ rv) | (rv << h);
        }
        uint32_t* o = side ? c.br(fi, k, p) : c.bl(fi, k, p);
        o[w] = v;
    }
    if (side == 0) {
        const int tp = c.FW << lP;
        for (int it = c.tid; it < tp; it += c.NT) {
            const int fi = it >> lP;
            const int p = it & (P - 1);
            c.ptrB(fi, c.cur, k)[p] = (uint8_t)p;
        }
    }
}

// ---------------------------------------------------------------------------
// Leaf list decoders.
// ---------------------------------------------------------------------------

// Candidate flip sets of the SPC decoder over the four least reliable bits
// m1..m4 (bit t <-> m_{t+1}), relative to the ML word: {}, {1,2}, {1,3},
// {1,4}, {2,3}, {2,4}, {3,4}, {1,2,3,4} (Sec. III-D).
__constant__ uint8_t kSpcFlips[8] = {0x0, 0x3, 0x5, 0x9, 0x6, 0xA, 0xC, 0xF};

DEV uint64_t umin64(uint64_t a, uint64_t b) { return a < b ? a : b; }
DEV uint64_t umax64(uint64_t a, uint64_t b) { return a < b ? b : a; }

DEV uint64_t shfl_xor64(uint64_t v, int m) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m, 64);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m, 64);
    return ((uint64_t)hi << 32) | lo;
}
DEV double shfl_xor_d(double v, int m) {
    return __longlong_as_double((long long)shfl_xor64((uint64_t)__double_as_longlong(v), m));
}
DEV int shfl_xor_i(int v, int m) { return __shfl_xor(v, m, 64); }

template <typename S>
DEV S shfl_xor_s(S v, int m);
template <>
DEV double shfl_xor_s<double>(double v, int m) { return shfl_xor_d(v, m); }
template <>
DEV int shfl_xor_s<int>(int v, int m) { return shfl_xor_i(v, m); }

// The 4 smallest of two ascending 4-lists, ascending (bitonic split of a
// reversed against b, then a 4-element bitonic merge).
DEV void merge4(uint64_t* a, const uint64_t* b) {
    const uint64_t l0 = umin64(a[0], b[3]), l1 = umin64(a[1], b[2]);
    const uint64_t l2 = umin64(a[2], b[1]), l3 = umin64(a[3], b[0]);
    const uint64_t x0 = umin64(l0, l2), x2 = umax64(l0, l2);
    const uint64_t x1 = umin64(l1, l3), x3 = umax64(l1, l3);
    a[0] = umin64(x0, x1);
    a[1] = umax64(x0, x1);
    a[2] = umin64(x2, x3);
    a[3] = umax64(x2, x3);
}

template <typename T>
DEV void leaf_rate0(const Ctx<T>& c, int k, int side, int P) {
    using D = Dom<T>;
    using A = typename D::A;
    using S = typename D::S;
    const int nv = 1 << k;
    const int G = nv < 64 ? nv : 64;
    const int lg = ilog2u(G);
    const int cnt = nv >> lg;
    const int lP = ilog2u(P);
    const int total = c.FW << (lP + lg);
    const int wave = c.tid >> 6;
    for (int base = wave * 64; base < total; base += c.NT) {
        const int it = base + c.lane;
        const bool act = it < total;
        const int itc = act ? it : total - 1;
        const int fi = itc >> (lP + lg);
        const int p = (itc >> lg) & (P - 1);
        const int g = itc & (G - 1);
        const T* in = c.leaf_in(fi, k, c.ptrA(fi, c.cur, k)[p]);
        S s = 0;
        for (int t = 0; t < cnt; ++t) {
            const A v = D::load(in[g + (t << lg)]);
            if (v < 0) s += D::widen_abs(v);
        }
        for (int m = 1; m < G; m <<= 1) s += shfl_xor_s<S>(s, m);
        if (act && g == 0) c.pm(fi)[p] = D::sub(c.pm(fi)[p], D::round_pen(s));
    }
    const int W = words_of(k);
    const int lw = ilog2u(W);
    const int tw = c.FW << (lP + lw);
    for (int it = c.tid; it < tw; it += c.NT) {
        const int fi = it >> (lP + lw);
        const int p = (it >> lw) & (P - 1);
        const int w = it & (W - 1);
        (side ? c.br(fi, k, p) : c.bl(fi, k, p))[w] = 0u;
    }
    if (side == 0) {
        const int tp = c.FW << lP;
        for (int it = c.tid; it < tp; it += c.NT) {
            c.ptrB(it >> lP, c.cur, k)[it & (P - 1)] = (uint8_t)(it & (P - 1));
        }
    }
}

// Forking leaves: repetition, Rate-1 and SPC.  Pass 1 scores the candidates
// of every source path; pass 2 ranks them; pass 3 writes the survivors'
// codewords, metrics and buffer indices.
template <typename T, int TYPE>
DEV void leaf_fork(Ctx<T>& c, int k, int side, int ccount, int P) {
    using D = Dom<T>;
    using A = typename D::A;
    using S = typename D::S;
    using M = typename D::M;
    const int nv = 1 << k;
    const int lP = ilog2u(P);
    const int lc = ilog2u(ccount);
    const int wave = c.tid >> 6;

    // ---- pass 1: per source path statistics and candidate metrics ----
    {
        const int G = nv < 64 ? nv : 64;
        const int lg = ilog2u(G);
        const int cnt = nv >> lg;
        const int total = c.FW << (lP + lg);
        for (int base = wave * 64; base < total; base += c.NT) {
            const int it = base + c.lane;
            const bool act = it < total;
            const int itc = act ? it : total - 1;
            const int fi = itc >> (lP + lg);
            const int s = (itc >> lg) & (P - 1);
            const int g = itc & (G - 1);
            const T* in = c.leaf_in(fi, k, c.ptrA(fi, c.cur, k)[s]);
            const M pms = c.pm(fi)[s];
            M* cp = c.cpm(fi) + (s << lc);
            uint16_t* si = c.sinfo(fi) + s * 8;
            if constexpr (TYPE == OP_REP) {
                // penalties of the all-zero and all-one words (Sec. III-E)
                S z = 0, o = 0;
                for (int t = 0; t < cnt; ++t) {
                    const A v = D::load(in[g + (t << lg)]);
                    if (v < 0) z += D::widen_abs(v);
                    else o += D::widen_abs(v);
                }
                for (int m = 1; m < G; m <<= 1) {
                    z += shfl_xor_s<S>(z, m);
                    o += shfl_xor_s<S>(o, m);
                }
                if (act && g == 0) {
                    const M zr = D::round_pen(z), orr = D::round_pen(o);
                    const bool one = orr < zr;  // ML word first; equal -> all-zero
                    cp[0] = D::sub(pms, one ? orr : zr);
                    cp[1] = D::sub(pms, one ? zr : orr);
                    si[4] = one ? 1 : 0;
                }
            } else if constexpr (TYPE == OP_R1) {
                if (k == 0) {
                    if (act) {
                        const A v = D::load(in[0]);
                        cp[0] = pms;
                        cp[1] = D::sub(pms, D::round_pen(D::widen_abs(v)));
                        si[4] = (v < 0) ? 1 : 0;
                    }
                } else {
                    // two least reliable positions, ties to the lower index
                    uint64_t k1 = ~0ull, k2 = ~0ull;
                    for (int t = 0; t < cnt; ++t) {
                        const int i = g + (t << lg);
                        const uint64_t key = ((uint64_t)D::mag_key(D::load(in[i])) << 32) | (uint32_t)i;
                        if (key < k1) {
                            k2 = k1;
                            k1 = key;
                        } else if (key < k2) {
                            k2 = key;
                        }
                    }
                    for (int m = 1; m < G; m <<= 1) {
                        const uint64_t o1 = shfl_xor64(k1, m), o2 = shfl_xor64(k2, m);
                        const uint64_t n1 = umin64(k1, o1);
                        const uint64_t n2 = umin64(umax64(k1, o1), umin64(k2, o2));
                        k1 = n1;
                        k2 = n2;
                    }
                    if (act && g == 0) {
                        const S a1 = D::mag_from_key((uint32_t)(k1 >> 32));
                        const S a2 = D::mag_from_key((uint32_t)(k2 >> 32));
                        cp[0] = pms;
                        cp[1] = D::sub(pms, D::round_pen(a1));
                        cp[2] = D::sub(pms, D::round_pen(a2));
                        cp[3] = D::sub(pms, D::round_pen(a1 + a2));
                        si[0] = (uint16_t)(k1 & 0xffff);
                        si[1] = (uint16_t)(k2 & 0xffff);
                    }
                }
            } else {  // OP_SPC
                uint64_t kk[4] = {~0ull, ~0ull, ~0ull, ~0ull};
                int par = 0;
                for (int t = 0; t < cnt; ++t) {
                    const int i = g + (t << lg);
                    const A v = D::load(in[i]);
                    par ^= (v < 0) ? 1 : 0;
                    uint64_t key = ((uint64_t)D::mag_key(v) << 32) | (uint32_t)i;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const uint64_t lo = umin64(kk[q], key);
                        key = umax64(kk[q], key);
                        kk[q] = lo;
                    }
                }
                for (int m = 1; m < G; m <<= 1) {
                    uint64_t ob[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) ob[q] = shfl_xor64(kk[q], m);
                    par ^= shfl_xor_i(par, m);
                    merge4(kk, ob);
                }
                if (act && g == 0) {
                    // The four positions re-sorted by index (carrying their
                    // reliability rank), so penalties sum in index order.
                    uint32_t idx[4], rk[4];
                    S mag[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        idx[q] = (uint32_t)(kk[q] & 0xffff);
                        mag[q] = D::mag_from_key((uint32_t)(kk[q] >> 32));
                        rk[q] = (uint32_t)q;
                        si[q] = (uint16_t)idx[q];
                    }
#pragma unroll
                    for (int x = 0; x < 3; ++x) {
#pragma unroll
                        for (int y = 0; y < 3 - x; ++y) {
                            const bool sw = idx[y] > idx[y + 1];
                            const uint32_t i0 = idx[y], i1 = idx[y + 1];
                            const uint32_t r0 = rk[y], r1 = rk[y + 1];
                            const S m0 = mag[y], m1 = mag[y + 1];
                            idx[y] = sw ? i1 : i0;
                            idx[y + 1] = sw ? i0 : i1;
                            rk[y] = sw ? r1 : r0;
                            rk[y + 1] = sw ? r0 : r1;
                            mag[y] = sw ? m1 : m0;
                            mag[y + 1] = sw ? m0 : m1;
                        }
                    }
                    si[4] = (uint16_t)par;
                    const uint32_t base_d = par ? 1u : 0u;  // ML flips m1 when parity fails
                    for (int r = 0; r < ccount; ++r) {
                        const uint32_t dm = kSpcFlips[r] ^ base_d;
                        S pen = 0;
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            if ((dm >> rk[q]) & 1u) pen += mag[q];
                        cp[r] = D::sub(pms, D::round_pen(pen));
                    }
                }
            }
        }
    }
    __syncthreads();

    // ---- pass 2: rank when candidates must be dropped ----
    const int C = P << lc;
    const int lC = lP + lc;
    const int L = c.L;
    const bool prune = C > L;
    if (prune) {
        const int total = c.FW << lC;
        for (int it = c.tid; it < total; it += c.NT) {
            const int fi = it >> lC;
            const int e = it & (C - 1);
            const M* cp = c.cpm(fi);
            const uint64_t mine = ((uint64_t)D::order(cp[e]) << 32) | (uint32_t)(0xffff - e);
            int rank = 0;
            for (int e2 = 0; e2 < C; ++e2) {
                const uint64_t other = ((uint64_t)D::order(cp[e2]) << 32) | (uint32_t)(0xffff - e2);
                rank += other > mine ? 1 : 0;
            }
            if (rank < L) c.surv(fi)[rank] = (uint16_t)e;
        }
        __syncthreads();
    }

    // ---- pass 3: survivors ----
    const int Pn = prune ? L : C;
    const int lPn = ilog2u(Pn);
    const int nxt = c.cur ^ 1;
    {
        const int levels = c.n + 1;
        const int total = c.FW * Pn * levels;
        for (int it = c.tid; it < total; it += c.NT) {
            const int fi = it / (Pn * levels);
            const int rem = it - fi * (Pn * levels);
            const int j = rem / levels;
            const int lv = rem - j * levels;
            const int e = prune ? c.surv(fi)[j] : j;
            const int s = e >> lc;
            c.ptrA(fi, nxt, lv)[j] = c.ptrA(fi, c.cur, lv)[s];
            c.ptrB(fi, nxt, lv)[j] =
                (lv == k && side == 0) ? (uint8_t)j : c.ptrB(fi, c.cur, lv)[s];
            if (lv == 0) c.pm(fi)[j] = c.cpm(fi)[e];
        }
    }
    {
        // codeword bits, assembled into words with a wave ballot
        const int total = c.FW << (lPn + k);
        for (int base = wave * 64; base < total; base += c.NT) {
            const int it = base + c.lane;
            const bool act = it < total;
            const int itc = act ? it : total - 1;
            const int fi = itc >> (lPn + k);
            const int j = (itc >> k) & (Pn - 1);
            const int i = itc & (nv - 1);
            const int e = prune ? c.surv(fi)[j] : j;
            const int s = e >> lc;
            const int r = e & (ccount - 1);
            const uint16_t* si = c.sinfo(fi) + s * 8;
            int bit;
            if constexpr (TYPE == OP_REP) {
                bit = (si[4] ^ r) & 1;
            } else {
                if (TYPE == OP_R1 && k == 0) {
                    bit = (si[4] ^ r) & 1;
                } else {
                    const T* in = c.leaf_in(fi, k, c.ptrA(fi, c.cur, k)[s]);
                    bit = (D::load(in[i]) < 0) ? 1 : 0;
                    uint32_t dm;
                    if constexpr (TYPE == OP_R1) dm = (uint32_t)r;
                    else dm = kSpcFlips[r] ^ (si[4] ? 1u : 0u);
                    const int nq = (TYPE == OP_R1) ? 2 : 4;
                    for (int q = 0; q < nq; ++q)
                        if (((dm >> q) & 1u) && i == si[q]) bit ^= 1;
                }
            }
            const uint64_t bal = __ballot(act && bit);
            if (act && (i & 31) == 0) {
                const uint32_t mask = nv >= 32 ? 0xffffffffu : ((1u << nv) - 1u);
                const uint32_t wv = (uint32_t)(bal >> c.lane) & mask;
                (side ? c.br(fi, k, j) : c.bl(fi, k, j))[i >> 5] = wv;
            }
        }
    }
    c.cur = nxt;
}

// ---------------------------------------------------------------------------
// Final choice: CRC syndromes, best passing path, u = x G_N, output.
// ---------------------------------------------------------------------------

template <typename T>
DEV void finish(const Ctx<T>& c, const KArgs& a, int P, uint8_t* u_hat, uint8_t* crc_ok,
                void* pm_out) {
    using D = Dom<T>;
    using M = typename D::M;
    const int n = c.n;
    const int W = words_of(n);
    const int lP = ilog2u(P);
    const int wave = c.tid >> 6;
    // syndromes: one group of lanes per (frame, path)
    {
        const int G = W < 64 ? W : 64;
        const int lg = ilog2u(G);
        const int cnt = W >> lg;
        const int total = c.FW << (lP + lg);
        for (int base = wave * 64; base < total; base += c.NT) {
            const int it = base + c.lane;
            const bool act = it < total;
            const int itc = act ? it : total - 1;
            const int fi = itc >> (lP + lg);
            const int j = (itc >> lg) & (P - 1);
            const int g = itc & (G - 1);
            const uint32_t* x = c.br(fi, n, j);
            uint64_t acc = 0;
            if (a.has_crc) {
                for (int t = 0; t < cnt; ++t) {
                    const int w = g + (t << lg);
                    uint32_t v = x[w];
                    while (v) {
                        const int b = __ffs(v) - 1;
                        v &= v - 1;
                        acc ^= a.syn[(w << 5) + b];
                    }
                }
                for (int m = 1; m < G; m <<= 1) acc ^= shfl_xor64(acc, m);
            }
            if (act && g == 0) c.surv(fi)[j] = (acc == 0) ? 1 : 0;
        }
    }
    __syncthreads();
    // pick: one lane per (frame, path), segments of P lanes
    {
        const int total = c.FW << lP;
        for (int base = wave * 64; base < total; base += c.NT) {
            const int it = base + c.lane;
            const bool act = it < total;
            const int itc = act ? it : total - 1;
            const int fi = itc >> lP;
            const int j = itc & (P - 1);
            const uint64_t pass = c.surv(fi)[j] & 1;
            uint64_t key = (pass << 40) | ((uint64_t)D::order(c.pm(fi)[j]) << 8) | (uint64_t)(255 - j);
            for (int m = 1; m < P; m <<= 1) key = umax64(key, shfl_xor64(key, m));
            if (act && j == 0) {
                const int best = 255 - (int)(key & 0xff);
                const int ok = (int)(key >> 40) & 1;
                c.sinfo(fi)[0] = (uint16_t)best;
                const int64_t f = c.f0 + fi;
                if (f < c.F) {
                    if (crc_ok) crc_ok[f] = (uint8_t)ok;
                    if (pm_out) ((uint32_t*)pm_out)[f] = D::bits(c.pm(fi)[best]);
                }
            }
        }
    }
    __syncthreads();
    // u = x G_N on the chosen codeword, in place: bits within words ...
    {
        const int total = c.FW * W;
        for (int it = c.tid; it < total; it += c.NT) {
            const int fi = it / W;
            const int w = it - fi * W;
            uint32_t* x = c.br(fi, n, c.sinfo(fi)[0]);
            uint32_t v = x[w];
            v ^= (v >> 1) & 0x55555555u;
            v ^= (v >> 2) & 0x33333333u;
            v ^= (v >> 4) & 0x0f0f0f0fu;
            v ^= (v >> 8) & 0x00ff00ffu;
            v ^= (v >> 16) & 0x0000ffffu;
            x[w] = v;
        }
    }
    // ... then across words
    for (int sw = 1; sw < W; sw <<= 1) {
        __syncthreads();
        const int total = c.FW * W;
        for (int it = c.tid; it < total; it += c.NT) {
            const int fi = it / W;
            const int w = it - fi * W;
            if (w & sw) continue;
            uint32_t* x = c.br(fi, n, c.sinfo(fi)[0]);
            x[w] ^= x[w + sw];
        }
    }
    __syncthreads();
    {
        const int K = a.K;
        const int total = c.FW * K;
        for (int it = c.tid; it < total; it += c.NT) {
            const int fi = it / K;
            const int t = it - fi * K;
            const int64_t f = c.f0 + fi;
            if (f >= c.F) continue;
            const uint32_t* x = c.br(fi, n, c.sinfo(fi)[0]);
            const int p = a.info_pos[t];
            u_hat[f * K + t] = (uint8_t)((x[p >> 5] >> (p & 31)) & 1u);
        }
    }
}

// ---------------------------------------------------------------------------
// The kernel: a persistent grid; each workgroup takes FW frames at a time.
// ---------------------------------------------------------------------------

template <typename T>
__global__ void __launch_bounds__(1024)
    decode_kernel(KArgs a, const T* __restrict__ llr, int64_t F, uint8_t* __restrict__ u_hat,
                  uint8_t* __restrict__ crc_ok, void* __restrict__ pm_out) {
    extern __shared__ __align__(16) unsigned char lds[];
    Ctx<T> c;
    c.lds = lds;
    c.wsb = a.ws + (int64_t)blockIdx.x * a.FW * a.ws_frame;
    c.llr = llr;
    c.tab = a.tab;
    c.F = F;
    c.ws_frame = a.ws_frame;
    c.lds_frame = a.lds_frame;
    c.N = a.N;
    c.n = a.n;
    c.L = a.L;
    c.lL = a.lL;
    c.FW = a.FW;
    c.k_glob = a.k_glob;
    c.tid = threadIdx.x;
    c.NT = blockDim.x;
    c.lane = threadIdx.x & 63;
    c.ptrA_off = a.ptrA_off;
    c.ptrB_off = a.ptrB_off;
    c.pm_off = a.pm_off;
    c.cpm_off = a.cpm_off;
    c.surv_off = a.surv_off;
    c.sinfo_off = a.sinfo_off;

    for (int64_t f0 = (int64_t)blockIdx.x * a.FW; f0 < F; f0 += (int64_t)gridDim.x * a.FW) {
        c.f0 = f0;
        c.cur = 0;
        for (int fi = c.tid; fi < c.FW; fi += c.NT) c.pm(fi)[0] = 0;
        __syncthreads();
        int P = 1;
        for (int oi = 0; oi < a.n_ops; ++oi) {
            const uint32_t op = a.ops[oi];
            const int type = op & 0xff;
            const int k = (op >> 8) & 0xff;
            const int side = (op >> 16) & 0xff;
            const int cc = (int)(op >> 24);
            switch (type) {
                case OP_F:
                    op_fg_dispatch<T, false>(c, k, P);
                    break;
                case OP_G:
                    op_fg_dispatch<T, true>(c, k, P);
                    break;
                case OP_COMB:
                    op_comb<T>(c, k, side, P);
                    break;
                case OP_R0:
                    leaf_rate0<T>(c, k, side, P);
                    break;
                case OP_REP:
                    leaf_fork<T, OP_REP>(c, k, side, cc, P);
                    P = min(c.L, P * cc);
                    break;
                case OP_R1:
                    leaf_fork<T, OP_R1>(c, k, side, cc, P);
                    P = min(c.L, P * cc);
                    break;
                default:
                    leaf_fork<T, OP_SPC>(c, k, side, cc, P);
                    P = min(c.L, P * cc);
                    break;
            }
            __syncthreads();
        }
        finish<T>(c, a, P, u_hat, crc_ok, pm_out);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------

static int elem_size(int dtype) { return dtype == PSCL_F32 ? 4 : (dtype == PSCL_I16 ? 2 : 1); }
static int words_host(int k) { return k >= 5 ? (1 << (k - 5)) : 1; }
static int align16(int x) { return (x + 15) & ~15; }

}  // namespace pscl

using namespace pscl;

struct pscl_plan {
    int N = 0, n = 0, K = 0, r = 0, L = 0, dtype = 0, spc_max = 0, mode = 0;
    uint64_t poly = 0;
    int device = 0;
    std::vector<SchedOp> sched;
    uint32_t* d_ops = nullptr;
    int32_t* d_tab = nullptr;
    uint64_t* d_syn = nullptr;
    uint16_t* d_info = nullptr;
    uint8_t* d_ws = nullptr;
    KArgs args{};
    int NT = 256, FW = 1, grid_max = 0, lds_bytes = 0;
    int64_t ws_bytes = 0;
    const void* kernel = nullptr;
};

namespace {

pscl_status hip_status(hipError_t e) {
    if (e == hipSuccess) return PSCL_OK;
    if (e == hipErrorOutOfMemory) return PSCL_E_NOMEM;
    return PSCL_E_HIP;
}

bool valid_L(int L) { return L == 1 || L == 2 || L == 4 || L == 8 || L == 16 || L == 32; }

const void* kernel_for(int dtype) {
    switch (dtype) {
        case PSCL_F32:
            return (const void*)&decode_kernel<float>;
        case PSCL_I16:
            return (const void*)&decode_kernel<int16_t>;
        default:
            return (const void*)&decode_kernel<int8_t>;
    }
}

// Per-frame LDS layout for a given first global stage; returns bytes.
int layout(pscl_plan* p, int k_glob, int32_t* tab, KArgs& a, int64_t* ws_frame) {
    const int L = p->L, n = p->n, es = elem_size(p->dtype);
    int off = 0;
    int64_t woff = 0;
    for (int k = 0; k < MAXLVL; ++k) tab[k] = 0;
    for (int k = 0; k < n; ++k) {
        const int bytes = L * (1 << k) * es;
        if (k < k_glob) {
            tab[k] = off;
            off = align16(off + bytes);
        } else {
            tab[k] = (int32_t)woff;
            woff += (bytes + 255) & ~255;
        }
    }
    for (int k = 0; k <= n; ++k) {
        tab[MAXLVL + k] = off;
        off = align16(off + L * words_host(k) * 4);
        tab[2 * MAXLVL + k] = off;
        off = align16(off + L * words_host(k) * 4);
    }
    a.ptrA_off = off;
    off = align16(off + 2 * MAXLVL * L);
    a.ptrB_off = off;
    off = align16(off + 2 * MAXLVL * L);
    a.pm_off = off;
    off = align16(off + 4 * L);
    a.cpm_off = off;
    off = align16(off + 4 * 8 * L);
    a.surv_off = off;
    off = align16(off + 2 * 8 * L);
    a.sinfo_off = off;
    off = align16(off + 16 * 8 * L);
    *ws_frame = woff;
    return off;
}

}  // namespace

extern "C" {

const char* pscl_status_str(pscl_status s) {
    switch (s) {
        case PSCL_OK:
            return "ok";
        case PSCL_E_INVALID:
            return "invalid argument";
        case PSCL_E_UNSUPPORTED:
            return "unsupported configuration";
        case PSCL_E_NOMEM:
            return "device out of memory";
        case PSCL_E_HIP:
            return "HIP runtime error";
        case PSCL_E_NODEV:
            return "no gfx950 device";
    }
    return "unknown status";
}

int pscl_version(void) { return 100; }

pscl_status pscl_schedule(int N, const uint8_t* frozen_mask, int L, int spc_max, int mode,
                          int32_t* ops, int cap, int* n_ops) {
    if (!frozen_mask || !n_ops || cap < 0 || !valid_L(L)) return PSCL_E_INVALID;
    std::vector<SchedOp> s;
    if (!build_schedule(N, frozen_mask, L, spc_max, mode, s)) return PSCL_E_INVALID;
    *n_ops = (int)s.size();
    if ((int)s.size() > cap || (!ops && !s.empty())) return PSCL_E_INVALID;
    for (size_t i = 0; i < s.size(); ++i) {
        ops[4 * i + 0] = s[i].type;
        ops[4 * i + 1] = s[i].k;
        ops[4 * i + 2] = s[i].side;
        ops[4 * i + 3] = s[i].paths;
    }
    return PSCL_OK;
}

void pscl_plan_destroy(pscl_plan* p) {
    if (!p) return;
    int cur = 0;
    if (hipGetDevice(&cur) == hipSuccess && cur != p->device) (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(p->d_ops);
    (void)hipFree(p->d_tab);
    (void)hipFree(p->d_syn);
    (void)hipFree(p->d_info);
    (void)hipFree(p->d_ws);
    if (cur != p->device) (void)hipSetDevice(cur);
    delete p;
}

pscl_status pscl_plan_create(int N, int K, const uint8_t* frozen_mask, uint64_t crc_poly,
                             int crc_len, int L, int dtype, int spc_max, int mode,
                             pscl_plan** out) {
    if (!out || !frozen_mask) return PSCL_E_INVALID;
    if (N < 2 || N > 4096 || (N & (N - 1))) return PSCL_E_INVALID;
    if (!valid_L(L) || dtype < PSCL_F32 || dtype > PSCL_I8) return PSCL_E_INVALID;
    if (mode != PSCL_MODE_TREE && mode != PSCL_MODE_SCL_LEAVES) return PSCL_E_INVALID;
    int kk = 0;
    for (int i = 0; i < N; ++i) kk += frozen_mask[i] ? 0 : 1;
    if (kk != K || K < 1 || crc_len < 0 || crc_len > 64 || crc_len > K) return PSCL_E_INVALID;

    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PSCL_E_NODEV;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return PSCL_E_NODEV;
    if (std::string(prop.gcnArchName).find("gfx950") == std::string::npos) return PSCL_E_NODEV;

    pscl_plan* p = new pscl_plan();
    p->N = N;
    p->K = K;
    p->r = crc_len;
    p->L = L;
    p->dtype = dtype;
    p->spc_max = spc_max;
    p->mode = mode;
    p->poly = crc_poly;
    p->device = dev;
    while ((1 << p->n) < N) p->n++;
    if (!build_schedule(N, frozen_mask, L, spc_max, mode, p->sched)) {
        delete p;
        return PSCL_E_INVALID;
    }

    // Layout: keep as many low stages in LDS as the per-workgroup budget
    // allows; larger stages go to the global workspace.
    const int lds_cap = (int)std::min<size_t>(prop.sharedMemPerBlock, 160 * 1024);
    int32_t tab[3 * MAXLVL];
    KArgs a{};
    int64_t wsf = 0;
    int k_glob = p->n;
    int bytes = layout(p, k_glob, tab, a, &wsf);
    while (bytes > lds_cap && k_glob > 0) {
        --k_glob;
        bytes = layout(p, k_glob, tab, a, &wsf);
    }
    if (bytes > lds_cap) {
        delete p;
        return PSCL_E_UNSUPPORTED;
    }
    // Frames per workgroup: fill up to a quarter of the LDS budget, at most 8.
    int FW = std::max(1, std::min(8, (lds_cap / 4) / bytes));
    p->FW = FW;
    p->NT = 256;
    p->lds_bytes = bytes * FW;
    p->kernel = kernel_for(dtype);

    hipError_t e = hipFuncSetAttribute(p->kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       p->lds_bytes);
    if (e != hipSuccess) {
        delete p;
        return hip_status(e);
    }
    int occ = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, p->kernel, p->NT, p->lds_bytes);
    if (e != hipSuccess || occ < 1) occ = 1;
    p->grid_max = occ * prop.multiProcessorCount;
    p->ws_bytes = wsf * FW * (int64_t)p->grid_max;

    std::vector<uint32_t> ops(p->sched.size());
    for (size_t i = 0; i < ops.size(); ++i) {
        const SchedOp& s = p->sched[i];
        ops[i] = (uint32_t)s.type | ((uint32_t)s.k << 8) | ((uint32_t)s.side << 16) |
                 ((uint32_t)s.cand << 24);
    }
    std::vector<uint64_t> syn(N, 0);
    if (crc_len > 0) syn = crc_codeword_table(N, frozen_mask, crc_poly, crc_len);
    std::vector<uint16_t> info;
    for (int i = 0; i < N; ++i)
        if (!frozen_mask[i]) info.push_back((uint16_t)i);

    pscl_status st = PSCL_OK;
    auto up = [&](void** dst, const void* src, size_t n) {
        if (st != PSCL_OK) return;
        hipError_t err = hipMalloc(dst, std::max<size_t>(n, 16));
        if (err == hipSuccess && n) err = hipMemcpy(*dst, src, n, hipMemcpyHostToDevice);
        st = hip_status(err);
    };
    up((void**)&p->d_ops, ops.data(), ops.size() * 4);
    up((void**)&p->d_tab, tab, sizeof(tab));
    up((void**)&p->d_syn, syn.data(), syn.size() * 8);
    up((void**)&p->d_info, info.data(), info.size() * 2);
    if (st == PSCL_OK && p->ws_bytes > 0) st = hip_status(hipMalloc((void**)&p->d_ws, p->ws_bytes));
    if (st != PSCL_OK) {
        pscl_plan_destroy(p);
        return st;
    }

    a.ops = p->d_ops;
    a.tab = p->d_tab;
    a.syn = p->d_syn;
    a.info_pos = p->d_info;
    a.ws = p->d_ws;
    a.ws_frame = wsf;
    a.n_ops = (int)ops.size();
    a.N = N;
    a.n = p->n;
    a.K = K;
    a.L = L;
    int lL = 0;
    while ((1 << lL) < L) ++lL;
    a.lL = lL;
    a.FW = FW;
    a.k_glob = k_glob;
    a.lds_frame = bytes;
    a.has_crc = crc_len > 0 ? 1 : 0;
    p->args = a;
    *out = p;
    return PSCL_OK;
}

pscl_status pscl_plan_info(const pscl_plan* p, int* frames_per_wg, int* threads, int* workgroups,
                           int* lds_bytes, int64_t* workspace_bytes, int* first_global_stage) {
    if (!p) return PSCL_E_INVALID;
    if (frames_per_wg) *frames_per_wg = p->FW;
    if (threads) *threads = p->NT;
    if (workgroups) *workgroups = p->grid_max;
    if (lds_bytes) *lds_bytes = p->lds_bytes;
    if (workspace_bytes) *workspace_bytes = p->ws_bytes;
    if (first_global_stage) *first_global_stage = p->args.k_glob;
    return PSCL_OK;
}

pscl_status pscl_decode(const pscl_plan* p, const void* llr, int64_t F, uint8_t* u_hat,
                        uint8_t* crc_ok, void* pm, void* stream) {
    if (!p || F < 0) return PSCL_E_INVALID;
    if (F == 0) return PSCL_OK;
    if (!llr || !u_hat) return PSCL_E_INVALID;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return PSCL_E_HIP;
    const int64_t groups = (F + p->FW - 1) / p->FW;
    const int grid = (int)std::min<int64_t>(groups, p->grid_max);
    hipStream_t s = (hipStream_t)stream;
    switch (p->dtype) {
        case PSCL_F32:
            hipLaunchKernelGGL(decode_kernel<float>, dim3(grid), dim3(p->NT), p->lds_bytes, s,
                               p->args, (const float*)llr, F, u_hat, crc_ok, pm);
            break;
        case PSCL_I16:
            hipLaunchKernelGGL(decode_kernel<int16_t>, dim3(grid), dim3(p->NT), p->lds_bytes, s,
                               p->args, (const int16_t*)llr, F, u_hat, crc_ok, pm);
            break;
        default:
            hipLaunchKernelGGL(decode_kernel<int8_t>, dim3(grid), dim3(p->NT), p->lds_bytes, s,
                               p->args, (const int8_t*)llr, F, u_hat, crc_ok, pm);
            break;
    }
    e = hipGetLastError();
    return e == hipSuccess ? PSCL_OK : PSCL_E_HIP;
}

pscl_status pscl_decode_oneshot(int N, int K, const uint8_t* frozen_mask, uint64_t crc_poly,
                                int crc_len, int L, int dtype, const void* llr, int64_t F,
                                uint8_t* u_hat, uint8_t* crc_ok, void* stream) {
    if (!frozen_mask || N < 2 || N > 4096) return PSCL_E_INVALID;
    static std::mutex mu;
    static std::map<std::string, pscl_plan*> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PSCL_E_NODEV;
    std::string key((const char*)frozen_mask, (size_t)N);
    key += std::to_string(N) + "/" + std::to_string(K) + "/" + std::to_string(crc_poly) + "/" +
           std::to_string(crc_len) + "/" + std::to_string(L) + "/" + std::to_string(dtype) + "/" +
           std::to_string(dev);
    pscl_plan* p = nullptr;
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = cache.find(key);
        if (it != cache.end()) {
            p = it->second;
        } else {
            pscl_status st = pscl_plan_create(N, K, frozen_mask, crc_poly, crc_len, L, dtype, 4,
                                              PSCL_MODE_TREE, &p);
            if (st != PSCL_OK) return st;
            cache[key] = p;
        }
    }
    return pscl_decode(p, llr, F, u_hat, crc_ok, nullptr, stream);
}

}  // extern "C"
