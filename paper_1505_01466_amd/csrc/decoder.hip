// CRC-aided list decoding of polar codes on gfx950 (MI355X).
//
// A persistent grid of small workgroups; each decodes one frame at a time by
// walking the code's schedule (Listing 2 generalised to the list decoder of
// Sec. III).  Between two forking leaves every operation acts on each path
// alone, so each path is owned by a group of lanes inside one wavefront and
// runs without workgroup barriers; candidate ranking and the survivors'
// write-back are the only workgroup-wide steps.  A frame's state:
//   - LLR stages S_k (Sec. V-A): L buffers of 2^k values per stage; stage n is
//     the channel row itself.  Low stages live in LDS, stages too large for
//     the LDS budget in a per-workgroup global workspace.
//   - Partial-sum (beta) stages (Sec. V-B) as bit-packed words, separate for
//     left and right children, split between LDS and workspace the same way.
//   - Per-slot path -> buffer tables: a fork shares its source's buffers by
//     copying indices, never data (the pointer sharing of Sec. V-A); every
//     write goes to the writer's own slot, which is always dead data at that
//     point of the depth-first walk.
// Leaves score candidates with eq. (pm) and keep the L best (Alg. 1) by
// ranking (larger metric first, ties to the smaller enumeration index).
// After the last operation each path's codeword is checked against the CRC
// through a codeword-domain syndrome table, the best passing path is chosen
// (Sec. II-B), and its bits are mapped back to u = x G_N.
#include <hip/hip_runtime.h>
#include <type_traits>

#include <algorithm>
#include <cstdlib>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "pscl.h"
#include "ring.h"
#include "schedule.h"

namespace pscl {

constexpr int MAXLVL = 13;  // tree levels 0..12 (N <= 4096)
constexpr int SP_LDS = 0;   // operand in LDS
constexpr int SP_WS = 1;    // operand in the global workspace
constexpr int SP_CH = 2;    // operand is the channel row
// operand is the stage below the root, recomputed from the channel row
// (the root's F for its left child, its G with the path's left-half partial
// sums for its right child) instead of stored
constexpr int SP_VT = 3;
constexpr int OP_NOP = 7;  // a record with nothing to do

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
    // inverse of order (metrics are never -0: they start at +0 and only
    // lose non-negative penalties)
    static DEV M from_order(uint32_t o) {
        return __uint_as_float((o & 0x80000000u) ? (o & 0x7fffffffu) : ~o);
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
    static DEV M from_order(uint32_t o) { return (int)(o ^ 0x80000000u); }
    static DEV uint32_t bits(M pm) { return (uint32_t)pm; }
};
template <>
struct Dom<int16_t> : DomI<32767> {};
template <>
struct Dom<int8_t> : DomI<127> {};

// Ranking keys of candidates, larger = better: the metric, then the smaller
// enumeration index e.  In general the metric's order above 0xffff - e in 64
// bits.  int8 metrics lie in [-127 N, 0] with N <= 4096, inside [-2^19, 0],
// and e < 1024, so the same order fits 32 bits: (PM + 2^19) << 12 | 0xfff - e
// (never 0, the padding every real key beats).
template <typename T>
struct Rank {
    using K = uint64_t;
    using M = typename Dom<T>::M;
    static DEV K make(M v, int e) {
        return ((uint64_t)Dom<T>::order(v) << 32) | (uint32_t)(0xffff - e);
    }
    static DEV M pm(K k) { return Dom<T>::from_order((uint32_t)(k >> 32)); }
    static DEV int idx(K k) { return 0xffff - (int)(k & 0xffff); }
};
// Keys of positions in a node for finding the least reliable ones: |value|,
// then the index (smaller = less reliable, ties to the lower index).  Integer
// magnitudes (at most 32767) and indices (below 4096) fit 32 bits in the
// same order.
template <typename T>
struct Lrb {
    using K = uint64_t;
    static DEV K make(typename Dom<T>::A v, int i) {
        return ((uint64_t)Dom<T>::mag_key(v) << 32) | (uint32_t)i;
    }
    static DEV typename Dom<T>::S mag(K k) { return Dom<T>::mag_from_key((uint32_t)(k >> 32)); }
    static DEV int idx(K k) { return (int)(k & 0xffff); }
};
template <typename T>
struct LrbI {
    using K = uint32_t;
    static DEV K make(int v, int i) { return ((uint32_t)abs(v) << 12) | (uint32_t)i; }
    static DEV int mag(K k) { return (int)(k >> 12); }
    static DEV int idx(K k) { return (int)(k & 0xfff); }
};
template <>
struct Lrb<int16_t> : LrbI<int16_t> {};
template <>
struct Lrb<int8_t> : LrbI<int8_t> {};

template <>
struct Rank<int8_t> {
    using K = uint32_t;
    static DEV K make(int v, int e) { return ((uint32_t)(v + (1 << 19)) << 12) | (uint32_t)(0xfff - e); }
    static DEV int pm(K k) { return (int)(k >> 12) - (1 << 19); }
    static DEV int idx(K k) { return 0xfff - (int)(k & 0xfff); }
};

// ---------------------------------------------------------------------------
// 16-byte vector access to LLR stages.
// ---------------------------------------------------------------------------

DEV uint32_t comp4(const uint4& q, int j) {
    return j == 0 ? q.x : (j == 1 ? q.y : (j == 2 ? q.z : q.w));
}

template <typename T>
struct VecIO;

template <>
struct VecIO<float> {
    static constexpr int LOGV = 2;
    static constexpr int V = 4;
    static DEV void unpack(const uint4& q, float* o) {
        o[0] = __uint_as_float(q.x);
        o[1] = __uint_as_float(q.y);
        o[2] = __uint_as_float(q.z);
        o[3] = __uint_as_float(q.w);
    }
    static DEV uint4 pack(const float* v) {
        return make_uint4(__float_as_uint(v[0]), __float_as_uint(v[1]), __float_as_uint(v[2]),
                          __float_as_uint(v[3]));
    }
};

template <>
struct VecIO<int16_t> {
    static constexpr int LOGV = 3;
    static constexpr int V = 8;
    static DEV void unpack(const uint4& q, int* o) {
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const uint32_t x = comp4(q, w);
            o[2 * w] = ((int)(x << 16)) >> 16;
            o[2 * w + 1] = ((int)x) >> 16;
        }
    }
    static DEV uint4 pack(const int* v) {
        uint32_t w[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) w[t] = ((uint32_t)v[2 * t] & 0xffffu) | ((uint32_t)v[2 * t + 1] << 16);
        return make_uint4(w[0], w[1], w[2], w[3]);
    }
};

template <>
struct VecIO<int8_t> {
    static constexpr int LOGV = 4;
    static constexpr int V = 16;
    static DEV void unpack(const uint4& q, int* o) {
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const uint32_t x = comp4(q, w);
#pragma unroll
            for (int j = 0; j < 4; ++j) o[4 * w + j] = ((int)(x << (24 - 8 * j))) >> 24;
        }
    }
    static DEV uint4 pack(const int* v) {
        uint32_t w[4];
#pragma unroll
        for (int t = 0; t < 4; ++t)
            w[t] = ((uint32_t)v[4 * t] & 0xffu) | (((uint32_t)v[4 * t + 1] & 0xffu) << 8) |
                   (((uint32_t)v[4 * t + 2] & 0xffu) << 16) | ((uint32_t)v[4 * t + 3] << 24);
        return make_uint4(w[0], w[1], w[2], w[3]);
    }
};

// ---------------------------------------------------------------------------
// F and G on a whole 16-byte chunk of stage values (both operands already
// within the domain's range).  F uses sign(a)sign(b)min(|a|,|b|) =
// max(min(a, b), -max(a, b)), which needs no sign or magnitude extraction.
// G takes the chunk's partial sums in the low V bits of bb (bit j <->
// element j).
// ---------------------------------------------------------------------------

typedef short s16x2 __attribute__((ext_vector_type(2)));
DEV s16x2 as_s16x2(uint32_t x) { return __builtin_bit_cast(s16x2, x); }
DEV uint32_t as_u32(s16x2 x) { return __builtin_bit_cast(uint32_t, x); }

// F on two 16-bit lanes.
DEV uint32_t f_x2(uint32_t a, uint32_t b) {
    const s16x2 x = as_s16x2(a), y = as_s16x2(b);
    const s16x2 lo = __builtin_elementwise_min(x, y), hi = __builtin_elementwise_max(x, y);
    return as_u32(__builtin_elementwise_max(lo, (s16x2)0 - hi));
}

// y + x on two 16-bit lanes, saturated to [-32768, 32767], then raised to
// at least lo.
DEV uint32_t addsat_x2(uint32_t a, uint32_t b, short lo) {
    const s16x2 z = __builtin_elementwise_add_sat(as_s16x2(a), as_s16x2(b));
    return as_u32(__builtin_elementwise_max(z, (s16x2)lo));
}

// The chunk's 16 low partial-sum bits in both 16-bit halves.
DEV uint32_t rep16(uint32_t bb) { return __builtin_amdgcn_perm(bb, bb, 0x01000100u); }

template <typename T>
struct ChunkFG;

template <>
struct ChunkFG<float> {
    static DEV uint4 clamp(const uint4& x) { return x; }
    // one IEEE min / max each: exact, and a zero's sign never decides
    // anything (hard decisions compare with < 0)
    static DEV uint4 f(const uint4& x, const uint4& y) {
        float o[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float a = __uint_as_float(comp4(x, j)), b = __uint_as_float(comp4(y, j));
            o[j] = __builtin_elementwise_maximum(__builtin_elementwise_minimum(a, b),
                                                 -__builtin_elementwise_maximum(a, b));
        }
        return VecIO<float>::pack(o);
    }
    static DEV uint4 g(const uint4& x, const uint4& y, uint32_t bb) {
        float o[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t xs = comp4(x, j) ^ ((bb << (31 - j)) & 0x80000000u);
            o[j] = __fadd_rn(__uint_as_float(comp4(y, j)), __uint_as_float(xs));
        }
        return VecIO<float>::pack(o);
    }
};

template <>
struct ChunkFG<int16_t> {
    // channel values into [-32767, 32767]
    static DEV uint32_t clamp_w(uint32_t w) {
        return as_u32(__builtin_elementwise_max(as_s16x2(w), (s16x2)(-32767)));
    }
    static DEV uint4 clamp(const uint4& x) {
        return make_uint4(clamp_w(x.x), clamp_w(x.y), clamp_w(x.z), clamp_w(x.w));
    }
    static DEV uint4 f(const uint4& x, const uint4& y) {
        return make_uint4(f_x2(x.x, y.x), f_x2(x.y, y.y), f_x2(x.z, y.z), f_x2(x.w, y.w));
    }
    // word w holds elements 2w (low half) and 2w + 1; m = -beta per half,
    // (x ^ m) - m = beta ? -x : x
    static DEV uint32_t g_word(uint32_t xw, uint32_t yw, uint32_t rep, int w) {
        const s16x2 sh = {(short)(15 - 2 * w), (short)(14 - 2 * w)};
        const s16x2 m = (as_s16x2(rep) << sh) >> (s16x2)15;
        const s16x2 xn = (as_s16x2(xw) ^ m) - m;
        return addsat_x2(yw, as_u32(xn), -32767);
    }
    static DEV uint4 g(const uint4& x, const uint4& y, uint32_t bb) {
        const uint32_t rep = rep16(bb);
        return make_uint4(g_word(x.x, y.x, rep, 0), g_word(x.y, y.y, rep, 1),
                          g_word(x.z, y.z, rep, 2), g_word(x.w, y.w, rep, 3));
    }
};

// int8: each value v goes to the high byte of a 16-bit half (256 v), so the
// 16-bit saturating arithmetic saturates where the byte arithmetic would,
// and the result is the high byte.  For G the low byte carries the partial
// sum as a mask byte B (0xff or 0): with x replaced by x ^ B, the halves
// hold 256 x + 0 or -256 x - 1, y's hold 256 y + B, and their sum has high
// byte y + x or y - x (low byte 0 or 254, no carry).  The clamp to -127
// (0x8100) completes the saturation to [-127, 127].
template <>
struct ChunkFG<int8_t> {
    // channel values into [-127, 127] (via the high bytes of 16-bit halves)
    static DEV uint32_t clamp_w(uint32_t w) {
        const s16x2 lo = __builtin_elementwise_max(as_s16x2(__builtin_amdgcn_perm(0u, w, 0x010c000cu)),
                                                   (s16x2)(-32512));
        const s16x2 hi = __builtin_elementwise_max(as_s16x2(__builtin_amdgcn_perm(0u, w, 0x030c020cu)),
                                                   (s16x2)(-32512));
        return __builtin_amdgcn_perm(as_u32(hi), as_u32(lo), 0x07050301u);
    }
    static DEV uint4 clamp(const uint4& x) {
        return make_uint4(clamp_w(x.x), clamp_w(x.y), clamp_w(x.z), clamp_w(x.w));
    }
    static DEV uint32_t f_word(uint32_t xw, uint32_t yw) {
        const uint32_t z0 = f_x2(__builtin_amdgcn_perm(0u, xw, 0x010c000cu),
                                 __builtin_amdgcn_perm(0u, yw, 0x010c000cu));
        const uint32_t z1 = f_x2(__builtin_amdgcn_perm(0u, xw, 0x030c020cu),
                                 __builtin_amdgcn_perm(0u, yw, 0x030c020cu));
        return __builtin_amdgcn_perm(z1, z0, 0x07050301u);
    }
    static DEV uint4 f(const uint4& x, const uint4& y) {
        return make_uint4(f_word(x.x, y.x), f_word(x.y, y.y), f_word(x.z, y.z), f_word(x.w, y.w));
    }
    // word w holds elements 4w .. 4w + 3 (bytes 0 .. 3)
    static DEV uint32_t g_word(uint32_t xw, uint32_t yw, uint32_t rep, int w) {
        // partial sums 4w, 4w + 1 to bits 15, 31 of s1; 4w + 2, 4w + 3 to
        // bits 15, 31 of s0; the sign-replicating selectors spread them
        // into mask bytes
        const s16x2 sh1 = {(short)(15 - 4 * w), (short)(14 - 4 * w)};
        const s16x2 sh0 = {(short)(13 - 4 * w), (short)(12 - 4 * w)};
        const uint32_t s1 = as_u32(as_s16x2(rep) << sh1);
        const uint32_t s0 = as_u32(as_s16x2(rep) << sh0);
        const uint32_t bm = __builtin_amdgcn_perm(s0, s1, 0x0b0a0908u);
        const uint32_t xp = xw ^ bm;
        const uint32_t z0 = addsat_x2(__builtin_amdgcn_perm(bm, yw, 0x01050004u),
                                      __builtin_amdgcn_perm(bm, xp, 0x01050004u), -32512);
        const uint32_t z1 = addsat_x2(__builtin_amdgcn_perm(bm, yw, 0x03070206u),
                                      __builtin_amdgcn_perm(bm, xp, 0x03070206u), -32512);
        return __builtin_amdgcn_perm(z1, z0, 0x07050301u);
    }
    static DEV uint4 g(const uint4& x, const uint4& y, uint32_t bb) {
        const uint32_t rep = rep16(bb);
        return make_uint4(g_word(x.x, y.x, rep, 0), g_word(x.y, y.y, rep, 1),
                          g_word(x.z, y.z, rep, 2), g_word(x.w, y.w, rep, 3));
    }
};

// ---------------------------------------------------------------------------
// Operation records (built on the host) and kernel arguments.
// ---------------------------------------------------------------------------

// One schedule entry, 8 bytes so that the schedule can sit in LDS.
// meta = type | k << 3 | side << 7 | cand << 8 | in_space << 12 | out_space << 14.
// Operands (x, y, z) and spaces:
//   F, G:     x = LLR stage k (in_space), y = LLR stage k - 1 (out_space),
//             z = left partial sums of level k - 1 (out_space);
//   Combine:  x, y = left, right partial sums of level k - 1 (in_space),
//             z = output partial sums of level k (out_space);
//   leaves:   x = LLR stage k (in_space), y = output partial sums of level k
//             (out_space).
// Offsets are in 16-byte units in LDS and 256-byte units in the workspace.
// Fused records: an F / G with candidate bit 2 also runs the next record's
// F (bit 1: and the F after it, float32), those records becoming no-ops
// that keep their output offset and space; the stage below the root uses
// candidate bits 3 (two recomputed levels) and 0 (under a right child).  A
// float32 forking leaf with z = 1 / 2 forms its values from the previous
// record, an F / G turned no-op with its other fields kept.
struct OpRec {
    uint16_t meta, x, y, z;
};
DEV int op_type(const OpRec& o) { return o.meta & 7; }
DEV int op_k(const OpRec& o) { return (o.meta >> 3) & 15; }
DEV int op_side(const OpRec& o) { return (o.meta >> 7) & 1; }
DEV int op_cand(const OpRec& o) { return (o.meta >> 8) & 15; }
DEV int op_isp(const OpRec& o) { return (o.meta >> 12) & 3; }
DEV int op_osp(const OpRec& o) { return (o.meta >> 14) & 3; }

struct KArgs {
    const OpRec* ops;
    const uint64_t* syn;  // N codeword-domain CRC syndromes
    const uint16_t* info_pos;
    uint8_t* ws;
    int64_t ws_frame;  // workspace bytes per workgroup
    int n_ops, N, n, K, L, has_crc;
    int ptrA_off, ptrB_off, pm_off, root_off, root_sp;
    int vt2_off;  // left partial sums of level n - 2 (stages n - 1, n - 2 recomputed)
    int fuse_k;   // float32: forking leaves of at most 2^fuse_k values run fused (-1: none)
    int rs;  // bytes per path-table row (one byte per tree level, 4-aligned)
    // candidate scratch
    int spm_off, ckey_off, surv_off, sinfo_off;
};

DEV int words_of(int k) { return k >= 5 ? (1 << (k - 5)) : 1; }
DEV int ilog2u(unsigned v) { return 31 - __clz(v); }

// Per-workgroup view of one frame's decoder state.
template <typename T>
struct Ctx {
    unsigned char* lds;
    uint8_t* wsb;
    const T* chan;  // the frame's channel LLRs
    int N, n, L, tid, NT, lane;
    int ptrA_off, ptrB_off, pm_off, rs;
    int spm_off, ckey_off, surv_off, sinfo_off;
    int vt2_off;
    int cur;  // which copy of the path tables is current

    // Path -> buffer tables, one 16-byte row per slot (entry k = tree level
    // k), double-buffered so that a selection can rebuild them from the old
    // rows.  ptrA maps LLR stages, ptrB left partial sums.
    DEV uint8_t* rowA(int buf, int slot) const { return lds + ptrA_off + (buf * L + slot) * rs; }
    DEV uint8_t* rowB(int buf, int slot) const { return lds + ptrB_off + (buf * L + slot) * rs; }
    // copies a row (rs / 4 words)
    DEV void copy_row(uint8_t* dst, const uint8_t* src) const {
#pragma unroll 1
        for (int w = 0; w < (rs >> 2); ++w) ((uint32_t*)dst)[w] = ((const uint32_t*)src)[w];
    }
    DEV int srcA(int k, int slot) const { return rowA(cur, slot)[k]; }
    DEV int srcB(int k, int slot) const { return rowB(cur, slot)[k]; }
    DEV void setA(int k, int slot) const { rowA(cur, slot)[k] = (uint8_t)slot; }
    DEV void setB(int k, int slot) const { rowB(cur, slot)[k] = (uint8_t)slot; }
    DEV typename Dom<T>::M* pm() const { return (typename Dom<T>::M*)(lds + pm_off); }
    // the survivors' ranking keys after a pruning selection, by slot
    DEV uint64_t* skey() const { return (uint64_t*)(lds + spm_off); }
    DEV uint64_t* ckey() const { return (uint64_t*)(lds + ckey_off); }
    DEV uint16_t* surv() const { return (uint16_t*)(lds + surv_off); }
    DEV uint16_t* sinfo() const { return (uint16_t*)(lds + sinfo_off); }
    // LLR stage buffer: space SP, stage offset off (units), node size 2^k.
    template <int SP>
    DEV T* stage(int off, int k, int slot) const {
        if constexpr (SP == SP_WS) return (T*)(wsb + (off << 8)) + (slot << k);
        else return (T*)(lds + (off << 4)) + (slot << k);
    }
    // Partial-sum words of a slot at level k.
    template <int SP>
    DEV uint32_t* bw(int off, int k, int slot) const {
        if constexpr (SP == SP_WS) return (uint32_t*)(wsb + (off << 8)) + slot * words_of(k);
        else return (uint32_t*)(lds + (off << 4)) + slot * words_of(k);
    }
    template <int SP>
    DEV const T* in_stage(int off, int k, int slot) const {
        if constexpr (SP == SP_CH) return chan;
        else return stage<SP>(off, k, slot);
    }
};

// ---------------------------------------------------------------------------
// Lane groups.  Between two forking leaves every operation acts on each path
// on its own (F, G, Combine, Rate-0), so each path is given to a group of G
// lanes inside one wavefront and the whole run of operations proceeds
// without workgroup barriers: memory operations of one wavefront complete in
// issue order, and a wavefront-level fence keeps the compiler from reordering
// them.
// ---------------------------------------------------------------------------

struct Grp {
    int p, g, G;
    bool valid;
};

DEV Grp make_grp(int tid, int NT, int P) {
    const int NW = NT >> 6;
    int ipw = (P + NW - 1) / NW;  // paths per wavefront
    ipw = ipw <= 1 ? 1 : (1 << (32 - __clz(ipw - 1)));
    Grp q;
    q.G = 64 / ipw;
    const int lg = ilog2u(q.G);
    const int lane = tid & 63;
    const int inst = (tid >> 6) * ipw + (lane >> lg);
    q.valid = inst < P;
    q.p = q.valid ? inst : 0;
    q.g = lane & (q.G - 1);
    return q;
}

// Orders this lane's earlier memory operations before its later ones as seen
// by the other lanes of its wavefront.  A wavefront's memory operations are
// performed in order, so at wavefront scope this costs no wait: the fences
// only keep the compiler from moving memory operations across it.
DEV void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// Per-path operations.
// ---------------------------------------------------------------------------

// F / G of one path at a level-k node, eqs. (f) and (g): lane g of the group
// takes 16-byte chunks g, g + G, ..., up to U of them loaded before any is
// stored.  The left partial sums of G share the output's space.
// F / G at the level below the root reading that level's stage without
// storing it: element j of the node's input is F(ch[j], ch[j + N/2]) for the
// root's left child and G(ch[j], ch[j + N/2], b[j]) with the path's
// left-half partial sums b (op.x, in the workspace) for its right child
// (op side bit).  Same arithmetic, in the same order, as storing it.
template <typename T, bool IS_G, int OSP>
DEV void pp_fg_virtual(const Ctx<T>& c, const OpRec& op, int k, const Grp& q) {
    using IO = VecIO<T>;
    constexpr int LOGV = IO::LOGV;
    const int M = 1 << (k - 1);  // outputs; the node has 2M inputs, the channel 4M
    const bool right = op_side(op) != 0;
    const T* ch = c.chan;
    T* out = c.template stage<OSP>(op.y, k - 1, q.p);
    const uint32_t* bl = nullptr;
    if constexpr (IS_G) bl = c.template bw<OSP>(op.z, k - 1, c.srcB(k - 1, q.p));
    const uint32_t* br = right ? c.template bw<SP_WS>(op.x, k, c.srcB(k, q.p)) : nullptr;
    const int nch = M >> LOGV;
    auto bits = [&](const uint32_t* w, int e) { return w[e >> 5] >> (e & 31); };
    for (int ch0 = q.g; ch0 < nch; ch0 += q.G) {
        const int e = ch0 << LOGV;  // first output element of the chunk
        // the node's inputs e.. and M + e.. from channel elements e, e + 2M,
        // M + e, 3M + e
        const uint4 c0 = ChunkFG<T>::clamp(*(const uint4*)(ch + e));
        const uint4 c2 = ChunkFG<T>::clamp(*(const uint4*)(ch + 2 * M + e));
        const uint4 c1 = ChunkFG<T>::clamp(*(const uint4*)(ch + M + e));
        const uint4 c3 = ChunkFG<T>::clamp(*(const uint4*)(ch + 3 * M + e));
        uint4 x, y;
        if (right) {
            x = ChunkFG<T>::g(c0, c2, bits(br, e));
            y = ChunkFG<T>::g(c1, c3, bits(br, M + e));
        } else {
            x = ChunkFG<T>::f(c0, c2);
            y = ChunkFG<T>::f(c1, c3);
        }
        uint4 r;
        if constexpr (IS_G) r = ChunkFG<T>::g(x, y, bits(bl, e));
        else r = ChunkFG<T>::f(x, y);
        *(uint4*)(out + e) = r;
    }
    if (q.g == 0) c.setA(k - 1, q.p);
}

// F / G two levels below the root (k = n - 2) reading the node's input
// without either stage above it being stored: with the channel of 8M values
// (M = node outputs), stage n - 1 is a1[i] = F(ch[i], ch[i + 4M]) in the
// root's left half or G(ch[i], ch[i + 4M], b1[i]) in its right half (b1 =
// the root-left partial sums, op.x), and the node's input is a2[j] =
// F(a1[j], a1[j + 2M]) under a left level-(n-1) parent or G(a1[j],
// a1[j + 2M], b2[j]) under a right one (b2 = that parent's left partial
// sums, at the plan's vt2_off).  Flags: side bit = right half of the root,
// candidate-count bit 0 = right child of its level-(n-1) parent.  Same
// arithmetic, in the same order, as storing both stages.
template <typename T, bool IS_G, int OSP>
DEV void pp_fg_virtual2(const Ctx<T>& c, const OpRec& op, int k, const Grp& q) {
    using IO = VecIO<T>;
    using CF = ChunkFG<T>;
    constexpr int LOGV = IO::LOGV;
    const int M = 1 << (k - 1);
    const bool right1 = op_side(op) != 0;
    const bool right2 = (op_cand(op) & 1) != 0;
    const T* ch = c.chan;
    T* out = c.template stage<OSP>(op.y, k - 1, q.p);
    const uint32_t* bl = nullptr;
    if constexpr (IS_G) bl = c.template bw<OSP>(op.z, k - 1, c.srcB(k - 1, q.p));
    const uint32_t* b1 = right1 ? c.template bw<SP_WS>(op.x, k + 1, c.srcB(k + 1, q.p)) : nullptr;
    const uint32_t* b2 = right2 ? c.template bw<SP_WS>(c.vt2_off, k, c.srcB(k, q.p)) : nullptr;
    const int nch = M >> LOGV;
    auto bits = [&](const uint32_t* w, int e) { return w[e >> 5] >> (e & 31); };
    auto ld = [&](int i) { return CF::clamp(*(const uint4*)(ch + i)); };
    auto op1 = [&](const uint4& u, const uint4& v, int i) {
        return right1 ? CF::g(u, v, bits(b1, i)) : CF::f(u, v);
    };
    auto op2 = [&](const uint4& u, const uint4& v, int j) {
        return right2 ? CF::g(u, v, bits(b2, j)) : CF::f(u, v);
    };
    for (int ch0 = q.g; ch0 < nch; ch0 += q.G) {
        const int e = ch0 << LOGV;
        // stage n - 1 at e, e + 2M (for input e) and M + e, 3M + e (for
        // input M + e), each from channel elements i and i + 4M
        const uint4 c0 = ld(e), c1 = ld(e + 4 * M);
        const uint4 c2 = ld(e + 2 * M), c3 = ld(e + 6 * M);
        const uint4 c4 = ld(M + e), c5 = ld(5 * M + e);
        const uint4 c6 = ld(3 * M + e), c7 = ld(7 * M + e);
        const uint4 x = op2(op1(c0, c1, e), op1(c2, c3, e + 2 * M), e);
        const uint4 y = op2(op1(c4, c5, M + e), op1(c6, c7, 3 * M + e), M + e);
        uint4 r;
        if constexpr (IS_G) r = CF::g(x, y, bits(bl, e));
        else r = CF::f(x, y);
        *(uint4*)(out + e) = r;
    }
    if (q.g == 0) c.setA(k - 1, q.p);
}

template <typename T, bool IS_G, int ISP, int OSP>
DEV void pp_fg(const Ctx<T>& c, const OpRec& op, int k, const Grp& q) {
    using IO = VecIO<T>;
    using D = Dom<T>;
    using A = typename D::A;
    constexpr int V = IO::V;
    constexpr int LOGV = IO::LOGV;
    constexpr int U = 4;
    if (!q.valid) return;
    const int M = 1 << (k - 1);
    if constexpr (ISP == SP_VT) {
        // two recomputed levels are not offered for int8 (their eight
        // clamped channel chunks per output chunk), so its kernels do not
        // carry that code
        if constexpr (!std::is_same<T, int8_t>::value) {
            if (op_cand(op) & 8) {
                pp_fg_virtual2<T, IS_G, OSP>(c, op, k, q);
                return;
            }
        }
        pp_fg_virtual<T, IS_G, OSP>(c, op, k, q);
        return;
    }
    const T* in = c.template in_stage<ISP>(op.x, k, ISP == SP_CH ? 0 : c.srcA(k, q.p));
    T* out = c.template stage<OSP>(op.y, k - 1, q.p);
    const uint32_t* bl = nullptr;
    if constexpr (IS_G) bl = c.template bw<OSP>(op.z, k - 1, c.srcB(k - 1, q.p));
    if (M >= V) {
        const int nch = M >> LOGV;
        for (int ch0 = q.g; ch0 < nch; ch0 += q.G * U) {
            uint4 xq[U], yq[U];
            uint32_t bb[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int ch = ch0 + u * q.G;
                const int chc = ch < nch ? ch : ch0;
                xq[u] = *(const uint4*)(in + (chc << LOGV));
                yq[u] = *(const uint4*)(in + M + (chc << LOGV));
                if constexpr (IS_G) bb[u] = bl[(chc << LOGV) >> 5] >> ((chc << LOGV) & 31);
                else bb[u] = 0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int ch = ch0 + u * q.G;
                if (ch >= nch) continue;
                uint4 r;
                if constexpr (ISP != SP_CH || std::is_same<T, float>::value) {
                    // stage values are already within range
                    if constexpr (IS_G) r = ChunkFG<T>::g(xq[u], yq[u], bb[u]);
                    else r = ChunkFG<T>::f(xq[u], yq[u]);
                } else {
                    // channel values are clamped into range first
                    A x[V], y[V], o[V];
                    IO::unpack(xq[u], x);
                    IO::unpack(yq[u], y);
#pragma unroll
                    for (int j = 0; j < V; ++j) {
                        const A xa = D::load(x[j]), ya = D::load(y[j]);
                        if constexpr (IS_G) o[j] = D::g(xa, ya, (bb[u] >> j) & 1u);
                        else o[j] = D::f(xa, ya);
                    }
                    r = IO::pack(o);
                }
                *(uint4*)(out + (ch << LOGV)) = r;
            }
        }
    } else {
        for (int i = q.g; i < M; i += q.G) {
            const A x = D::load(in[i]);
            const A y = D::load(in[i + M]);
            A v;
            if constexpr (IS_G) v = D::g(x, y, (bl[i >> 5] >> (i & 31)) & 1u);
            else v = D::f(x, y);
            out[i] = (T)v;
        }
    }
    if (q.g == 0) c.setA(k - 1, q.p);
}

// F or G at a level-k node followed at once by the F of its left child
// (two tree levels in one pass; the child's record then does nothing): lane
// g of the group takes output chunks g, g + G, ... of the child's F, forms
// for each the two chunks of the node's output that this F combines from
// four input chunks, stores both (the child's G reads them later) and stores
// the F's chunk.  The child's input is never re-read.  Same arithmetic, in
// the same order, as the two operations.
template <typename T, bool IS_G, int ISP, int OSP1, int OSP2>
DEV void pp_fg_chain(const Ctx<T>& c, const OpRec& op, int y2, int k, const Grp& q) {
    using IO = VecIO<T>;
    using CF = ChunkFG<T>;
    constexpr int LOGV = IO::LOGV;
    // int8 (one wavefront per frame, five per SIMD) keeps its registers
    // within that budget with one chunk in flight
    constexpr int U = sizeof(T) == 1 ? 1 : 2;
    if (!q.valid) return;
    const int M = 1 << (k - 1);  // the node's outputs
    const int H = M >> 1;        // the child's F outputs
    const T* in = c.template stage<ISP>(op.x, k, c.srcA(k, q.p));
    T* mid = c.template stage<OSP1>(op.y, k - 1, q.p);
    T* out = c.template stage<OSP2>(y2, k - 2, q.p);
    const uint32_t* bl = nullptr;
    if constexpr (IS_G) bl = c.template bw<OSP1>(op.z, k - 1, c.srcB(k - 1, q.p));
    const int nch = H >> LOGV;
    for (int ch0 = q.g; ch0 < nch; ch0 += q.G * U) {
        uint4 a0[U], a1[U], b0[U], b1[U];
        uint32_t s0[U], s1[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int ch = ch0 + u * q.G;
            const int e = (ch < nch ? ch : ch0) << LOGV;
            a0[u] = *(const uint4*)(in + e);
            a1[u] = *(const uint4*)(in + M + e);
            b0[u] = *(const uint4*)(in + H + e);
            b1[u] = *(const uint4*)(in + M + H + e);
            if constexpr (IS_G) {
                s0[u] = bl[e >> 5] >> (e & 31);
                s1[u] = bl[(H + e) >> 5] >> ((H + e) & 31);
            } else {
                s0[u] = s1[u] = 0;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int ch = ch0 + u * q.G;
            if (ch >= nch) continue;
            const int e = ch << LOGV;
            uint4 x, y;
            if constexpr (IS_G) {
                x = CF::g(a0[u], a1[u], s0[u]);
                y = CF::g(b0[u], b1[u], s1[u]);
            } else {
                x = CF::f(a0[u], a1[u]);
                y = CF::f(b0[u], b1[u]);
            }
            *(uint4*)(mid + e) = x;
            *(uint4*)(mid + H + e) = y;
            *(uint4*)(out + e) = CF::f(x, y);
        }
    }
    if (q.g == 0) {
        c.setA(k - 1, q.p);
        c.setA(k - 2, q.p);
    }
}

// Three tree levels in one pass (float32): an F or G at a level-k node, the
// F of its left child and the F of that child's left child, the two F
// records then doing nothing.  For each output chunk e of the last F
// (Q = 2^(k-3) outputs), a lane loads the eight input chunks e + jQ, forms
// the node's four output chunks e + jQ (j < 4), the child's two (e, Q + e)
// and the grandchild's one, and stores all seven; no stage is re-read.
template <typename T, bool IS_G, int ISP, int OSP1, int OSP2, int OSP3>
DEV void pp_fg_chain3(const Ctx<T>& c, const OpRec& op, int y2, int y3, int k, const Grp& q) {
    using CF = ChunkFG<T>;
    constexpr int LOGV = VecIO<T>::LOGV;
    if (!q.valid) return;
    const int M = 1 << (k - 1);  // the node's outputs
    const int Q = M >> 2;        // the grandchild's F outputs
    const T* in = c.template stage<ISP>(op.x, k, c.srcA(k, q.p));
    T* m1 = c.template stage<OSP1>(op.y, k - 1, q.p);
    T* m2 = c.template stage<OSP2>(y2, k - 2, q.p);
    T* m3 = c.template stage<OSP3>(y3, k - 3, q.p);
    const uint32_t* bl = nullptr;
    if constexpr (IS_G) bl = c.template bw<OSP1>(op.z, k - 1, c.srcB(k - 1, q.p));
    const int nch = Q >> LOGV;
    for (int ch = q.g; ch < nch; ch += q.G) {
        const int e = ch << LOGV;
        uint4 a[4], b[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            a[j] = *(const uint4*)(in + e + j * Q);
            b[j] = *(const uint4*)(in + M + e + j * Q);
        }
        uint4 x[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if constexpr (IS_G) {
                const int i = e + j * Q;
                x[j] = CF::g(a[j], b[j], bl[i >> 5] >> (i & 31));
            } else {
                x[j] = CF::f(a[j], b[j]);
            }
            *(uint4*)(m1 + e + j * Q) = x[j];
        }
        const uint4 y0 = CF::f(x[0], x[2]);
        const uint4 y1 = CF::f(x[1], x[3]);
        *(uint4*)(m2 + e) = y0;
        *(uint4*)(m2 + Q + e) = y1;
        *(uint4*)(m3 + e) = CF::f(y0, y1);
    }
    if (q.g == 0) {
        c.setA(k - 1, q.p);
        c.setA(k - 2, q.p);
        c.setA(k - 3, q.p);
    }
}

// The F / G below the root reading the recomputed stage (as pp_fg_virtual)
// chained with its left child's F: for each output chunk e of the child's F,
// the node's output chunks e and H + e (four channel chunks each), both
// stored, and their F.
template <typename T, bool IS_G, int OSP1, int OSP2>
DEV void pp_fg_virtual_chain(const Ctx<T>& c, const OpRec& op, int y2, int k, const Grp& q) {
    using CF = ChunkFG<T>;
    constexpr int LOGV = VecIO<T>::LOGV;
    if (!q.valid) return;
    const int M = 1 << (k - 1);  // the node's outputs; the channel has 4M values
    const int H = M >> 1;
    const bool right = op_side(op) != 0;
    const T* ch = c.chan;
    T* mid = c.template stage<OSP1>(op.y, k - 1, q.p);
    T* out = c.template stage<OSP2>(y2, k - 2, q.p);
    const uint32_t* bl = nullptr;
    if constexpr (IS_G) bl = c.template bw<OSP1>(op.z, k - 1, c.srcB(k - 1, q.p));
    const uint32_t* br = right ? c.template bw<SP_WS>(op.x, k, c.srcB(k, q.p)) : nullptr;
    auto bits = [&](const uint32_t* w, int e) { return w[e >> 5] >> (e & 31); };
    auto node_out = [&](int e) {
        const uint4 c0 = CF::clamp(*(const uint4*)(ch + e));
        const uint4 c2 = CF::clamp(*(const uint4*)(ch + 2 * M + e));
        const uint4 c1 = CF::clamp(*(const uint4*)(ch + M + e));
        const uint4 c3 = CF::clamp(*(const uint4*)(ch + 3 * M + e));
        uint4 x, y;
        if (right) {
            x = CF::g(c0, c2, bits(br, e));
            y = CF::g(c1, c3, bits(br, M + e));
        } else {
            x = CF::f(c0, c2);
            y = CF::f(c1, c3);
        }
        if constexpr (IS_G) return CF::g(x, y, bits(bl, e));
        else return CF::f(x, y);
    };
    const int nch = H >> LOGV;
    for (int ch0 = q.g; ch0 < nch; ch0 += q.G) {
        const int e = ch0 << LOGV;
        const uint4 a = node_out(e);
        const uint4 b = node_out(H + e);
        *(uint4*)(mid + e) = a;
        *(uint4*)(mid + H + e) = b;
        *(uint4*)(out + e) = CF::f(a, b);
    }
    if (q.g == 0) {
        c.setA(k - 1, q.p);
        c.setA(k - 2, q.p);
    }
}

// The chained form's spaces: input, node output and child output, each in
// LDS or the workspace, a level in LDS only if every level below it is.
template <typename T, bool IS_G>
DEV void pp_fg_chain_any(const Ctx<T>& c, const OpRec& op, uint64_t next, uint64_t next2, int k,
                         const Grp& q) {
    const int isp = op_isp(op);
    const int osp = op_osp(op);
    const int y2 = (int)(uint16_t)(next >> 32);
    const int osp2 = ((int)(uint16_t)next >> 14) & 3;
    if constexpr (std::is_same<T, float>::value) {
        if (op_cand(op) & 2) {
            // three levels (candidate bit 1): the record after next holds the
            // grandchild's F output
            const int y3 = (int)(uint16_t)(next2 >> 32);
            const int osp3 = ((int)(uint16_t)next2 >> 14) & 3;
            if (isp == SP_LDS)
                pp_fg_chain3<T, IS_G, SP_LDS, SP_LDS, SP_LDS, SP_LDS>(c, op, y2, y3, k, q);
            else if (osp == SP_LDS)
                pp_fg_chain3<T, IS_G, SP_WS, SP_LDS, SP_LDS, SP_LDS>(c, op, y2, y3, k, q);
            else if (osp2 == SP_LDS)
                pp_fg_chain3<T, IS_G, SP_WS, SP_WS, SP_LDS, SP_LDS>(c, op, y2, y3, k, q);
            else if (osp3 == SP_LDS)
                pp_fg_chain3<T, IS_G, SP_WS, SP_WS, SP_WS, SP_LDS>(c, op, y2, y3, k, q);
            else
                pp_fg_chain3<T, IS_G, SP_WS, SP_WS, SP_WS, SP_WS>(c, op, y2, y3, k, q);
            return;
        }
    }
    if constexpr (std::is_same<T, float>::value) {
        // the recomputed stage below the root (chained for float32 only)
        if (isp == SP_VT) {
            if (osp == SP_LDS) pp_fg_virtual_chain<T, IS_G, SP_LDS, SP_LDS>(c, op, y2, k, q);
            else if (osp2 == SP_LDS) pp_fg_virtual_chain<T, IS_G, SP_WS, SP_LDS>(c, op, y2, k, q);
            else pp_fg_virtual_chain<T, IS_G, SP_WS, SP_WS>(c, op, y2, k, q);
            return;
        }
    }
    if (isp == SP_LDS) pp_fg_chain<T, IS_G, SP_LDS, SP_LDS, SP_LDS>(c, op, y2, k, q);
    else if (osp == SP_LDS) pp_fg_chain<T, IS_G, SP_WS, SP_LDS, SP_LDS>(c, op, y2, k, q);
    else if (osp2 == SP_LDS) pp_fg_chain<T, IS_G, SP_WS, SP_WS, SP_LDS>(c, op, y2, k, q);
    else pp_fg_chain<T, IS_G, SP_WS, SP_WS, SP_WS>(c, op, y2, k, q);
}

template <typename T, bool IS_G>
DEV void pp_fg_any(const Ctx<T>& c, const OpRec& op, int k, const Grp& q) {
    const int isp = op_isp(op);
    const int osp = op_osp(op);
    if (isp == SP_LDS) pp_fg<T, IS_G, SP_LDS, SP_LDS>(c, op, k, q);
    else if (isp == SP_WS) {
        if (osp == SP_WS) pp_fg<T, IS_G, SP_WS, SP_WS>(c, op, k, q);
        else pp_fg<T, IS_G, SP_WS, SP_LDS>(c, op, k, q);
    } else if (isp == SP_VT) {
        if (osp == SP_WS) pp_fg<T, IS_G, SP_VT, SP_WS>(c, op, k, q);
        else pp_fg<T, IS_G, SP_VT, SP_LDS>(c, op, k, q);
    } else {
        if (osp == SP_WS) pp_fg<T, IS_G, SP_CH, SP_WS>(c, op, k, q);
        else pp_fg<T, IS_G, SP_CH, SP_LDS>(c, op, k, q);
    }
}

// Combine, eq. (combine), on bit-packed words: beta_v = (beta_l ^ beta_r, beta_r).
template <typename T, int ISP, int OSP>
DEV void pp_comb(const Ctx<T>& c, const OpRec& op, int k, int side, const Grp& q) {
    if (!q.valid) return;
    const int W = words_of(k);
    const uint32_t* l = c.template bw<ISP>(op.x, k - 1, c.srcB(k - 1, q.p));
    const uint32_t* r = c.template bw<ISP>(op.y, k - 1, q.p);
    uint32_t* o = c.template bw<OSP>(op.z, k, q.p);
    if (k >= 6) {
        const int hw = W >> 1;
        for (int w = q.g; w < hw; w += q.G) {
            const uint32_t lv = l[w], rv = r[w];
            o[w] = lv ^ rv;
            o[w + hw] = rv;
        }
    } else if (q.g == 0) {
        const int h = 1 << (k - 1);
        const uint32_t m = (1u << h) - 1u;
        const uint32_t lv = l[0] & m, rv = r[0] & m;
        o[0] = (lv ^ rv) | (rv << h);
    }
    if (side == 0 && q.g == 0) c.setB(k, q.p);
}

template <typename T>
DEV void pp_comb_any(const Ctx<T>& c, const OpRec& op, int k, int side, const Grp& q) {
    const int isp = op_isp(op), osp = op_osp(op);
    if (isp == SP_LDS && osp == SP_LDS) pp_comb<T, SP_LDS, SP_LDS>(c, op, k, side, q);
    else if (isp == SP_LDS) pp_comb<T, SP_LDS, SP_WS>(c, op, k, side, q);
    else pp_comb<T, SP_WS, SP_WS>(c, op, k, side, q);
}

// ---------------------------------------------------------------------------
// Leaf list decoders.
// ---------------------------------------------------------------------------

// Candidate flip sets of the SPC decoder over the four least reliable bits
// m1..m4 (bit t <-> m_{t+1}), relative to the ML word: {}, {1,2}, {1,3},
// {1,4}, {2,3}, {2,4}, {3,4}, {1,2,3,4} (Sec. III-D).
// Packed as nibbles: rank r's set is (kSpcFlips >> 4r) & 0xF.
constexpr uint32_t kSpcFlips = 0xFCA69530u;
DEV uint32_t spc_flips(int r) { return (kSpcFlips >> (4 * r)) & 0xFu; }

DEV uint64_t umin64(uint64_t a, uint64_t b) { return a < b ? a : b; }
DEV uint64_t umax64(uint64_t a, uint64_t b) { return a < b ? b : a; }

// ---------------------------------------------------------------------------
// Exchanges between lanes i and i ^ M of a wavefront in VALU (DPP and the
// permlane swaps), without the LDS round trip of a permute.  On return
// {a, b} = {this lane's value, lane (i ^ M)'s value}, in an order that may
// depend on the lane, which is all that compare-exchanges and symmetric
// reductions need.  Every lane of the wavefront must be active.
// ---------------------------------------------------------------------------

template <int CTRL>
DEV uint32_t dpp(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xf, 0xf, true);
}

template <int M>
DEV void xpair32(uint32_t v, uint32_t& a, uint32_t& b) {
    if constexpr (M == 1) {
        a = v;
        b = dpp<0xb1>(v);  // quad_perm [1,0,3,2]
    } else if constexpr (M == 2) {
        a = v;
        b = dpp<0x4e>(v);  // quad_perm [2,3,0,1]
    } else if constexpr (M == 4) {
        a = v;
        b = dpp<0x141>(dpp<0x1b>(v));  // (i ^ 3) ^ 7: quad_perm [3,2,1,0], row_half_mirror
    } else if constexpr (M == 8) {
        a = v;
        b = dpp<0x128>(v);  // row_ror:8
    } else if constexpr (M == 16) {
        const auto sw = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        a = sw[0];
        b = sw[1];
    } else {
        static_assert(M == 32, "lane distance");
        const auto sw = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        a = sw[0];
        b = sw[1];
    }
}

template <int M>
DEV void xpair64(uint64_t v, uint64_t& a, uint64_t& b) {
    uint32_t al, bl, ah, bh;
    xpair32<M>((uint32_t)v, al, bl);
    xpair32<M>((uint32_t)(v >> 32), ah, bh);
    a = ((uint64_t)ah << 32) | al;
    b = ((uint64_t)bh << 32) | bl;
}

// The same for a distance m known only at run time (uniform across the
// wavefront); after unrolling with a constant m the switch folds away.
// Either key width.
template <int M>
DEV void xpair(uint32_t v, uint32_t& a, uint32_t& b) {
    xpair32<M>(v, a, b);
}
template <int M>
DEV void xpair(uint64_t v, uint64_t& a, uint64_t& b) {
    xpair64<M>(v, a, b);
}
template <typename K>
DEV void xpair_dyn(K v, int m, K& a, K& b) {
    switch (m) {
        case 1: xpair<1>(v, a, b); break;
        case 2: xpair<2>(v, a, b); break;
        case 4: xpair<4>(v, a, b); break;
        case 8: xpair<8>(v, a, b); break;
        case 16: xpair<16>(v, a, b); break;
        default: xpair<32>(v, a, b); break;
    }
}

DEV void xpair64_dyn(uint64_t v, int m, uint64_t& a, uint64_t& b) {
    switch (m) {
        case 1: xpair64<1>(v, a, b); break;
        case 2: xpair64<2>(v, a, b); break;
        case 4: xpair64<4>(v, a, b); break;
        case 8: xpair64<8>(v, a, b); break;
        case 16: xpair64<16>(v, a, b); break;
        default: xpair64<32>(v, a, b); break;
    }
}

// Calls fn(integral_constant<M>) for M = 1, 2, 4, ... below G (G a power
// of two, at most 64): the steps of a butterfly over groups of G lanes.
template <typename Fn>
DEV void xor_steps(int G, Fn&& fn) {
    if (G > 1) fn(std::integral_constant<int, 1>{});
    if (G > 2) fn(std::integral_constant<int, 2>{});
    if (G > 4) fn(std::integral_constant<int, 4>{});
    if (G > 8) fn(std::integral_constant<int, 8>{});
    if (G > 16) fn(std::integral_constant<int, 16>{});
    if (G > 32) fn(std::integral_constant<int, 32>{});
}

// Sum over each group of G lanes (every lane gets the group's sum).
// Integers are exact; doubles here hold sums of single-precision values,
// which are exact as long as they span fewer than 2^29 binades of spread.
DEV int group_sum(int v, int G) {
    xor_steps(G, [&](auto mc) {
        uint32_t a, b;
        xpair32<decltype(mc)::value>((uint32_t)v, a, b);
        v = (int)a + (int)b;
    });
    return v;
}
DEV double group_sum(double v, int G) {
    xor_steps(G, [&](auto mc) {
        uint64_t a, b;
        xpair64<decltype(mc)::value>((uint64_t)__double_as_longlong(v), a, b);
        v = __longlong_as_double((long long)a) + __longlong_as_double((long long)b);
    });
    return v;
}

// The 4 smallest of two ascending 4-lists, ascending (bitonic split of a
// against reversed b, then a 4-element bitonic merge).
template <typename K>
DEV K kmin(K a, K b) {
    return a < b ? a : b;
}
template <typename K>
DEV K kmax(K a, K b) {
    return a < b ? b : a;
}

template <typename K>
DEV void merge4(K* a, const K* b) {
    const K l0 = kmin(a[0], b[3]), l1 = kmin(a[1], b[2]);
    const K l2 = kmin(a[2], b[1]), l3 = kmin(a[3], b[0]);
    const K x0 = kmin(l0, l2), x2 = kmax(l0, l2);
    const K x1 = kmin(l1, l3), x3 = kmax(l1, l3);
    a[0] = kmin(x0, x1);
    a[1] = kmax(x0, x1);
    a[2] = kmin(x2, x3);
    a[3] = kmax(x2, x3);
}

template <typename K>
DEV void insert4(K* kk, K key) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const K lo = kmin(kk[q], key);
        key = kmax(kk[q], key);
        kk[q] = lo;
    }
}

// Visits every element of one path's leaf input: lane g of a group of G lanes
// takes chunks g, g + G, ... of one 16-byte vector (of single elements when
// the node is shorter than a vector), two chunks loaded at a time.
// fn(index, value).
template <typename T, int ISP, class Fn>
DEV void leaf_scan(const T* in, int nv, int g, int G, Fn fn) {
    using IO = VecIO<T>;
    using D = Dom<T>;
    using A = typename D::A;
    if (nv >= IO::V) {
        const int nch = nv >> IO::LOGV;
        for (int ch = g; ch < nch; ch += 2 * G) {
            const int ch2 = ch + G;
            const uint4 q0 = *(const uint4*)(in + (ch << IO::LOGV));
            const uint4 q1 = *(const uint4*)(in + ((ch2 < nch ? ch2 : ch) << IO::LOGV));
            A v[IO::V];
            IO::unpack(q0, v);
#pragma unroll
            for (int j = 0; j < IO::V; ++j)
                fn((ch << IO::LOGV) + j, (ISP == SP_CH) ? D::load(v[j]) : v[j]);
            if (ch2 < nch) {
                IO::unpack(q1, v);
#pragma unroll
                for (int j = 0; j < IO::V; ++j)
                    fn((ch2 << IO::LOGV) + j, (ISP == SP_CH) ? D::load(v[j]) : v[j]);
            }
        }
    } else {
        for (int i = g; i < nv; i += G) fn(i, D::load(in[i]));
    }
}

// Hard decisions (eq. (info)) of elements 32w .. 32w + 31 of a leaf input
// as one word (bit x = element 32w + x; nodes shorter than 32 use the low
// bits).
template <typename T>
DEV uint32_t hd_word(const T* in, int w, int nv) {
    using IO = VecIO<T>;
    using D = Dom<T>;
    using A = typename D::A;
    const T* iw = in + (w << 5);
    const int nb = nv < 32 ? nv : 32;
    uint32_t word = 0u;
    if (nb >= IO::V) {
        constexpr int NQ = 32 / IO::V;
        uint4 v4[NQ];
        const int nq = nb >> IO::LOGV;
#pragma unroll
        for (int t = 0; t < NQ; ++t)
            if (t < nq) v4[t] = *(const uint4*)(iw + (t << IO::LOGV));
#pragma unroll
        for (int t = 0; t < NQ; ++t) {
            if (t >= nq) break;
            A v[IO::V];
            IO::unpack(v4[t], v);
#pragma unroll
            for (int x = 0; x < IO::V; ++x)
                word |= (D::load(v[x]) < 0 ? 1u : 0u) << ((t << IO::LOGV) + x);
        }
    } else {
        for (int x = 0; x < nb; ++x) word |= (D::load(iw[x]) < 0 ? 1u : 0u) << x;
    }
    return word;
}

// Rate-0 of one path, Sec. III-B: the metric loses the distance of the
// all-zero word (eq. (rel:frozen-h)); the output is all zeros.
template <typename T, int ISP, int OSP>
DEV void pp_rate0(const Ctx<T>& c, const OpRec& op, int k, int side, const Grp& q) {
    using D = Dom<T>;
    using A = typename D::A;
    using S = typename D::S;
    const int nv = 1 << k;
    const T* in = c.template in_stage<ISP>(op.x, k, ISP == SP_CH ? 0 : c.srcA(k, q.p));
    S s = 0;
    if (q.valid) {
        leaf_scan<T, ISP>(in, nv, q.g, q.G, [&](int, A v) {
            if (v < 0) s += D::widen_abs(v);
        });
    }
    s = group_sum(s, q.G);
    if (!q.valid) return;
    if (q.g == 0) c.pm()[q.p] = D::sub(c.pm()[q.p], D::round_pen(s));
    uint32_t* o = c.template bw<OSP>(op.y, k, q.p);
    for (int w = q.g; w < words_of(k); w += q.G) o[w] = 0u;
    if (side == 0 && q.g == 0) c.setB(k, q.p);
}

// Pass 1 of a forking leaf for one source path: its statistics and the
// metrics of its candidates, in rank order (the ML candidate first).
template <typename T, int TYPE, int ISP>
DEV void pp_fork_score(const Ctx<T>& c, const OpRec& op, int k, int ccount, const Grp& q) {
    using D = Dom<T>;
    using A = typename D::A;
    using S = typename D::S;
    using M = typename D::M;
    const int nv = 1 << k;
    const int lc = ilog2u(ccount);
    const int s = q.p;
    const T* in = c.template in_stage<ISP>(op.x, k, ISP == SP_CH ? 0 : c.srcA(k, s));
    using RK = Rank<T>;
    typename RK::K* ck = (typename RK::K*)c.ckey() + (s << lc);
    uint16_t* si = c.sinfo() + s * 8;
    const M pms = c.pm()[s];
    auto put = [&](int r, M v) { ck[r] = RK::make(v, (s << lc) + r); };
    if constexpr (TYPE == OP_REP) {
        // penalties of the all-zero and all-one words (Sec. III-E)
        S z = 0, o = 0;
        if (q.valid) {
            leaf_scan<T, ISP>(in, nv, q.g, q.G, [&](int, A v) {
                if (v < 0) z += D::widen_abs(v);
                else o += D::widen_abs(v);
            });
        }
        z = group_sum(z, q.G);
        o = group_sum(o, q.G);
        if (q.valid && q.g == 0) {
            const M zr = D::round_pen(z), orr = D::round_pen(o);
            const bool one = orr < zr;  // ML word first; equal -> all-zero
            put(0, D::sub(pms, one ? orr : zr));
            put(1, D::sub(pms, one ? zr : orr));
            si[4] = one ? 1 : 0;
        }
    } else if constexpr (TYPE == OP_R1) {
        if (k == 0) {
            if (q.valid && q.g == 0) {
                const A v = D::load(in[0]);
                put(0, pms);
                put(1, D::sub(pms, D::round_pen(D::widen_abs(v))));
                si[4] = (v < 0) ? 1 : 0;
            }
        } else {
            // two least reliable positions, ties to the lower index
            using LK = typename Lrb<T>::K;
            LK k1 = ~LK(0), k2 = ~LK(0);
            uint32_t hd = 0u;  // hard decisions of a node of at most 32 values
            if (q.valid) {
                leaf_scan<T, ISP>(in, nv, q.g, q.G, [&](int i, A v) {
                    if (nv <= 32) hd |= (v < 0 ? 1u : 0u) << i;
                    const LK key = Lrb<T>::make(v, i);
                    const LK lo = kmin(k1, key);
                    k2 = kmin(kmax(k1, key), k2);
                    k1 = lo;
                });
            }
            xor_steps(q.G, [&](auto mc) {
                constexpr int M = decltype(mc)::value;
                LK a1, b1, a2, b2;
                xpair<M>(k1, a1, b1);
                xpair<M>(k2, a2, b2);
                k1 = kmin(a1, b1);
                k2 = kmin(kmax(a1, b1), kmin(a2, b2));
                uint32_t ha, hb;
                xpair32<M>(hd, ha, hb);
                hd = ha | hb;
            });
            if (q.valid && q.g == 0) {
                const S a1 = Lrb<T>::mag(k1);
                const S a2 = Lrb<T>::mag(k2);
                put(0, pms);
                put(1, D::sub(pms, D::round_pen(a1)));
                put(2, D::sub(pms, D::round_pen(a2)));
                put(3, D::sub(pms, D::round_pen(a1 + a2)));
                si[0] = (uint16_t)Lrb<T>::idx(k1);
                si[1] = (uint16_t)Lrb<T>::idx(k2);
                si[6] = (uint16_t)hd;
                si[7] = (uint16_t)(hd >> 16);
            }
        }
    } else {  // OP_SPC
        using LK = typename Lrb<T>::K;
        LK kk[4] = {~LK(0), ~LK(0), ~LK(0), ~LK(0)};
        int par = 0;
        uint32_t hd = 0u;  // hard decisions of a node of at most 32 values
        if (q.valid) {
            leaf_scan<T, ISP>(in, nv, q.g, q.G, [&](int i, A v) {
                par ^= (v < 0) ? 1 : 0;
                if (nv <= 32) hd |= (v < 0 ? 1u : 0u) << i;
                insert4(kk, Lrb<T>::make(v, i));
            });
        }
        xor_steps(q.G, [&](auto mc) {
            constexpr int M = decltype(mc)::value;
            LK ob[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) xpair<M>(kk[t], kk[t], ob[t]);
            uint32_t pa, pb;
            xpair32<M>((uint32_t)par, pa, pb);
            par = (int)(pa ^ pb);
            xpair32<M>(hd, pa, pb);
            hd = pa | pb;
            merge4(kk, ob);
        });
        if (q.valid && q.g == 0) {
            // The four positions re-sorted by index (carrying their
            // reliability rank), so penalties sum in index order.
            uint32_t idx[4], rk[4];
            S mag[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                idx[t] = (uint32_t)Lrb<T>::idx(kk[t]);
                mag[t] = Lrb<T>::mag(kk[t]);
                rk[t] = (uint32_t)t;
                si[t] = (uint16_t)idx[t];
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
            si[6] = (uint16_t)hd;
            si[7] = (uint16_t)(hd >> 16);
            const uint32_t base_d = par ? 1u : 0u;  // ML flips m1 when parity fails
            for (int r = 0; r < ccount; ++r) {
                const uint32_t dm = spc_flips(r) ^ base_d;
                S pen = 0;
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    if ((dm >> rk[t]) & 1u) pen += mag[t];
                put(r, D::sub(pms, D::round_pen(pen)));
            }
        }
    }
}

template <typename T, int TYPE>
DEV void pp_fork_score_any(const Ctx<T>& c, const OpRec& op, int k, int cc, const Grp& q) {
    const int isp = op_isp(op);
    if (isp == SP_LDS) pp_fork_score<T, TYPE, SP_LDS>(c, op, k, cc, q);
    else if (isp == SP_WS) pp_fork_score<T, TYPE, SP_WS>(c, op, k, cc, q);
    else pp_fork_score<T, TYPE, SP_CH>(c, op, k, cc, q);
}

template <typename T>
DEV void pp_rate0_any(const Ctx<T>& c, const OpRec& op, int k, int side, const Grp& q) {
    const int isp = op_isp(op), osp = op_osp(op);
    if (isp == SP_LDS) pp_rate0<T, SP_LDS, SP_LDS>(c, op, k, side, q);
    else if (isp == SP_WS) pp_rate0<T, SP_WS, SP_WS>(c, op, k, side, q);
    else if (osp == SP_LDS) pp_rate0<T, SP_CH, SP_LDS>(c, op, k, side, q);
    else pp_rate0<T, SP_CH, SP_WS>(c, op, k, side, q);
}

// Candidate selection, Alg. 1, in one wavefront: the C ranking keys (larger
// = better: metric, then smaller enumeration index) are sorted in descending
// order by a bitonic network, E keys per lane (element i = lane * E + t,
// missing elements padded with key 0, which every real key beats); the first
// L positions are the survivors, best first.
// Lanes l of a wavefront with (l & b) == 0, as a mask (b a power of two;
// b >= 64: every lane).
DEV constexpr uint64_t lanes_bit_clear(int b) {
    return b >= 64   ? ~0ull
           : b == 32 ? 0x00000000ffffffffull
           : b == 16 ? 0x0000ffff0000ffffull
           : b == 8  ? 0x00ff00ff00ff00ffull
           : b == 4  ? 0x0f0f0f0f0f0f0f0full
           : b == 2  ? 0x3333333333333333ull
                     : 0x5555555555555555ull;
}

// Sorts the keys v (element i = lane * E + t of NL * E, over lanes
// 0 .. NL - 1; NL = 32 or 64, lanes beyond NL sort their own values)
// into descending order.
template <int E, int NL, typename K>
DEV void bitonic_sort(K (&v)[E]) {
    // In a step (k, j) element i keeps the larger of its pair when
    // (i & k) == 0 and (i & j) == 0 agree.  Once k >= E that is the same
    // for the E elements of a lane, so each step's direction is a constant
    // lane mask and a compare-exchange is one 64-bit compare, a mask XOR
    // and two selects.
    constexpr int CP = NL * E;
#pragma unroll
    for (int k = 2; k <= CP; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j < E) {
                // both elements of a pair in this lane
#pragma unroll
                for (int t = 0; t < E; ++t) {
                    const int l = t ^ j;
                    if (l > t) {
                        const K a = v[t], b2 = v[l];
                        bool keep;  // v[t] keeps the larger key
                        if (k < E) {
                            const bool desc = (t & k) == 0;
                            keep = (a > b2) == desc;
                        } else {
                            const uint64_t desc = lanes_bit_clear(k / E);
                            keep = __builtin_amdgcn_inverse_ballot_w64(~(__ballot(a > b2) ^ desc));
                        }
                        v[t] = keep ? a : b2;
                        v[l] = keep ? b2 : a;
                    }
                }
            } else {
                // partner in lane ^ (j / E), same position
                const int m = j / E;
                const uint64_t want_max = ~(lanes_bit_clear(k / E) ^ lanes_bit_clear(m));
#pragma unroll
                for (int t = 0; t < E; ++t) {
                    K pa, pb;
                    xpair_dyn(v[t], m, pa, pb);
                    const bool take_a =
                        __builtin_amdgcn_inverse_ballot_w64(~(__ballot(pa > pb) ^ want_max));
                    v[t] = take_a ? pa : pb;
                }
            }
        }
    }
}

template <int E, typename K, int NL = 64>
DEV void bitonic_select(const K* ck, K* skey, int lane, int C, int L) {
    K v[E];
#pragma unroll
    for (int t = 0; t < E; ++t) {
        const int e = lane * E + t;
        v[t] = e < C ? ck[e] : K(0);
    }
    bitonic_sort<E, NL>(v);
#pragma unroll
    for (int t = 0; t < E; ++t) {
        const int pos = lane * E + t;
        if (pos < L) skey[pos] = v[t];
    }
}

// With P = L sources, the L rank-0 (ML) candidates all have keys at least
// T0 = the smallest of them, so the L-th best key is at least T0 and every
// candidate below T0 is dropped before sorting.  The candidates that remain
// are compacted (wavefront ballots) and sorted; ties cannot occur since keys
// carry the enumeration index.
template <typename T, bool WIDE>
DEV void select_rank(const Ctx<T>& c, int C, int L, int P, int lc) {
    if (c.tid >= 64) return;
    using K = typename Rank<T>::K;
    const int lane = c.lane;
    K* ck = (K*)c.ckey();
    K* sk = (K*)c.skey();
    if (C <= 64) {
        bitonic_select<1>(ck, sk, lane, C, L);
        return;
    }
    K t0 = 0;
    if (P == L) {
        K v;
        if constexpr (WIDE) {
            v = ~K(0);
            for (int s = lane; s < P; s += 64) v = ck[s << lc] < v ? ck[s << lc] : v;
        } else {
            v = lane < P ? ck[lane << lc] : ~K(0);
        }
        xor_steps(64, [&](auto mc) {
            K pa, pb;
            xpair<decltype(mc)::value>(v, pa, pb);
            v = pa < pb ? pa : pb;
        });
        t0 = v;
    }
    // compacted in place: a chunk writes only below the end of the chunk it
    // has just read, and the wavefront's LDS accesses complete in order
    K* kept = ck;
    int n = 0;
    for (int base = 0; base < C; base += 64) {
        const int e = base + lane;
        const K key = e < C ? ck[e] : K(0);
        const bool keep = e < C && key >= t0;
        const uint64_t bal = __ballot(keep);
        const int pos = n + (int)__builtin_popcountll(bal & ((1ull << lane) - 1ull));
        if (keep) kept[pos] = key;
        n += (int)__builtin_popcountll(bal);
    }
    wave_sync();
    if constexpr (WIDE) {
        // More than 256 left (L = 64 or 128 only): the best L of each chunk of
        // 256 are kept, chunk c's at [c L, c L + L), until 256 or fewer remain;
        // the overall best L are among them.  A chunk's keys are in registers
        // before any of its results are written, and those writes land below
        // the chunk's end.  One call site per network width keeps the code
        // small.
        for (;;) {
            const bool last = n <= 256;
            int m = 0;
            for (int base = 0; base < n; base += 256) {
                const int cn = last ? n : (n - base < 256 ? n - base : 256);
                const int keep = last ? L : (cn < L ? cn : L);
                K* dst = last ? sk : kept + m;
                if (cn <= 64) bitonic_select<1>(kept + base, dst, lane, cn, keep);
                else if (cn <= 128) bitonic_select<2>(kept + base, dst, lane, cn, keep);
                else bitonic_select<4>(kept + base, dst, lane, cn, keep);
                wave_sync();
                m += keep;
                if (last) break;
            }
            if (last) break;
            n = m;
        }
    } else {
        if (n <= 32) bitonic_select<1, K, 32>(kept, sk, lane, n, L);
        else if (n <= 64) bitonic_select<1>(kept, sk, lane, n, L);
        else if (n <= 128) bitonic_select<2>(kept, sk, lane, n, L);
        else bitonic_select<4>(kept, sk, lane, n, L);
    }
}

// Pass 3 of a forking leaf for one destination slot j: its metric, its path
// tables (a copy of its source's, sharing every stage buffer), and its
// codeword (the source's saved hard decisions with the candidate's flips).
template <typename T, int TYPE, int ISP, int OSP>
DEV void pp_fork_emit(Ctx<T>& c, const OpRec& op, int k, int side, int ccount, bool prune,
                      const Grp& q) {
    if (!q.valid) return;
    const int nv = 1 << k;
    const int lc = ilog2u(ccount);
    const int j = q.p;
    // the candidate taking slot j and its key (nothing dropped: candidate j,
    // whose key is intact)
    using RK = Rank<T>;
    const typename RK::K kj = prune ? ((const typename RK::K*)c.skey())[j]
                                    : ((const typename RK::K*)c.ckey())[j];
    const int e = prune ? RK::idx(kj) : j;
    const int s = e >> lc;
    const int r = e & (ccount - 1);
    const uint16_t* si = c.sinfo() + s * 8;
    const int W = words_of(k);
    const uint32_t full = nv >= 32 ? 0xffffffffu : ((1u << nv) - 1u);
    const T* in = c.template in_stage<ISP>(op.x, k, ISP == SP_CH ? 0 : c.srcA(k, s));
    uint32_t* o = c.template bw<OSP>(op.y, k, j);
    for (int w = q.g; w < W; w += q.G) {
        uint32_t word;
        if (TYPE == OP_REP || (TYPE == OP_R1 && k == 0)) {
            word = ((si[4] ^ r) & 1) ? full : 0u;
        } else {
            // hard decisions: kept by the scoring pass for nodes of at most
            // 32 values, else recomputed from the source's input
            word = nv <= 32 ? ((uint32_t)si[6] | ((uint32_t)si[7] << 16)) : hd_word<T>(in, w, nv);
            uint32_t dm;
            if constexpr (TYPE == OP_R1) dm = (uint32_t)r;
            else dm = spc_flips(r) ^ (si[4] ? 1u : 0u);
            const int nflip = (TYPE == OP_R1) ? 2 : 4;
            for (int t = 0; t < nflip; ++t) {
                const int pos = (int)si[t] - (w << 5);
                if (((dm >> t) & 1u) && pos >= 0 && pos < 32) word ^= 1u << pos;
            }
        }
        o[w] = word;
    }
    if (q.g == 0) {
        const int nxt = c.cur ^ 1;
        c.copy_row(c.rowA(nxt, j), c.rowA(c.cur, s));
        c.copy_row(c.rowB(nxt, j), c.rowB(c.cur, s));
        if (side == 0) c.rowB(nxt, j)[k] = (uint8_t)j;
        // a survivor's metric: from the selection, or (nothing dropped)
        // from its intact ranking key
        c.pm()[j] = RK::pm(kj);
    }
}

// Pass 3 of the pending fork described by op.
template <typename T, int TYPE>
DEV void pp_emit_typed(Ctx<T>& c, const OpRec& op, bool prune, const Grp& q) {
    const int k = op_k(op), side = op_side(op), cc = op_cand(op);
    const int isp = op_isp(op), osp = op_osp(op);
    if (isp == SP_LDS) pp_fork_emit<T, TYPE, SP_LDS, SP_LDS>(c, op, k, side, cc, prune, q);
    else if (isp == SP_WS) pp_fork_emit<T, TYPE, SP_WS, SP_WS>(c, op, k, side, cc, prune, q);
    else if (osp == SP_LDS) pp_fork_emit<T, TYPE, SP_CH, SP_LDS>(c, op, k, side, cc, prune, q);
    else pp_fork_emit<T, TYPE, SP_CH, SP_WS>(c, op, k, side, cc, prune, q);
}

template <typename T>
DEV void pp_emit_pending(Ctx<T>& c, const OpRec& op, bool prune, const Grp& q) {
    const int type = op_type(op);
    if (type == OP_REP) pp_emit_typed<T, OP_REP>(c, op, prune, q);
    else if (type == OP_R1) pp_emit_typed<T, OP_R1>(c, op, prune, q);
    else pp_emit_typed<T, OP_SPC>(c, op, prune, q);
    c.cur ^= 1;  // path tables now in the other buffer
}

// ---------------------------------------------------------------------------
// Forking leaves of at most 32 values (one partial-sum word), fused in one
// wavefront.  Lane s scores source path s in registers; the candidates are
// ranked in registers (repetition: each lane's two keys are already in the
// order a two-per-lane network expects) or, for Rate-1 / SPC, first
// compacted below the rank-0 threshold through the key scratch; then the
// lane holding survivor j writes slot j itself: its metric (recovered from
// the key), its path tables (its source's rows) and its codeword word.  The
// candidates, keys and survivors are those of the three-pass form, with one
// workgroup barrier instead of three and no survivor list.
// ---------------------------------------------------------------------------

template <typename T>
DEV int fork_small(Ctx<T>& c, const OpRec& op, int type, int k, int side, int cc, int P,
                   uint64_t praw) {
    using D = Dom<T>;
    using A = typename D::A;
    using S = typename D::S;
    using M = typename D::M;
    const int L = c.L;
    const int C = P * cc;
    const int lc = ilog2u(cc);
    const bool prune = C > L;
    // wavefront 0 reads every path's input, which other wavefronts may have
    // just written
    if (c.NT > 64) __syncthreads();
    if (c.tid < 64) {
        const int lane = c.lane;
        const bool act = lane < P;
        const int s = act ? lane : 0;  // idle lanes score path 0 and are ignored
        const int nv = 1 << k;
        // leaves run here only with their input and output in LDS (the
        // others take the three-pass form), so every access is an LDS one
        const T* in = c.template stage<SP_LDS>(op.x, k, c.srcA(k, s));
        const bool clamp = false;
        // op.z = 1 / 2: the previous record, the F / G forming this leaf's
        // input, did nothing, and the leaf's values are formed here from
        // that record's input stage (and, for a G, the left partial sums)
        // with the same arithmetic, never stored
        const int fz = op.z;
        const T* pin = nullptr;
        uint32_t pbits = 0;
        if (fz) {
            // the parent's stage and partial sums are in LDS as well
            const int px = (int)(uint16_t)(praw >> 16), pz = (int)(uint16_t)(praw >> 48);
            pin = c.template stage<SP_LDS>(px, k + 1, c.srcA(k + 1, s));
            if (fz == 2) pbits = *c.template bw<SP_LDS>(pz, k, c.srcB(k, s));
        }
        const M pms = c.pm()[s];
        uint64_t key[8];
        auto put = [&](int r, M v) {
            key[r] = ((uint64_t)D::order(v) << 32) | (uint32_t)(0xffff - ((s << lc) + r));
        };
#pragma unroll
        for (int r = 0; r < 8; ++r) key[r] = 0ull;
        uint16_t inf[4] = {0, 0, 0, 0};
        uint32_t bit4 = 0, hd = 0;
        // the node's values, one at a time (at most 32)
        auto scan = [&](auto fn) {
            using IO = VecIO<T>;
            if (fz) {
                // at least one chunk, at most 32 values (one partial-sum word)
                for (int ch = 0; ch < (nv >> IO::LOGV); ++ch) {
                    const int e = ch << IO::LOGV;
                    const uint4 x = *(const uint4*)(pin + e);
                    const uint4 y = *(const uint4*)(pin + nv + e);
                    const uint4 q0 = fz == 2 ? ChunkFG<T>::g(x, y, pbits >> e) : ChunkFG<T>::f(x, y);
                    A v[IO::V];
                    IO::unpack(q0, v);
#pragma unroll
                    for (int j = 0; j < IO::V; ++j) fn(e + j, v[j]);
                }
            } else if (nv >= IO::V) {
                for (int ch = 0; ch < (nv >> IO::LOGV); ++ch) {
                    const uint4 q0 = *(const uint4*)(in + (ch << IO::LOGV));
                    A v[IO::V];
                    IO::unpack(q0, v);
#pragma unroll
                    for (int j = 0; j < IO::V; ++j)
                        fn((ch << IO::LOGV) + j, clamp ? D::load(v[j]) : v[j]);
                }
            } else {
                for (int i = 0; i < nv; ++i) fn(i, D::load(in[i]));
            }
        };
        if (type == OP_REP) {
            // penalties of the all-zero and all-one words (Sec. III-E)
            S z = 0, o = 0;
            scan([&](int, A v) {
                if (v < 0) z += D::widen_abs(v);
                else o += D::widen_abs(v);
            });
            const M zr = D::round_pen(z), orr = D::round_pen(o);
            const bool one = orr < zr;  // ML word first; equal -> all-zero
            put(0, D::sub(pms, one ? orr : zr));
            put(1, D::sub(pms, one ? zr : orr));
            bit4 = one ? 1u : 0u;
        } else if (type == OP_R1 && k == 0) {
            const A v = D::load(in[0]);
            put(0, pms);
            put(1, D::sub(pms, D::round_pen(D::widen_abs(v))));
            bit4 = (v < 0) ? 1u : 0u;
        } else if (type == OP_R1) {
            // two least reliable positions, ties to the lower index
            uint64_t k1 = ~0ull, k2 = ~0ull;
            scan([&](int i, A v) {
                hd |= (v < 0 ? 1u : 0u) << i;
                const uint64_t kv = ((uint64_t)D::mag_key(v) << 32) | (uint32_t)i;
                const uint64_t lo = umin64(k1, kv);
                k2 = umin64(umax64(k1, kv), k2);
                k1 = lo;
            });
            const S a1 = D::mag_from_key((uint32_t)(k1 >> 32));
            const S a2 = D::mag_from_key((uint32_t)(k2 >> 32));
            put(0, pms);
            put(1, D::sub(pms, D::round_pen(a1)));
            put(2, D::sub(pms, D::round_pen(a2)));
            put(3, D::sub(pms, D::round_pen(a1 + a2)));
            inf[0] = (uint16_t)(k1 & 0xffff);
            inf[1] = (uint16_t)(k2 & 0xffff);
        } else {  // OP_SPC
            uint64_t kk[4] = {~0ull, ~0ull, ~0ull, ~0ull};
            int par = 0;
            scan([&](int i, A v) {
                const int b = (v < 0) ? 1 : 0;
                hd |= (uint32_t)b << i;
                par ^= b;
                insert4(kk, ((uint64_t)D::mag_key(v) << 32) | (uint32_t)i);
            });
            // the four positions re-sorted by index (carrying their
            // reliability rank), so penalties sum in index order
            uint32_t idx[4], rk[4];
            S mag[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                idx[t] = (uint32_t)(kk[t] & 0xffff);
                mag[t] = D::mag_from_key((uint32_t)(kk[t] >> 32));
                rk[t] = (uint32_t)t;
                inf[t] = (uint16_t)idx[t];
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
            bit4 = (uint32_t)par;
            const uint32_t base_d = par ? 1u : 0u;  // ML flips m1 when parity fails
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                if (r < cc) {
                    const uint32_t dm = spc_flips(r) ^ base_d;
                    S pen = 0;
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        if ((dm >> rk[t]) & 1u) pen += mag[t];
                    put(r, D::sub(pms, D::round_pen(pen)));
                }
            }
        }
        // what a survivor's writer needs from its source
        if (act) {
            uint16_t* si = c.sinfo() + s * 8;
            si[0] = inf[0];
            si[1] = inf[1];
            si[2] = inf[2];
            si[3] = inf[3];
            si[4] = (uint16_t)bit4;
            si[6] = (uint16_t)hd;
            si[7] = (uint16_t)(hd >> 16);
        }
        const uint32_t full = nv >= 32 ? 0xffffffffu : ((1u << nv) - 1u);
        const int nxt = c.cur ^ 1;
        const bool whole = type == OP_REP || (type == OP_R1 && k == 0);
        const int nflip = type == OP_R1 ? 2 : 4;
        // writes slot j from the candidate with key kv
        auto emit = [&](int j, uint64_t kv) {
            const int e = 0xffff - (int)(kv & 0xffff);
            const int src = e >> lc;
            const int r = e & (cc - 1);
            const uint16_t* sj = c.sinfo() + src * 8;
            uint32_t word;
            if (whole) {
                word = ((sj[4] ^ r) & 1) ? full : 0u;
            } else {
                word = (uint32_t)sj[6] | ((uint32_t)sj[7] << 16);
                const uint32_t dm = type == OP_R1 ? (uint32_t)r : (spc_flips(r) ^ (sj[4] ? 1u : 0u));
                for (int t = 0; t < nflip; ++t)
                    if ((dm >> t) & 1u) word ^= 1u << sj[t];
            }
            uint32_t* o = c.template bw<SP_LDS>(op.y, k, j);
            *o = word;
            c.copy_row(c.rowA(nxt, j), c.rowA(c.cur, src));
            c.copy_row(c.rowB(nxt, j), c.rowB(c.cur, src));
            if (side == 0) c.rowB(nxt, j)[k] = (uint8_t)j;
            c.pm()[j] = D::from_order((uint32_t)(kv >> 32));
        };
        wave_sync();
        if (!prune) {
            // every candidate survives, in enumeration order
            if (act)
                for (int r = 0; r < cc; ++r) {
                    uint64_t kv = key[0];
#pragma unroll
                    for (int t = 1; t < 8; ++t) kv = r == t ? key[t] : kv;
                    emit((s << lc) + r, kv);
                }
        } else if (type == OP_REP) {
            // two keys per lane, source s's at positions 2s, 2s + 1
            uint64_t v[2] = {act ? key[0] : 0ull, act ? key[1] : 0ull};
            bitonic_sort<2, 32>(v);
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int pos = lane * 2 + t;
                if (lane < 32 && pos < L) emit(pos, v[t]);
            }
        } else {
            // keys through the scratch, dropped below the rank-0 threshold
            // when every slot holds a path, compacted, sorted
            uint64_t* ck = c.ckey();
            if (act) {
#pragma unroll
                for (int r = 0; r < 8; ++r)
                    if (r < cc) ck[(s << lc) + r] = key[r];
            }
            uint64_t t0 = 0ull;
            if (P == L) {
                uint64_t v = act ? key[0] : ~0ull;
                xor_steps(64, [&](auto mc) {
                    uint64_t pa, pb;
                    xpair64<decltype(mc)::value>(v, pa, pb);
                    v = umin64(pa, pb);
                });
                t0 = v;
            }
            wave_sync();
            int n = 0;
            for (int base = 0; base < C; base += 64) {
                const int e = base + lane;
                const uint64_t kv = e < C ? ck[e] : 0ull;
                const bool keep = e < C && kv >= t0;
                const uint64_t bal = __ballot(keep);
                const int pos = n + (int)__builtin_popcountll(bal & ((1ull << lane) - 1ull));
                if (keep) ck[pos] = kv;
                n += (int)__builtin_popcountll(bal);
            }
            wave_sync();
            if (n <= 32) {
                // exactly L = 32 kept: a 32-key network
                uint64_t v[1] = {lane < n ? ck[lane] : 0ull};
                bitonic_sort<1, 32>(v);
                if (lane < L) emit(lane, v[0]);
            } else if (n <= 64) {
                uint64_t v[1] = {lane < n ? ck[lane] : 0ull};
                bitonic_sort<1, 64>(v);
                if (lane < L) emit(lane, v[0]);
            } else if (n <= 128) {
                // two keys per lane (every Rate-1 selection fits)
                uint64_t v[2];
#pragma unroll
                for (int t = 0; t < 2; ++t) v[t] = lane * 2 + t < n ? ck[lane * 2 + t] : 0ull;
                bitonic_sort<2, 64>(v);
#pragma unroll
                for (int t = 0; t < 2; ++t)
                    if (lane * 2 + t < L) emit(lane * 2 + t, v[t]);
            } else {
                // at most 8 L = 256 keys, four per lane
                uint64_t v[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) v[t] = lane * 4 + t < n ? ck[lane * 4 + t] : 0ull;
                bitonic_sort<4, 64>(v);
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    if (lane * 4 + t < L) emit(lane * 4 + t, v[t]);
            }
        }
    }
    c.cur ^= 1;  // path tables now in the other buffer (every thread)
    return prune ? L : C;
}

// A device-memory pointer read from memory (a job table, a frame record, a
// plan table) marked as global, so that its loads are global ones rather
// than generic (flat) ones, whose completion the LDS waits would also cover.
template <typename T>
DEV const T* global_row(const void* p) {
    typedef const __attribute__((address_space(1))) T* GP;
    return (const T*)(GP)(uintptr_t)p;
}

// ---------------------------------------------------------------------------
// Final choice: CRC syndromes, best passing path, u = x G_N, output.
// ---------------------------------------------------------------------------

// Syndrome contribution of one 32-bit codeword word w (nb valid bits): the
// XOR of the table rows of its set bits.
DEV uint64_t word_syndrome(uint32_t v, const uint64_t* sy, int nb) {
    uint64_t acc = 0;
#pragma unroll 8
    for (int b = 0; b < nb; ++b) acc ^= ((v >> b) & 1u) ? sy[b] : 0ull;
    return acc;
}

// Output stores: plain, or (SYS) system-scope stores that write through the
// L2, so that a persistent kernel's outputs reach memory without a cache
// write-back.
template <bool SYS, typename V>
DEV void out_store(V* p, V v) {
    if constexpr (SYS) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    else *p = v;
}

template <typename T, int RSP, bool WIDE, bool SYS = false>
DEV void finish(const Ctx<T>& c, const KArgs& a, int P, int64_t f, uint8_t* u_hat,
                uint8_t* crc_ok, void* pm_out) {
    using D = Dom<T>;
    const int n = c.n;
    const int W = words_of(n);
    const int lP = ilog2u(P);
    const int wave = c.tid >> 6;
    const int nb = c.N < 32 ? c.N : 32;
    // sinfo[0] = chosen slot, sinfo[1] = its CRC verdict; sinfo[4..7] one
    // 64-bit syndrome accumulator
    uint16_t* si = c.sinfo();
    uint64_t* syn_acc = (uint64_t*)(si + 4);
    // The answer is the best-metric path among those passing the CRC (ties
    // to the lower slot).  If the best-metric path passes, that is it;
    // only otherwise is every path's syndrome needed.
    if (c.tid < 64) {
        // one lane per path; lists above 64 give a lane two paths
        uint64_t key;
        if constexpr (WIDE) {
            auto path_key = [&](int j) {
                return ((uint64_t)D::order(c.pm()[j]) << 8) | (uint64_t)(255 - j);
            };
            key = path_key(c.lane < P ? c.lane : 0);
            if (P > 64) key = umax64(key, path_key(c.lane + 64 < P ? c.lane + 64 : 0));
        } else {
            const int j = c.lane < P ? c.lane : 0;
            key = ((uint64_t)D::order(c.pm()[j]) << 8) | (uint64_t)(255 - j);
        }
        xor_steps(P, [&](auto mc) {
            uint64_t pa, pb;
            xpair64<decltype(mc)::value>(key, pa, pb);
            key = umax64(pa, pb);
        });
        if (c.lane == 0) {
            si[0] = (uint16_t)(255 - (int)(key & 0xff));
            si[1] = 1;
            *syn_acc = 0ull;
        }
    }
    __syncthreads();
    const uint64_t* syn = global_row<uint64_t>(a.syn);
    if (a.has_crc) {
        {
            const uint32_t* x = c.template bw<RSP>(a.root_off, n, si[0]);
            uint64_t acc = 0;
            for (int w = c.tid; w < W; w += c.NT) acc ^= word_syndrome(x[w], syn + (w << 5), nb);
            xor_steps(64, [&](auto mc) {
                uint64_t pa, pb;
                xpair64<decltype(mc)::value>(acc, pa, pb);
                acc = pa ^ pb;
            });
            if (c.lane == 0 && acc) atomicXor((unsigned long long*)syn_acc, (unsigned long long)acc);
        }
        __syncthreads();
        if (*syn_acc != 0ull) {
            // every path's syndrome: one group of lanes per path
            const int G = W < 64 ? W : 64;
            const int lg = ilog2u(G);
            const int cnt = W >> lg;
            const int total = 1 << (lP + lg);
            for (int base = wave * 64; base < total; base += c.NT) {
                const int it = base + c.lane;
                const bool act = it < total;
                const int itc = act ? it : total - 1;
                const int j = itc >> lg;
                const int g = itc & (G - 1);
                const uint32_t* x = c.template bw<RSP>(a.root_off, n, j);
                uint64_t acc = 0;
                for (int t = 0; t < cnt; ++t) {
                    const int w = g + (t << lg);
                    acc ^= word_syndrome(x[w], syn + (w << 5), nb);
                }
                xor_steps(G, [&](auto mc) {
                    uint64_t pa, pb;
                    xpair64<decltype(mc)::value>(acc, pa, pb);
                    acc = pa ^ pb;
                });
                if (act && g == 0) c.surv()[j] = (acc == 0) ? 1 : 0;
            }
            __syncthreads();
            // pick: one lane per path
            if (c.tid < 64) {
                uint64_t key;
                if constexpr (WIDE) {
                    auto path_key = [&](int j) {
                        const uint64_t pass = c.surv()[j] & 1;
                        return (pass << 40) | ((uint64_t)D::order(c.pm()[j]) << 8) |
                               (uint64_t)(255 - j);
                    };
                    key = path_key(c.lane < P ? c.lane : 0);
                    if (P > 64) key = umax64(key, path_key(c.lane + 64 < P ? c.lane + 64 : 0));
                } else {
                    const int j = c.lane < P ? c.lane : 0;
                    const uint64_t pass = c.surv()[j] & 1;
                    key = (pass << 40) | ((uint64_t)D::order(c.pm()[j]) << 8) | (uint64_t)(255 - j);
                }
                xor_steps(P, [&](auto mc) {
                    uint64_t pa, pb;
                    xpair64<decltype(mc)::value>(key, pa, pb);
                    key = umax64(pa, pb);
                });
                if (c.lane == 0) {
                    si[0] = (uint16_t)(255 - (int)(key & 0xff));
                    si[1] = (uint16_t)((key >> 40) & 1);
                }
            }
            __syncthreads();
        }
    }
    if (c.tid == 0) {
        const int best = si[0];
        if (crc_ok) out_store<SYS>(crc_ok + f, (uint8_t)si[1]);
        if (pm_out) out_store<SYS>((uint32_t*)pm_out + f, (uint32_t)D::bits(c.pm()[best]));
    }
    __syncthreads();
    // u = x G_N on the chosen codeword, in place: bits within words ...
    for (int w = c.tid; w < W; w += c.NT) {
        uint32_t* x = c.template bw<RSP>(a.root_off, n, c.sinfo()[0]);
        uint32_t v = x[w];
        v ^= (v >> 1) & 0x55555555u;
        v ^= (v >> 2) & 0x33333333u;
        v ^= (v >> 4) & 0x0f0f0f0fu;
        v ^= (v >> 8) & 0x00ff00ffu;
        v ^= (v >> 16) & 0x0000ffffu;
        x[w] = v;
    }
    // ... then across words
    for (int sw = 1; sw < W; sw <<= 1) {
        __syncthreads();
        for (int w = c.tid; w < W; w += c.NT) {
            if (w & sw) continue;
            uint32_t* x = c.template bw<RSP>(a.root_off, n, c.sinfo()[0]);
            x[w] ^= x[w + sw];
        }
    }
    __syncthreads();
    {
        const uint32_t* x = c.template bw<RSP>(a.root_off, n, c.sinfo()[0]);
        const int K = a.K;
        for (int t = c.tid; t < K; t += c.NT) {
            const int p = global_row<uint16_t>(a.info_pos)[t];
            out_store<SYS>(u_hat + f * K + t, (uint8_t)((x[p >> 5] >> (p & 31)) & 1u));
        }
    }
}

// ---------------------------------------------------------------------------
// One frame through the whole schedule, by the whole workgroup.
// ---------------------------------------------------------------------------

// Points the context at a plan's LDS layout and workspace region.
template <typename T>
DEV void bind_plan(Ctx<T>& c, const KArgs& a, uint8_t* wsb) {
    c.wsb = wsb;
    c.N = a.N;
    c.n = a.n;
    c.L = a.L;
    c.ptrA_off = a.ptrA_off;
    c.ptrB_off = a.ptrB_off;
    c.pm_off = a.pm_off;
    c.spm_off = a.spm_off;
    c.rs = a.rs;
    c.ckey_off = a.ckey_off;
    c.surv_off = a.surv_off;
    c.sinfo_off = a.sinfo_off;
    c.vt2_off = a.vt2_off;
}

// The record after next for a three-level pass (float32 only).
template <typename T>
DEV uint64_t chain3_next(const uint64_t* __restrict__ sched, int oi, int cc) {
    if constexpr (std::is_same<T, float>::value)
        if (cc & 2) return sched[oi + 2];
    return 0;
}

// Schedule records are read with scalar loads (sched points into a
// read-only kernel argument), the next one while the current operation
// runs.  Outputs go to entry f of u_hat / crc_ok / pm_out.
template <typename T, bool WIDE, bool SYS = false>
DEV void decode_frame(Ctx<T>& c, const KArgs& a, const uint64_t* __restrict__ sched, int64_t f,
                      uint8_t* __restrict__ u_hat, uint8_t* __restrict__ crc_ok,
                      void* __restrict__ pm_out) {
    c.cur = 0;
    if (c.tid == 0) c.pm()[0] = 0;
    __syncthreads();
    int P = 1;
    Grp q = make_grp(c.tid, c.NT, P);
    // a fork whose survivors still have to be written (pass 3)
    int pend = 0;
    OpRec pop{};
    int pprune = 0;
    uint64_t nraw = sched[0];
    uint64_t praw = 0;  // the previous record
    for (int oi = 0; oi < a.n_ops; ++oi) {
        const uint64_t raw = nraw;
        nraw = sched[oi + 1 < a.n_ops ? oi + 1 : oi];
        OpRec op;
        op.meta = (uint16_t)raw;
        op.x = (uint16_t)(raw >> 16);
        op.y = (uint16_t)(raw >> 32);
        op.z = (uint16_t)(raw >> 48);
        const int type = op_type(op);
        const int k = op_k(op);
        const int side = op_side(op);
        const int cc = op_cand(op);
        if (pend) {
            // every survivor is written before any path's next operation
            // overwrites a stage buffer or the candidate scratch
            pp_emit_pending<T>(c, pop, pprune, q);
            pend = 0;
            __syncthreads();
        }
        switch (type) {
            case OP_F:
                if (cc & 4) pp_fg_chain_any<T, false>(c, op, nraw, chain3_next<T>(sched, oi, cc), k, q);
                else pp_fg_any<T, false>(c, op, k, q);
                break;
            case OP_G:
                if (cc & 4) pp_fg_chain_any<T, true>(c, op, nraw, chain3_next<T>(sched, oi, cc), k, q);
                else pp_fg_any<T, true>(c, op, k, q);
                break;
            case OP_COMB:
                pp_comb_any<T>(c, op, k, side, q);
                break;
            case OP_R0:
                pp_rate0_any<T>(c, op, k, side, q);
                break;
            case OP_NOP:
                break;
            default: {
                if constexpr (std::is_same<T, float>::value && !WIDE) {
                    // a short forking leaf: fused in one wavefront (measured
                    // faster for float32 only, whose workgroups span two
                    // wavefronts; its networks hold at most 32 paths)
                    if (k <= a.fuse_k && op_isp(op) == SP_LDS && op_osp(op) == SP_LDS) {
                        P = fork_small<T>(c, op, type, k, side, cc, P, praw);
                        q = make_grp(c.tid, c.NT, P);
                        __syncthreads();
                        break;
                    }
                }
                // a forking leaf: score, select across the workgroup, and
                // leave the survivors to be written by their new owners
                if (type == OP_REP) pp_fork_score_any<T, OP_REP>(c, op, k, cc, q);
                else if (type == OP_R1) pp_fork_score_any<T, OP_R1>(c, op, k, cc, q);
                else pp_fork_score_any<T, OP_SPC>(c, op, k, cc, q);
                const int C = P * cc;
                pprune = C > c.L;
                __syncthreads();
                if (pprune) {
                    select_rank<T, WIDE>(c, C, c.L, P, ilog2u(cc));
                    __syncthreads();
                }
                P = pprune ? c.L : C;
                q = make_grp(c.tid, c.NT, P);
                pend = 1;
                pop = op;
                break;
            }
        }
        praw = raw;
        wave_sync();
    }
    if (pend) pp_emit_pending<T>(c, pop, pprune, q);
    __syncthreads();
    if (a.root_sp == SP_LDS) finish<T, SP_LDS, WIDE, SYS>(c, a, P, f, u_hat, crc_ok, pm_out);
    else finish<T, SP_WS, WIDE, SYS>(c, a, P, f, u_hat, crc_ok, pm_out);
    __syncthreads();
}

// ---------------------------------------------------------------------------
// The kernels: persistent grids; each workgroup decodes one frame at a time.
// ---------------------------------------------------------------------------

// Hands out work items one at a time from a device counter (vector
// atomics): a workgroup that becomes resident only after others have
// finished simply finds fewer items left, so the launch never waits on a
// fixed share of a late workgroup.
struct WorkCounter {
    unsigned long long* counter;
    DEV int64_t next(int tid, long long& slot) const {
        if (tid == 0) slot = (long long)atomicAdd(counter, 1ull);
        __syncthreads();
        const int64_t g = slot;
        __syncthreads();
        return g;
    }
};

// Waves per SIMD the multi-code kernels are compiled for: five for int8,
// whose default launch (64 threads, 8 KiB of LDS per frame) is otherwise
// limited by registers to four resident frames per SIMD; four (up to 128
// VGPRs) for the others, which LDS limits first.  The single-code kernel
// fits five int8 waves without the bound, and is faster without it (the
// bound makes the compiler trade registers for instructions).
template <typename T>
struct WavesPerSimd {
    static constexpr int value = 4;
};
template <>
struct WavesPerSimd<int8_t> {
    static constexpr int value = 5;
};
#define PSCL_KERNEL_BOUNDS(T) \
    __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(WavesPerSimd<T>::value)))

// One code: frames taken from the counter, any workgroup any frame.
template <typename T, bool WIDE>
__global__ void __launch_bounds__(1024)
    decode_kernel(KArgs a, const uint64_t* __restrict__ sched, const T* __restrict__ llr, int64_t F,
                  uint8_t* __restrict__ u_hat, uint8_t* __restrict__ crc_ok,
                  void* __restrict__ pm_out, unsigned long long* __restrict__ counter) {
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ long long slot;
    Ctx<T> c;
    c.lds = lds;
    c.tid = threadIdx.x;
    c.NT = blockDim.x;
    c.lane = threadIdx.x & 63;
    bind_plan(c, a, a.ws + (int64_t)blockIdx.x * a.ws_frame);
    const WorkCounter wc{counter};
    for (;;) {
        const int64_t f = wc.next(c.tid, slot);
        if (f >= F) break;
        c.chan = llr + f * a.N;
        decode_frame<T, WIDE>(c, a, sched, f, u_hat, crc_ok, pm_out);
    }
}

// Several codes of one dtype in one launch.  Plan p's schedule starts at
// record op_base of the concatenated schedules; job j covers global frames
// [base, base + F) of plan `plan`, with its own input and output buffers.
struct DevPlan {
    KArgs a;
    int64_t op_base;
};
struct DevJob {
    const void* llr;
    uint8_t* u_hat;
    uint8_t* crc_ok;
    void* pm;
    int64_t F, base;
    int plan, pad;
};

// Frames are handed out one at a time from a counter (vector atomics), so
// that frames of very different cost balance across workgroups; every
// workgroup leaves once the counter has passed the last frame.
template <typename T, bool WIDE>
__global__ void PSCL_KERNEL_BOUNDS(T)
    decode_mixed_kernel(const DevPlan* __restrict__ plans, const DevJob* __restrict__ jobs,
                        int n_jobs, int64_t total, const uint64_t* __restrict__ sched,
                        uint8_t* __restrict__ ws, int64_t ws_frame,
                        unsigned long long* __restrict__ counter) {
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ long long slot;
    Ctx<T> c;
    c.lds = lds;
    c.tid = threadIdx.x;
    c.NT = blockDim.x;
    c.lane = threadIdx.x & 63;
    uint8_t* wsb = ws + (int64_t)blockIdx.x * ws_frame;
    const WorkCounter wc{counter};
    for (;;) {
        const int64_t g = wc.next(c.tid, slot);
        if (g >= total) break;
        int lo = 0, hi = n_jobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (jobs[mid].base <= g) lo = mid;
            else hi = mid - 1;
        }
        const DevJob& J = jobs[lo];
        const DevPlan& D = plans[J.plan];
        const KArgs a = D.a;
        const int64_t f = g - J.base;
        bind_plan(c, a, wsb);
        c.chan = global_row<T>(J.llr) + f * a.N;
        decode_frame<T, WIDE>(c, a, sched + D.op_base, f, J.u_hat, J.crc_ok, J.pm);
    }
}

__global__ void zero_counter(unsigned long long* counter) { *counter = 0ull; }

// ---------------------------------------------------------------------------
// Persistent serving: workgroups claim published frames of a request ring
// (ring.h) until the host stops them or no frame arrives for idle_us.
// ---------------------------------------------------------------------------

DEV uint64_t ld_sys(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
DEV uint32_t ld_sys(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Reads the host's published count, stop flag and active workgroups per CU
// into their device copies, if no other workgroup is doing so; returns the
// published count (or pub when another workgroup holds the lease).
DEV unsigned long long ring_refresh(const pscl_ring::Args& r, unsigned long long pub) {
    constexpr int AG = __HIP_MEMORY_SCOPE_AGENT;
    pscl_ring::Dev* dv = r.dev;
    if (__hip_atomic_load(&dv->lease, __ATOMIC_RELAXED, AG) != 0u ||
        __hip_atomic_exchange(&dv->lease, 1u, __ATOMIC_ACQUIRE, AG) != 0u)
        return pub;
    const uint64_t hp =
        __hip_atomic_load(&r.ctl->published, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
    if (ld_sys(&r.ctl->stop)) __hip_atomic_store(&dv->stop, 1u, __ATOMIC_RELAXED, AG);
    __hip_atomic_store(&dv->active, ld_sys(&r.ctl->active), __ATOMIC_RELAXED, AG);
    __hip_atomic_fetch_max(&dv->published, (unsigned long long)hp, __ATOMIC_RELEASE, AG);
    __hip_atomic_store(&dv->lease, 0u, __ATOMIC_RELEASE, AG);
    return hp > pub ? hp : pub;
}

// Waits until this workgroup's rank among those started on its CU is below
// the active count: 1 then, 0 when the host has raised stop or nothing new
// was published for idle_us (as ring_wait).  Waiting workgroups only read
// the device copies (the workgroups waiting for a ticket refresh them), and
// poll every ~55 us.
DEV int ring_admit(const pscl_ring::Args& r, uint32_t rank) {
    constexpr int AG = __HIP_MEMORY_SCOPE_AGENT;
    pscl_ring::Dev* dv = r.dev;
    // the workgroup of rank r on its CU takes frames while r is below the
    // host's fixed count `active`, or, with none set, while more than
    // r x CUs frames are outstanding (published, not yet finished): one or
    // two frames per CU at low load, every resident workgroup under load,
    // following the load as it is on the device
    auto wanted = [&]() {
        const uint32_t act = __hip_atomic_load(&dv->active, __ATOMIC_RELAXED, AG);
        if (act) return rank < act;
        const unsigned long long pub = __hip_atomic_load(&dv->published, __ATOMIC_RELAXED, AG);
        const unsigned long long dn = __hip_atomic_load(&dv->done, __ATOMIC_RELAXED, AG);
        return pub > dn && pub - dn > (unsigned long long)rank * r.cus;
    };
    // the first workgroup of every CU always takes frames (and, waiting for
    // tickets, refreshes the device copies, `active` among them)
    if (rank == 0 || wanted()) return 1;
    uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    const uint64_t idle = (uint64_t)r.idle_us * 100u;
    const uint32_t max_polls = r.idle_us / 16u + 64u;
    unsigned long long last = __hip_atomic_load(&dv->published, __ATOMIC_RELAXED, AG);
    for (uint32_t poll = 0;; ++poll) {
        for (int i = 0; i < 16; ++i) __builtin_amdgcn_s_sleep(127);
        if (wanted()) return 1;
        if (__hip_atomic_load(&dv->stop, __ATOMIC_RELAXED, AG)) return 0;
        const unsigned long long now = __hip_atomic_load(&dv->published, __ATOMIC_RELAXED, AG);
        if (now != last) {  // progress: the idle clock restarts
            last = now;
            t0 = __builtin_amdgcn_s_memrealtime();
            poll = 0;
        }
        if (__builtin_amdgcn_s_memrealtime() - t0 > idle || poll >= max_polls) return 0;
    }
}

// The compute unit this wave runs on, as an index below kCuSlots: the XCC
// (HW_REG_XCC_ID) and the shader engine, shader array and CU fields of
// HW_REG_HW_ID.
DEV uint32_t cu_slot() {
    const uint32_t hw = __builtin_amdgcn_s_getreg((31 << 11) | 4);    // HW_ID
    const uint32_t xcc = __builtin_amdgcn_s_getreg((31 << 11) | 20);  // XCC_ID
    const uint32_t cu = (hw >> 8) & 0xfu, sh = (hw >> 12) & 1u, se = (hw >> 13) & 7u;
    return ((xcc & 7u) << 8) | (se << 5) | (sh << 4) | cu;
}

// A ticket: the next frame left unclaimed by the previous launch, else a
// new frame number.
DEV int64_t ring_ticket(const pscl_ring::Args& r) {
    constexpr int AG = __HIP_MEMORY_SCOPE_AGENT;
    pscl_ring::Dev* dv = r.dev;
    const uint32_t prev = r.parity ^ 1u;
    const uint32_t n = __hip_atomic_load(&dv->orphan_n[prev], __ATOMIC_RELAXED, AG);
    if (__hip_atomic_load(&dv->orphan_take[prev], __ATOMIC_RELAXED, AG) < n) {
        const uint32_t k = __hip_atomic_fetch_add(&dv->orphan_take[prev], 1u, __ATOMIC_RELAXED, AG);
        if (k < n) return (int64_t)r.orphans[(uint64_t)prev * r.orphan_cap + k];
    }
    return (int64_t)__hip_atomic_fetch_add(&dv->next, 1ull, __ATOMIC_RELAXED, AG);
}

// Waits until frame t is published: 1 then, 0 when the host has raised stop
// or nothing new was published for idle_us (the real-time counter runs at
// 100 MHz; the number of polls is bounded as well).  Host memory is read
// by one idle workgroup at a time; the others poll its device copy, less
// often the further their frame is from the published count.
DEV int ring_wait(const pscl_ring::Args& r, uint64_t t) {
    constexpr int AG = __HIP_MEMORY_SCOPE_AGENT;
    pscl_ring::Dev* dv = r.dev;
    uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    const uint64_t idle = (uint64_t)r.idle_us * 100u;
    const uint32_t max_polls = r.idle_us + 64u;
    unsigned long long last = __hip_atomic_load(&dv->published, __ATOMIC_ACQUIRE, AG);
    for (uint32_t poll = 0;; ++poll) {
        unsigned long long pub = __hip_atomic_load(&dv->published, __ATOMIC_ACQUIRE, AG);
        if (pub <= t) pub = ring_refresh(r, pub);
        if (pub > t) return 1;
        if (__hip_atomic_load(&dv->stop, __ATOMIC_RELAXED, AG)) return 0;
        if (pub != last) {  // progress: the idle clock restarts
            last = pub;
            t0 = __builtin_amdgcn_s_memrealtime();
            poll = 0;
        }
        if (__builtin_amdgcn_s_memrealtime() - t0 > idle || poll >= max_polls) return 0;
        // about 3.4 us per sleep, more when the frame is far ahead
        const uint64_t ahead = t - pub;
        const int naps = ahead < 256 ? 1 : (ahead < 4096 ? 2 : 4);
        for (int i = 0; i < naps; ++i) __builtin_amdgcn_s_sleep(127);
    }
}

template <typename T, bool WIDE>
__global__ void PSCL_KERNEL_BOUNDS(T)
    serve_kernel(const DevPlan* __restrict__ plans, const uint64_t* __restrict__ sched,
                 uint8_t* __restrict__ ws, int64_t ws_frame, pscl_ring::Args r) {
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ long long slot;
    __shared__ pscl_ring::Rec d;
    Ctx<T> c;
    c.lds = lds;
    c.tid = threadIdx.x;
    c.NT = blockDim.x;
    c.lane = threadIdx.x & 63;
    uint8_t* wsb = ws + (int64_t)blockIdx.x * ws_frame;
    // this workgroup's rank among those started on its CU
    uint32_t rank = 0;
    if (c.tid == 0)
        rank = __hip_atomic_fetch_add(r.cu_rank + cu_slot(), 1u, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
        if (c.tid == 0) {
            int64_t g = -1;
            if (ring_admit(r, rank)) {
                const int64_t t = ring_ticket(r);
                g = t;
                if (!ring_wait(r, (uint64_t)t)) {
                // leaving with an unpublished frame: the next launch takes it
                const uint32_t k = __hip_atomic_fetch_add(&r.dev->orphan_n[r.parity], 1u,
                                                          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    r.orphans[(uint64_t)r.parity * r.orphan_cap + k] = (unsigned long long)t;
                    g = -1;
                }
            }
            slot = g;
        }
        __syncthreads();
        const int64_t g = slot;
        if (g < 0) break;
        // inputs may have been written since this CU last cached them
        if (c.tid == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        // the frame's record: eight words read from host memory by eight
        // lanes in one load
        static_assert(sizeof(pscl_ring::Rec) == 8 * sizeof(uint64_t), "record of eight words");
        if (c.tid < 8) {
            const uint64_t* w = (const uint64_t*)(r.rec + ((uint64_t)g & r.rec_mask));
            ((uint64_t*)&d)[c.tid] = ld_sys(w + c.tid);
        }
        __syncthreads();
        const DevPlan& D = plans[d.plan];
        const KArgs a = D.a;
        bind_plan(c, a, wsb);
        c.chan = global_row<T>(d.llr);
        // outputs written through the L2 at system scope (no write-back of
        // the whole cache per frame), complete before the count
        decode_frame<T, WIDE, true>(c, a, sched + D.op_base, 0, d.u_hat, d.crc_ok, d.pm);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (c.tid == 0) {
            __hip_atomic_fetch_add(&r.dev->done, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t s = d.slot;
            const uint32_t prev =
                __hip_atomic_fetch_add(r.count + s, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((int64_t)prev + 1 == d.F) {
                // the request's last frame: reset the slot's count, then
                // report the ticket
                __hip_atomic_store(r.count + s, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
                __hip_atomic_store(r.done + s, d.ticket, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
        __syncthreads();
    }
}

// Device memory of pscl_decode_noalloc: the frame counter in the first 256
// bytes, then the global workspaces of as many workgroups as fit.  One copy
// per device, held from the library's load until the process ends.
constexpr size_t kScratchBytes = size_t(128) << 20;
constexpr size_t kScratchHead = 256;
__device__ __align__(256) uint8_t scratch[kScratchBytes];

// ---------------------------------------------------------------------------
// Adaptive decoding (Sec. VI): after a single-path pass over every frame,
// the frames whose CRC failed are gathered and list-decoded again.
// ---------------------------------------------------------------------------

// Indices of the frames with crc_ok == 0, in no particular order.
__global__ void gather_failed(const uint8_t* __restrict__ crc_ok, int64_t F,
                              int64_t* __restrict__ idx, unsigned long long* __restrict__ count) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f < F && crc_ok[f] == 0) idx[atomicAdd(count, 1ull)] = f;
}

// The gathered frames, each written back at its own index.
template <typename T, bool WIDE>
__global__ void PSCL_KERNEL_BOUNDS(T)
    decode_gathered_kernel(KArgs a, const uint64_t* __restrict__ sched, const T* __restrict__ llr,
                           const int64_t* __restrict__ idx,
                           const unsigned long long* __restrict__ count,
                           uint8_t* __restrict__ u_hat, uint8_t* __restrict__ crc_ok,
                           void* __restrict__ pm_out, unsigned long long* __restrict__ counter) {
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ long long slot;
    Ctx<T> c;
    c.lds = lds;
    c.tid = threadIdx.x;
    c.NT = blockDim.x;
    c.lane = threadIdx.x & 63;
    bind_plan(c, a, a.ws + (int64_t)blockIdx.x * a.ws_frame);
    const int64_t n = (int64_t)*count;
    const WorkCounter wc{counter};
    for (;;) {
        const int64_t i = wc.next(c.tid, slot);
        if (i >= n) break;
        const int64_t f = idx[i];
        c.chan = llr + f * a.N;
        decode_frame<T, WIDE>(c, a, sched, f, u_hat, crc_ok, pm_out);
    }
}

__global__ void copy_count(const unsigned long long* __restrict__ count, int64_t* __restrict__ out) {
    *out = (int64_t)*count;
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
    OpRec* d_ops = nullptr;
    uint64_t* d_syn = nullptr;
    uint16_t* d_info = nullptr;
    // workspace: allocated by the first call that needs it (or by
    // pscl_plan_reserve), so that plans used only inside groups and
    // servers never hold one
    mutable uint8_t* d_ws = nullptr;
    mutable int ws_grid = 0;  // workgroups the allocated workspace serves
    mutable std::mutex ws_mu;
    unsigned long long* d_counter = nullptr;  // frames handed out
    mutable KArgs args{};
    int NT = 128, grid_max = 0, lds_bytes = 0, k_glob = 0;
    int recompute = 0;  // stages below the root recomputed at most (0..2)
    int fuse_k = -1;    // float32 fused forks up to 2^fuse_k values (-1: none)
    int chain = 0;      // F / G chained with the left child's F when it follows (0 / 1)
    std::vector<OpRec> recs;  // the operation records (a host copy of d_ops)
    const void* kernel = nullptr;
    std::vector<uint8_t> frozen;
};

struct pscl_adaptive {
    const pscl_plan* fast = nullptr;
    const pscl_plan* list = nullptr;
    int64_t max_frames = 0;
    int64_t* d_idx = nullptr;
    unsigned long long* d_count = nullptr;  // frames gathered
    unsigned long long* d_next = nullptr;   // gathered frames handed out
    uint8_t* d_ok = nullptr;  // CRC flags when the caller wants none
};

struct pscl_group {
    int device = 0, dtype = 0, NT = 64, lds_bytes = 0, grid = 0, max_jobs = 0;
    bool wide = false;  // some plan's list is above 32 paths
    int slots = 0;  // calls in flight
    int64_t ws_frame = 0;
    std::vector<const pscl_plan*> plans;
    std::vector<double> cost;  // relative work per frame, for ordering jobs
    uint64_t* d_sched = nullptr;
    DevPlan* d_plans = nullptr;
    // per call in flight: workspace, job table (device and pinned staging),
    // frame counter, completion event
    std::vector<uint8_t*> d_ws;
    std::vector<DevJob*> d_jobs, h_jobs;
    std::vector<unsigned long long*> d_counter;
    std::vector<hipEvent_t> ev;
    std::vector<char> used;
    int next_slot = 0;
    std::mutex mu;
};

template <bool W>
const void* mixed_kernel_for(int dtype) {
    return dtype == PSCL_F32   ? (const void*)&decode_mixed_kernel<float, W>
           : dtype == PSCL_I16 ? (const void*)&decode_mixed_kernel<int16_t, W>
                               : (const void*)&decode_mixed_kernel<int8_t, W>;
}

template <bool W>
void launch_mixed(const pscl_group* g, int slot, int grid, int nj, int64_t total, hipStream_t s) {
    switch (g->dtype) {
        case PSCL_F32:
            hipLaunchKernelGGL((decode_mixed_kernel<float, W>), dim3(grid), dim3(g->NT),
                               g->lds_bytes, s, g->d_plans, g->d_jobs[slot], nj, total, g->d_sched,
                               g->d_ws[slot], g->ws_frame, g->d_counter[slot]);
            break;
        case PSCL_I16:
            hipLaunchKernelGGL((decode_mixed_kernel<int16_t, W>), dim3(grid), dim3(g->NT),
                               g->lds_bytes, s, g->d_plans, g->d_jobs[slot], nj, total, g->d_sched,
                               g->d_ws[slot], g->ws_frame, g->d_counter[slot]);
            break;
        default:
            hipLaunchKernelGGL((decode_mixed_kernel<int8_t, W>), dim3(grid), dim3(g->NT),
                               g->lds_bytes, s, g->d_plans, g->d_jobs[slot], nj, total, g->d_sched,
                               g->d_ws[slot], g->ws_frame, g->d_counter[slot]);
            break;
    }
}

template <bool W>
const void* serve_kernel_for(int dtype) {
    return dtype == PSCL_F32   ? (const void*)&serve_kernel<float, W>
           : dtype == PSCL_I16 ? (const void*)&serve_kernel<int16_t, W>
                               : (const void*)&serve_kernel<int8_t, W>;
}

template <bool W>
void launch_serve(const pscl_group* g, int grid, const pscl_ring::Args& r, hipStream_t s) {
    switch (g->dtype) {
        case PSCL_F32:
            hipLaunchKernelGGL((serve_kernel<float, W>), dim3(grid), dim3(g->NT), g->lds_bytes, s,
                               g->d_plans, g->d_sched, g->d_ws[0], g->ws_frame, r);
            break;
        case PSCL_I16:
            hipLaunchKernelGGL((serve_kernel<int16_t, W>), dim3(grid), dim3(g->NT), g->lds_bytes,
                               s, g->d_plans, g->d_sched, g->d_ws[0], g->ws_frame, r);
            break;
        default:
            hipLaunchKernelGGL((serve_kernel<int8_t, W>), dim3(grid), dim3(g->NT), g->lds_bytes,
                               s, g->d_plans, g->d_sched, g->d_ws[0], g->ws_frame, r);
            break;
    }
}

template <bool W>
const void* gathered_kernel_for(int dtype) {
    return dtype == PSCL_F32   ? (const void*)&decode_gathered_kernel<float, W>
           : dtype == PSCL_I16 ? (const void*)&decode_gathered_kernel<int16_t, W>
                               : (const void*)&decode_gathered_kernel<int8_t, W>;
}

template <bool W>
void launch_gathered(const pscl_adaptive* ad, const void* llr, uint8_t* u_hat, uint8_t* ok,
                     void* pm, hipStream_t s) {
    const pscl_plan* p = ad->list;
    switch (p->dtype) {
        case PSCL_F32:
            hipLaunchKernelGGL((decode_gathered_kernel<float, W>), dim3(p->grid_max), dim3(p->NT),
                               p->lds_bytes, s, p->args, (const uint64_t*)p->d_ops,
                               (const float*)llr, ad->d_idx, ad->d_count, u_hat, ok, pm, ad->d_next);
            break;
        case PSCL_I16:
            hipLaunchKernelGGL((decode_gathered_kernel<int16_t, W>), dim3(p->grid_max),
                               dim3(p->NT), p->lds_bytes, s, p->args, (const uint64_t*)p->d_ops,
                               (const int16_t*)llr, ad->d_idx, ad->d_count, u_hat, ok, pm, ad->d_next);
            break;
        default:
            hipLaunchKernelGGL((decode_gathered_kernel<int8_t, W>), dim3(p->grid_max), dim3(p->NT),
                               p->lds_bytes, s, p->args, (const uint64_t*)p->d_ops,
                               (const int8_t*)llr, ad->d_idx, ad->d_count, u_hat, ok, pm, ad->d_next);
            break;
    }
}

namespace {

pscl_status hip_status(hipError_t e) {
    if (e == hipSuccess) return PSCL_OK;
    if (e == hipErrorOutOfMemory) return PSCL_E_NOMEM;
    return PSCL_E_HIP;
}

bool valid_L(int L) {
    return L == 1 || L == 2 || L == 4 || L == 8 || L == 16 || L == 32 || L == 64 || L == 128;
}

// Lists above 32 paths run a separate instance of each kernel (selection
// over more than 256 candidates, more than 64 paths in the final pick, no
// fused short forks), so that the code of the smaller lists is unchanged.
bool wide_list(int L) { return L > 32; }

template <bool W>
const void* kernel_for_t(int dtype) {
    switch (dtype) {
        case PSCL_F32:
            return (const void*)&decode_kernel<float, W>;
        case PSCL_I16:
            return (const void*)&decode_kernel<int16_t, W>;
        default:
            return (const void*)&decode_kernel<int8_t, W>;
    }
}
const void* kernel_for(int dtype, int L) {
    return wide_list(L) ? kernel_for_t<true>(dtype) : kernel_for_t<false>(dtype);
}

// One decode_kernel launch of plan p with kernel arguments a (a.ws: the
// workspaces of `grid` workgroups) and frame counter `counter`.
template <bool W>
void launch_decode(const pscl_plan* p, const KArgs& a, unsigned long long* counter, int grid,
                   hipStream_t s, const void* llr, int64_t F, uint8_t* u_hat, uint8_t* crc_ok,
                   void* pm) {
    switch (p->dtype) {
        case PSCL_F32:
            hipLaunchKernelGGL((decode_kernel<float, W>), dim3(grid), dim3(p->NT), p->lds_bytes, s,
                               a, (const uint64_t*)p->d_ops, (const float*)llr, F, u_hat, crc_ok,
                               pm, counter);
            break;
        case PSCL_I16:
            hipLaunchKernelGGL((decode_kernel<int16_t, W>), dim3(grid), dim3(p->NT), p->lds_bytes,
                               s, a, (const uint64_t*)p->d_ops, (const int16_t*)llr, F, u_hat,
                               crc_ok, pm, counter);
            break;
        default:
            hipLaunchKernelGGL((decode_kernel<int8_t, W>), dim3(grid), dim3(p->NT), p->lds_bytes,
                               s, a, (const uint64_t*)p->d_ops, (const int8_t*)llr, F, u_hat,
                               crc_ok, pm, counter);
            break;
    }
}

// Per-frame layout for a given first global level k_glob: LLR stages and
// partial-sum levels below k_glob live in LDS, the others in the global
// workspace; path tables, metrics and candidate scratch always in LDS.
// Offsets are recorded in 16-byte (LDS) or 256-byte (workspace) units.
// Returns the LDS bytes.
struct Layout {
    int a_off[MAXLVL];  // LLR stages
    int bl_off[MAXLVL], br_off[MAXLVL];
    int64_t ws_frame;
};

int virtual_depth(const pscl_plan* p, int k_glob);

int layout(const pscl_plan* p, int k_glob, Layout& lay, KArgs& a) {
    const int L = p->L, n = p->n, es = elem_size(p->dtype);
    const int vd = virtual_depth(p, k_glob);
    int off = 0;
    int64_t woff = 0;
    auto place = [&](int bytes, bool lds) {
        if (lds) {
            const int v = off >> 4;
            off = align16(off + bytes);
            return v;
        }
        const int v = (int)(woff >> 8);
        woff += (bytes + 255) & ~255;
        return v;
    };
    for (int k = 0; k < MAXLVL; ++k) lay.a_off[k] = lay.bl_off[k] = lay.br_off[k] = 0;
    // the levels the schedule touches: the LLR stage of level k is read or
    // written by an F / G at level k or k + 1 or a leaf at level k, the
    // partial sums of level k by a leaf or Combine at level k or a Combine
    // or G at level k + 1 (a code whose leaves all sit above level 0 has no
    // level-0 buffers)
    bool st_need[MAXLVL + 1] = {}, ps_need[MAXLVL + 1] = {};
    for (const SchedOp& s : p->sched) {
        const bool fg = s.type == OP_F || s.type == OP_G;
        if (fg) {
            st_need[s.k] = true;
            if (s.k >= 1) st_need[s.k - 1] = true;
        } else if (s.type != OP_COMB) {
            st_need[s.k] = true;
        }
        if (!fg) ps_need[s.k] = true;
        if ((s.type == OP_COMB || s.type == OP_G) && s.k >= 1) ps_need[s.k - 1] = true;
    }
    ps_need[n] = true;
    for (int k = 0; k < n; ++k)  // the stages below the root are not stored when recomputed
        lay.a_off[k] = (k >= n - vd || !st_need[k]) ? 0 : place(L * (1 << k) * es, k < k_glob);
    for (int k = 0; k <= n; ++k) {
        if (!ps_need[k]) continue;
        const int bytes = L * words_host(k) * 4;
        if (k < n) lay.bl_off[k] = place(bytes, k < k_glob);  // the root is never a left child
        lay.br_off[k] = place(bytes, k < k_glob);
    }
    // path tables: one byte per tree level 0..n, rows padded to words
    a.rs = (n + 1 + 3) & ~3;
    a.ptrA_off = off;
    off = align16(off + 2 * a.rs * L);
    a.ptrB_off = off;
    off = align16(off + 2 * a.rs * L);
    a.pm_off = off;
    off = align16(off + 4 * L);
    // candidate scratch: ranking keys of up to 8 candidates per path, the
    // survivors and their metrics, per-source statistics
    a.ckey_off = off;
    off = align16(off + 8 * 8 * L);
    a.surv_off = off;  // pass flags of the final pick
    off = align16(off + 2 * L);
    a.spm_off = off;  // survivors' keys
    off = align16(off + 8 * L);
    a.sinfo_off = off;
    off = align16(off + 16 * L);
    a.root_off = lay.br_off[n];
    a.root_sp = n < k_glob ? SP_LDS : SP_WS;
    a.vt2_off = n >= 2 ? lay.bl_off[n - 2] : 0;
    lay.ws_frame = woff;
    return off;
}

// Operation records: the schedule with every operand offset and space.
// The stages below the root can be recomputed instead of stored when they
// would live in the workspace and only F / G / Combine operations touch
// their levels: the stage of level n - 1 (depth 1: the F / G at level n - 1
// read four channel chunks per output chunk) or those of levels n - 1 and
// n - 2 as well (depth 2: the F / G at level n - 2 read eight), at most the
// plan's `recompute` levels.
int virtual_depth(const pscl_plan* p, int k_glob) {
    const int n = p->n;
    if (p->recompute <= 0) return 0;
    if (n < 3 || n - 1 < k_glob || p->sched.empty()) return 0;
    if (p->sched[0].type != OP_F || p->sched[0].k != n) return 0;  // root is split
    auto only_fgc = [&](int lvl) {
        for (const SchedOp& s : p->sched)
            if (s.k == lvl && s.type != OP_F && s.type != OP_G && s.type != OP_COMB) return false;
        return true;
    };
    // the stage must be wide enough for whole vector chunks
    const int V = 16 / elem_size(p->dtype);
    if (!only_fgc(n - 1) || (1 << (n - 2)) < V) return 0;
    if (p->recompute >= 2 && p->dtype != PSCL_I8 && n - 2 >= k_glob && only_fgc(n - 2) &&
        (1 << (n - 3)) >= V)
        return 2;
    return 1;
}

std::vector<OpRec> make_records(const pscl_plan* p, const Layout& lay, int k_glob) {
    const int n = p->n;
    auto lvl = [&](int k) { return k < k_glob ? SP_LDS : SP_WS; };
    const int vd = virtual_depth(p, k_glob);
    bool right1 = false;  // past the root's G
    bool right2 = false;  // under the right child of a level-(n - 1) node
    std::vector<OpRec> out;
    for (const SchedOp& s : p->sched) {
        OpRec r{};
        const int k = s.k;
        int isp, osp;
        const bool fg = s.type == OP_F || s.type == OP_G;
        if (vd >= 1 && k == n && fg) {
            // the root's F / G: recomputed where used
            if (s.type == OP_G) right1 = true;
            r.meta = (uint16_t)OP_NOP;
            out.push_back(r);
            continue;
        }
        if (vd == 2 && k == n - 1 && fg) {
            right2 = s.type == OP_G;
            r.meta = (uint16_t)OP_NOP;
            out.push_back(r);
            continue;
        }
        if (fg && vd >= 1 && k == n - vd) {
            isp = SP_VT;
            osp = lvl(k - 1);
            r.x = (uint16_t)lay.bl_off[n - 1];  // the root's left-half partial sums
            r.y = (uint16_t)lay.a_off[k - 1];
            r.z = (uint16_t)lay.bl_off[k - 1];
            const uint32_t cand = vd == 2 ? (8u | (right2 ? 1u : 0u)) : 0u;
            r.meta = (uint16_t)((uint32_t)s.type | ((uint32_t)k << 3) |
                                ((uint32_t)(right1 ? 1 : 0) << 7) | (cand << 8) |
                                ((uint32_t)isp << 12) | ((uint32_t)osp << 14));
            out.push_back(r);
            continue;
        }
        if (fg) {
            isp = k == n ? SP_CH : lvl(k);
            osp = lvl(k - 1);
            r.x = (uint16_t)(k < n ? lay.a_off[k] : 0);
            r.y = (uint16_t)lay.a_off[k - 1];
            r.z = (uint16_t)lay.bl_off[k - 1];
        } else if (s.type == OP_COMB) {
            isp = lvl(k - 1);
            osp = lvl(k);
            r.x = (uint16_t)lay.bl_off[k - 1];
            r.y = (uint16_t)lay.br_off[k - 1];
            r.z = (uint16_t)(s.side ? lay.br_off[k] : lay.bl_off[k]);
        } else {
            isp = k == n ? SP_CH : lvl(k);
            osp = lvl(k);
            r.x = (uint16_t)(k < n ? lay.a_off[k] : 0);
            r.y = (uint16_t)(s.side ? lay.br_off[k] : lay.bl_off[k]);
        }
        r.meta = (uint16_t)((uint32_t)s.type | ((uint32_t)k << 3) | ((uint32_t)s.side << 7) |
                            ((uint32_t)s.cand << 8) | ((uint32_t)isp << 12) | ((uint32_t)osp << 14));
        out.push_back(r);
    }
    if (p->chain > 0) {
        // an F / G whose output the next record's F reads at once: both run
        // as one chained pass (candidate bit 2 of the first; the second
        // becomes a no-op keeping its output offset and space), where the
        // child's F output is at least one vector chunk
        const int V = 16 / elem_size(p->dtype);
        auto f_type = [](const OpRec& r) { return (int)(r.meta & 7); };
        auto f_k = [](const OpRec& r) { return (int)((r.meta >> 3) & 15); };
        auto f_isp = [](const OpRec& r) { return (int)((r.meta >> 12) & 3); };
        auto f_osp = [](const OpRec& r) { return (int)((r.meta >> 14) & 3); };
        for (size_t i = 0; i + 1 < out.size(); ++i) {
            OpRec& a = out[i];
            OpRec& b = out[i + 1];
            const int ta = f_type(a), ka = f_k(a), ia = f_isp(a);
            if (ta != OP_F && ta != OP_G) continue;
            // the recomputed stage below the root chains too for float32
            // (the level n - 2 stage is then never re-read by its F; time
            // unchanged); int16 lost 2.4 % to the registers of its eight
            // channel chunks per output chunk
            if (ia != SP_LDS && ia != SP_WS && !(ia == SP_VT && p->dtype == PSCL_F32)) continue;
            if (((a.meta >> 8) & 15) != 0) continue;
            if (f_type(b) != OP_F || f_k(b) != ka - 1 || f_isp(b) != f_osp(a) || b.x != a.y)
                continue;
            if (ka < 2 || (1 << (ka - 2)) < V) continue;
            // float32: a third level when the grandchild's F follows too
            // (+1 %; the integer kernels stay at two, their registers being
            // at the limit of their residency)
            if (p->dtype == PSCL_F32 && ia != SP_VT && i + 2 < out.size() && ka >= 3 &&
                (1 << (ka - 3)) >= V) {
                OpRec& c3 = out[i + 2];
                if (f_type(c3) == OP_F && f_k(c3) == ka - 2 && f_isp(c3) == f_osp(b) &&
                    c3.x == b.y) {
                    a.meta = (uint16_t)(a.meta | (6u << 8));
                    b.meta = (uint16_t)(OP_NOP | ((uint32_t)f_osp(b) << 14));
                    c3.meta = (uint16_t)(OP_NOP | ((uint32_t)f_osp(c3) << 14));
                    i += 2;
                    continue;
                }
            }
            a.meta = (uint16_t)(a.meta | (4u << 8));
            b.meta = (uint16_t)(OP_NOP | ((uint32_t)f_osp(b) << 14));
            ++i;
        }
        if (p->dtype == PSCL_F32 && p->fuse_k >= 2) {
            // a forking leaf run fused in one wavefront (float32, 4 to
            // 2^fuse_k values) right after the F / G forming its input: the
            // leaf forms its values from that F / G's input stage (z = 1
            // after an F, 2 after a G) and the F / G record becomes a no-op
            // keeping everything but its type (after the chains: F / G
            // records they hold are not taken; measured slightly faster
            // than the other order)
            for (size_t i = 1; i < out.size(); ++i) {
                OpRec& a = out[i - 1];
                OpRec& b = out[i];
                const int tb = f_type(b), kb = f_k(b), ta = f_type(a), ia = f_isp(a);
                if (tb != OP_REP && tb != OP_R1 && tb != OP_SPC) continue;
                if (kb < 2 || kb > p->fuse_k || (ta != OP_F && ta != OP_G)) continue;
                if (f_k(a) != kb + 1 || (ia != SP_LDS && ia != SP_WS)) continue;
                if (((a.meta >> 8) & 15) != 0 || a.y != b.x || f_osp(a) != f_isp(b)) continue;
                // float32 leaves run fused only with everything in LDS
                if (p->dtype == PSCL_F32 &&
                    (ia != SP_LDS || f_isp(b) != SP_LDS || f_osp(b) != SP_LDS))
                    continue;
                b.z = (uint16_t)(ta == OP_F ? 1 : 2);
                a.meta = (uint16_t)((a.meta & ~7u) | OP_NOP);
            }
        }
    }
    return out;
}

}  // namespace

// Default launch shape per dtype (measured at (2048,1723) L=32, 65536
// frames): few waves per frame, since every schedule operation costs each
// wave its control overhead and more resident frames per CU hide each
// frame's dependent chain better than more waves per frame; an LDS budget
// that keeps tree levels up to 2^5 (int8, int16) or 2^6 (float32) on chip.
// PSCL_THREADS / PSCL_LDS_BUDGET / PSCL_MAX_WG_PER_CU override.
// Groups made by pscl_decode_mixed for a set of plans, kept until one of
// those plans is destroyed.
static std::mutex g_group_mu;
static std::map<std::vector<const pscl_plan*>, pscl_group*> g_groups;
extern "C" void pscl_group_destroy(pscl_group* g);
static void drop_cached_groups(const pscl_plan* p) {
    std::vector<pscl_group*> dead;
    {
        std::lock_guard<std::mutex> lk(g_group_mu);
        for (auto it = g_groups.begin(); it != g_groups.end();) {
            if (std::find(it->first.begin(), it->first.end(), p) != it->first.end()) {
                dead.push_back(it->second);
                it = g_groups.erase(it);
            } else {
                ++it;
            }
        }
    }
    for (pscl_group* g : dead) pscl_group_destroy(g);
}

// Measured defaults at (2048,1723) L = 32: recomputing the stage below the
// root pays for float32 and int16 (it saves its write and re-read), not for
// int8 (four clamped channel chunks per output chunk cost more than the
// traffic saved), and recomputing two levels costs more than it saves in
// every dtype; fusing forking leaves of up to 32 values in one wavefront
// pays for float32 (two wavefronts per frame) and not for the integer
// dtypes (one), whose kernels do not carry the fused form; chaining an F / G
// with its left child's F pays in every dtype (float32 +5 %, int16 +3 %,
// int8 +2 %).
static void default_layout(int dtype, int L, int& recompute, int& fuse_k, int& chain) {
    recompute = dtype == PSCL_I8 ? 0 : 1;
    fuse_k = (dtype == PSCL_F32 && L <= 32) ? 5 : -1;
    chain = 1;
}

static void default_launch(int dtype, int L, int& threads, int& budget, int& wg_cap) {
    threads = dtype == PSCL_F32 ? 128 : 64;
    budget = dtype == PSCL_F32 ? 24 * 1024 : (dtype == PSCL_I16 ? 12 * 1024 : 10 * 1024);
    if (L > 32) {
        // measured at (2048,1723), 32,768 frames: the path tables and
        // candidate scratch grow with L, and two wavefronts per frame pay
        // off from 64 paths on
        const bool big = L > 64;
        threads = dtype == PSCL_F32 && big ? 256 : 128;
        budget = dtype == PSCL_F32   ? (big ? 48 : 32) * 1024
                 : dtype == PSCL_I16 ? (big ? 32 : 20) * 1024
                                     : (big ? 20 : 16) * 1024;
    }
    wg_cap = 0;
    if (const char* e = getenv("PSCL_THREADS")) threads = atoi(e);
    if (const char* e = getenv("PSCL_LDS_BUDGET")) budget = atoi(e);
    if (const char* e = getenv("PSCL_MAX_WG_PER_CU")) wg_cap = atoi(e);
}

// The plan's own workspace, for at least `grid` workgroups: allocated on
// first use, enlarged (to the next power of two workgroups, at most the full
// grid) when a call needs more, so that plans used only for small calls hold
// little memory.  Calls on one plan are ordered, so the old workspace is
// idle once the device has finished the previous calls.
static pscl_status ensure_workspace(const pscl_plan* p, int grid) {
    if (p->args.ws_frame <= 0) return PSCL_OK;
    std::lock_guard<std::mutex> lk(p->ws_mu);
    if (p->d_ws && p->ws_grid >= grid) return PSCL_OK;
    int want = 1;
    while (want < grid) want <<= 1;
    want = std::min(want, p->grid_max);
    want = std::max(want, grid);
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return PSCL_E_HIP;
    if (cur != p->device && hipSetDevice(p->device) != hipSuccess) return PSCL_E_HIP;
    pscl_status st = PSCL_OK;
    if (p->d_ws) {
        st = hip_status(hipDeviceSynchronize());
        if (st == PSCL_OK) st = hip_status(hipFree(p->d_ws));
        if (st == PSCL_OK) {
            p->d_ws = nullptr;
            p->ws_grid = 0;
            p->args.ws = nullptr;
        }
    }
    uint8_t* ws = nullptr;
    if (st == PSCL_OK) st = hip_status(hipMalloc((void**)&ws, (size_t)(p->args.ws_frame * want)));
    if (cur != p->device) (void)hipSetDevice(cur);
    if (st != PSCL_OK) return st;
    p->d_ws = ws;
    p->ws_grid = want;
    p->args.ws = ws;
    return PSCL_OK;
}

// Device address of `scratch` on device dev (current), looked up once per
// device: host code never uses the symbol's name as an address.
static pscl_status scratch_base(int dev, uint8_t** out) {
    constexpr int kMaxDev = 64;
    static std::mutex mu;
    static uint8_t* base[kMaxDev] = {};
    if (dev < 0 || dev >= kMaxDev) return PSCL_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(mu);
    if (!base[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return PSCL_E_HIP;
        base[dev] = (uint8_t*)ptr;
    }
    *out = base[dev];
    return PSCL_OK;
}

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
        case PSCL_E_BUSY:
            return "busy: the server holds as many requests as it admits";
        case PSCL_E_TIMEOUT:
            return "timed out";
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
    drop_cached_groups(p);
    int cur = 0;
    if (hipGetDevice(&cur) == hipSuccess && cur != p->device) (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(p->d_ops);
    (void)hipFree(p->d_syn);
    (void)hipFree(p->d_info);
    (void)hipFree(p->d_ws);
    (void)hipFree(p->d_counter);
    if (cur != p->device) (void)hipSetDevice(cur);
    delete p;
}

pscl_status pscl_plan_create(int N, int K, const uint8_t* frozen_mask, uint64_t crc_poly,
                             int crc_len, int L, int dtype, int spc_max, int mode,
                             pscl_plan** out) {
    return pscl_plan_create_cfg(N, K, frozen_mask, crc_poly, crc_len, L, dtype, spc_max, mode,
                                nullptr, out);
}

pscl_status pscl_plan_create_cfg(int N, int K, const uint8_t* frozen_mask, uint64_t crc_poly,
                                 int crc_len, int L, int dtype, int spc_max, int mode,
                                 const pscl_launch_cfg* cfg, pscl_plan** out) {
    if (!out || !frozen_mask) return PSCL_E_INVALID;
    if (N < 2 || N > 4096 || (N & (N - 1))) return PSCL_E_INVALID;
    if (!valid_L(L) || dtype < PSCL_F32 || dtype > PSCL_I8) return PSCL_E_INVALID;
    if (mode != PSCL_MODE_TREE && mode != PSCL_MODE_SCL_LEAVES) return PSCL_E_INVALID;
    int NT = 0, budget = 0, wg_cap = 0;
    default_launch(dtype, L, NT, budget, wg_cap);
    if (cfg && cfg->threads) NT = cfg->threads;
    if (cfg && cfg->lds_budget) budget = cfg->lds_budget;
    if (cfg && cfg->max_wg_per_cu) wg_cap = cfg->max_wg_per_cu;
    if (NT != 64 && NT != 128 && NT != 256 && NT != 512 && NT != 1024) return PSCL_E_INVALID;
    if (budget < 0 || wg_cap < 0) return PSCL_E_INVALID;
    int recompute = 0, fuse_k = -1, chain = 0;
    default_layout(dtype, L, recompute, fuse_k, chain);
    if (cfg && cfg->unroll) {
        if (cfg->unroll < 1 || cfg->unroll > 2) return PSCL_E_INVALID;
        chain = cfg->unroll - 1;
    }
    if (cfg && cfg->recompute) {
        if (cfg->recompute < 1 || cfg->recompute > 3) return PSCL_E_INVALID;
        recompute = cfg->recompute - 1;
    }
    if (cfg && cfg->fuse_log2) {
        if (cfg->fuse_log2 < -1 || cfg->fuse_log2 > 5) return PSCL_E_INVALID;
        // only the float32 kernels for lists of at most 32 paths carry the
        // fused form
        fuse_k = (dtype == PSCL_F32 && L <= 32) ? cfg->fuse_log2 : -1;
    }
    if (NT < L && L > 64) return PSCL_E_UNSUPPORTED;
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
    p->frozen.assign(frozen_mask, frozen_mask + N);
    p->recompute = recompute;
    p->fuse_k = fuse_k;
    p->chain = chain;
    while ((1 << p->n) < N) p->n++;
    if (!build_schedule(N, frozen_mask, L, spc_max, mode, p->sched)) {
        delete p;
        return PSCL_E_INVALID;
    }

    // Layout: keep as many low stages in LDS as the per-workgroup budget
    // allows; larger stages go to the global workspace.  The budget trades
    // LDS per frame (stages kept on chip) against frames resident per CU.
    const int lds_hw = (int)std::min<size_t>(prop.sharedMemPerBlock, 160 * 1024);
    // A small budget keeps many frames resident per CU (their dependent
    // chains overlap); the top stages then live in the workspace.
    int lds_cap = std::max(4096, std::min(lds_hw, budget));
    Layout lay;
    KArgs a{};
    int k_glob = p->n + 1;
    int bytes = layout(p, k_glob, lay, a);
    const int sched_need = 0;
    while (bytes + sched_need > lds_cap && k_glob > 0) {
        --k_glob;
        bytes = layout(p, k_glob, lay, a);
    }
    // a budget too small even for the path tables and candidate scratch
    // (k_glob = 0, every tree level in the workspace) takes that smallest
    // layout
    if (bytes + sched_need > lds_cap) lds_cap = std::min(lds_hw, bytes + sched_need);
    if (bytes + sched_need > lds_cap) {
        delete p;
        return PSCL_E_UNSUPPORTED;
    }
    const int64_t wsf = lay.ws_frame;
    p->lds_bytes = bytes + sched_need;
    p->NT = NT;
    p->kernel = kernel_for(dtype, L);

    hipError_t e = hipFuncSetAttribute(p->kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       p->lds_bytes);
    if (e != hipSuccess) {
        delete p;
        return hip_status(e);
    }
    int occ = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, p->kernel, p->NT, p->lds_bytes);
    if (e != hipSuccess || occ < 1) occ = 1;
    if (wg_cap > 0 && occ > wg_cap) occ = wg_cap;
    p->grid_max = occ * prop.multiProcessorCount;

    std::vector<OpRec> ops = make_records(p, lay, k_glob);
    p->recs = ops;
    std::vector<uint64_t> syn(N, 0);
    if (crc_len > 0) syn = crc_codeword_table(N, frozen_mask, crc_poly, crc_len);
    std::vector<uint16_t> info;
    for (int i = 0; i < N; ++i)
        if (!frozen_mask[i]) info.push_back((uint16_t)i);

    pscl_status st = PSCL_OK;
    auto up = [&](void** dst, const void* src, size_t nbytes) {
        if (st != PSCL_OK) return;
        hipError_t err = hipMalloc(dst, std::max<size_t>(nbytes, 16));
        if (err == hipSuccess && nbytes) err = hipMemcpy(*dst, src, nbytes, hipMemcpyHostToDevice);
        st = hip_status(err);
    };
    up((void**)&p->d_ops, ops.data(), ops.size() * sizeof(OpRec));
    up((void**)&p->d_syn, syn.data(), syn.size() * 8);
    up((void**)&p->d_info, info.data(), info.size() * 2);
    if (st == PSCL_OK) st = hip_status(hipMalloc((void**)&p->d_counter, 8));
    if (st != PSCL_OK) {
        pscl_plan_destroy(p);
        return st;
    }

    a.ops = p->d_ops;
    a.syn = p->d_syn;
    a.info_pos = p->d_info;
    a.ws = nullptr;  // set when the workspace is allocated
    a.ws_frame = wsf;
    a.n_ops = (int)ops.size();
    a.N = N;
    a.n = p->n;
    a.K = K;
    a.L = L;
    p->k_glob = k_glob;
    a.has_crc = crc_len > 0 ? 1 : 0;
    a.fuse_k = fuse_k;
    p->args = a;
    *out = p;
    return PSCL_OK;
}

pscl_status pscl_plan_info(const pscl_plan* p, int* frames_per_wg, int* threads, int* workgroups,
                           int* lds_bytes, int64_t* workspace_bytes, int* first_global_stage) {
    if (!p) return PSCL_E_INVALID;
    if (frames_per_wg) *frames_per_wg = 1;
    if (threads) *threads = p->NT;
    if (workgroups) *workgroups = p->grid_max;
    if (lds_bytes) *lds_bytes = p->lds_bytes;
    if (workspace_bytes) *workspace_bytes = p->args.ws_frame * (int64_t)p->grid_max;
    if (first_global_stage) *first_global_stage = p->k_glob;
    return PSCL_OK;
}

pscl_status pscl_plan_code(const pscl_plan* p, int* N, int* K, int* crc_len, int* L,
                           int* dtype) {
    if (!p) return PSCL_E_INVALID;
    if (N) *N = p->N;
    if (K) *K = p->K;
    if (crc_len) *crc_len = p->r;
    if (L) *L = p->L;
    if (dtype) *dtype = p->dtype;
    return PSCL_OK;
}

pscl_status pscl_plan_footprint(const pscl_plan* p, int64_t* bytes_per_frame) {
    if (!p || !bytes_per_frame) return PSCL_E_INVALID;
    *bytes_per_frame = p->args.ws_frame + p->lds_bytes + (int64_t)p->N * elem_size(p->dtype) +
                       p->K + 1 + 4;
    return PSCL_OK;
}

pscl_status pscl_plan_reserve(const pscl_plan* p) {
    if (!p) return PSCL_E_INVALID;
    return ensure_workspace(p, p->grid_max);
}

pscl_status pscl_decode(const pscl_plan* p, const void* llr, int64_t F, uint8_t* u_hat,
                        uint8_t* crc_ok, void* pm, void* stream) {
    if (!p || F < 0) return PSCL_E_INVALID;
    if (F == 0) return PSCL_OK;
    if (!llr || !u_hat) return PSCL_E_INVALID;
    if (((uintptr_t)llr & 15u) != 0) return PSCL_E_INVALID;  // 16-byte vector loads
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return PSCL_E_HIP;
    const int grid = (int)std::min<int64_t>(F, p->grid_max);
    if (p->ws_grid < grid) {
        const pscl_status st = ensure_workspace(p, grid);
        if (st != PSCL_OK) return st;
    }
    hipStream_t s = (hipStream_t)stream;
    // the frame counter starts at zero (a one-thread kernel, so that the
    // call can be captured in a graph)
    hipLaunchKernelGGL(zero_counter, dim3(1), dim3(1), 0, s, p->d_counter);
    if (wide_list(p->L))
        launch_decode<true>(p, p->args, p->d_counter, grid, s, llr, F, u_hat, crc_ok, pm);
    else
        launch_decode<false>(p, p->args, p->d_counter, grid, s, llr, F, u_hat, crc_ok, pm);
    e = hipGetLastError();
    return e == hipSuccess ? PSCL_OK : PSCL_E_HIP;
}

pscl_status pscl_decode_noalloc(const pscl_plan* p, const void* llr, int64_t F, uint8_t* u_hat,
                                uint8_t* crc_ok, void* pm, void* stream) {
    if (!p || F < 0) return PSCL_E_INVALID;
    if (F == 0) return PSCL_OK;
    if (!llr || !u_hat) return PSCL_E_INVALID;
    if (((uintptr_t)llr & 15u) != 0) return PSCL_E_INVALID;  // 16-byte vector loads
    // the workspace of one workgroup must fit beside the counter
    const int64_t room = (int64_t)(kScratchBytes - kScratchHead);
    if (p->args.ws_frame > room) return PSCL_E_UNSUPPORTED;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PSCL_E_HIP;
    if (dev != p->device) return PSCL_E_INVALID;
    uint8_t* base = nullptr;
    const pscl_status st = scratch_base(dev, &base);
    if (st != PSCL_OK) return st;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return PSCL_E_HIP;
    // as many workgroups as have a workspace in the scratch (the frame
    // counter hands every frame to one of them)
    int64_t grid = std::min<int64_t>(F, p->grid_max);
    if (p->args.ws_frame > 0) grid = std::min<int64_t>(grid, room / p->args.ws_frame);
    KArgs a = p->args;
    a.ws = base + kScratchHead;
    unsigned long long* counter = (unsigned long long*)base;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(zero_counter, dim3(1), dim3(1), 0, s, counter);
    if (wide_list(p->L))
        launch_decode<true>(p, a, counter, (int)grid, s, llr, F, u_hat, crc_ok, pm);
    else
        launch_decode<false>(p, a, counter, (int)grid, s, llr, F, u_hat, crc_ok, pm);
    e = hipGetLastError();
    return e == hipSuccess ? PSCL_OK : PSCL_E_HIP;
}

pscl_status pscl_decode_oneshot(int N, int K, const uint8_t* frozen_mask, uint64_t crc_poly,
                                int crc_len, int L, int dtype, const void* llr, int64_t F,
                                uint8_t* u_hat, uint8_t* crc_ok, void* stream) {
    if (!frozen_mask || N < 2 || N > 4096 || F < 0) return PSCL_E_INVALID;
    if (F == 0) return PSCL_OK;
    // The caller never sees the plan, so calls for one code may come from
    // several threads and streams at once: each code gets a cached group
    // whose calls in flight have their own workspace and frame counter.
    static std::mutex mu;
    static std::map<std::string, std::pair<pscl_plan*, pscl_group*>> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PSCL_E_NODEV;
    std::string key((const char*)frozen_mask, (size_t)N);
    key += std::to_string(N) + "/" + std::to_string(K) + "/" + std::to_string(crc_poly) + "/" +
           std::to_string(crc_len) + "/" + std::to_string(L) + "/" + std::to_string(dtype) + "/" +
           std::to_string(dev);
    pscl_group* g = nullptr;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) {
            g = it->second.second;
        } else {
            pscl_plan* p = nullptr;
            pscl_status st = pscl_plan_create(N, K, frozen_mask, crc_poly, crc_len, L, dtype, 4,
                                              PSCL_MODE_TREE, &p);
            if (st != PSCL_OK) return st;
            const pscl_plan* pp = p;
            pscl_launch_cfg cfg{p->NT, 0, 0};
            st = pscl_group_create(&pp, 1, 1, 2, &cfg, &g);
            if (st != PSCL_OK) {
                pscl_plan_destroy(p);
                return st;
            }
            cache[key] = {p, g};
        }
    }
    pscl_job job{0, llr, F, u_hat, crc_ok, nullptr};
    return pscl_group_decode(g, &job, 1, stream);
}

pscl_status pscl_autotune(int N, int K, const uint8_t* frozen_mask, uint64_t crc_poly,
                          int crc_len, int L, int dtype, int spc_max, int mode,
                          const void* llr, int64_t F, void* stream, pscl_launch_cfg* best,
                          float* best_ms) {
    if (!best || !llr || F < 1) return PSCL_E_INVALID;
    hipStream_t s = (hipStream_t)stream;
    uint8_t* u = nullptr;
    uint8_t* ok = nullptr;
    void* pm = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    pscl_status st = hip_status(hipMalloc((void**)&u, (size_t)F * (size_t)std::max(K, 1)));
    if (st == PSCL_OK) st = hip_status(hipMalloc((void**)&ok, (size_t)F));
    if (st == PSCL_OK) st = hip_status(hipMalloc(&pm, (size_t)F * 4));
    if (st == PSCL_OK) st = hip_status(hipEventCreate(&e0));
    if (st == PSCL_OK) st = hip_status(hipEventCreate(&e1));
    float best_t = -1.f;
    pscl_launch_cfg cur{};
    // plans already timed: (threads, LDS bytes, workgroups, recompute, fuse)
    std::vector<std::tuple<int, int, int, int, int, int>> seen;
    // times one shape (skipped when it builds a plan already timed);
    // remembers the fastest
    auto trial = [&](const pscl_launch_cfg& cfg) {
        if (st != PSCL_OK) return;
        pscl_plan* p = nullptr;
        const pscl_status cs = pscl_plan_create_cfg(N, K, frozen_mask, crc_poly, crc_len, L, dtype,
                                                    spc_max, mode, &cfg, &p);
        if (cs != PSCL_OK) {
            if (cs != PSCL_E_UNSUPPORTED && cs != PSCL_E_NOMEM) st = cs;
            return;
        }
        const std::tuple<int, int, int, int, int, int> key{
            p->NT, p->lds_bytes, p->grid_max, virtual_depth(p, p->k_glob), p->fuse_k, p->chain};
        if (std::find(seen.begin(), seen.end(), key) != seen.end()) {
            pscl_plan_destroy(p);
            return;
        }
        seen.push_back(key);
        st = pscl_decode(p, llr, F, u, ok, pm, stream);  // warm-up (allocates the workspace)
        if (st == PSCL_OK) st = hip_status(hipEventRecord(e0, s));
        for (int r = 0; r < 2 && st == PSCL_OK; ++r) st = pscl_decode(p, llr, F, u, ok, pm, stream);
        if (st == PSCL_OK) st = hip_status(hipEventRecord(e1, s));
        if (st == PSCL_OK) st = hip_status(hipEventSynchronize(e1));
        float ms = 0.f;
        if (st == PSCL_OK) st = hip_status(hipEventElapsedTime(&ms, e0, e1));
        pscl_plan_destroy(p);
        ms *= 0.5f;
        if (st == PSCL_OK && (best_t < 0.f || ms < best_t)) {
            best_t = ms;
            cur = cfg;
        }
    };
    // 1. waves per frame and LDS budget (which tree levels stay on chip)
    const int threads[] = {64, 128, 256};
    const int budgets[] = {8192, 10240, 12288, 16384, 20480, 24576, 32768, 49152};
    for (int t : threads)
        for (int b : budgets) trial(pscl_launch_cfg{t, b, 0, 0, 0, 0});
    // 2. stages recomputed below the root, at the best shape
    const pscl_launch_cfg shape = cur;
    for (int rc = 1; rc <= 3; ++rc) {
        pscl_launch_cfg c = shape;
        c.recompute = rc;
        trial(c);
    }
    // 3. fused short forks (float32, L <= 32)
    if (dtype == PSCL_F32 && L <= 32) {
        const pscl_launch_cfg lay = cur;
        for (int fz : {-1, 3, 4, 5}) {
            pscl_launch_cfg c = lay;
            c.fuse_log2 = fz;
            trial(c);
        }
    }
    // 4. tree levels per F / G pass
    {
        const pscl_launch_cfg lay = cur;
        for (int u : {1, 2}) {
            pscl_launch_cfg c = lay;
            c.unroll = u;
            trial(c);
        }
    }
    // 5. residency cap at the best so far (fewer frames per CU)
    {
        const pscl_launch_cfg lay = cur;
        for (int cap : {2, 4, 8}) {
            pscl_launch_cfg c = lay;
            c.max_wg_per_cu = cap;
            trial(c);
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(u);
    (void)hipFree(ok);
    (void)hipFree(pm);
    if (st == PSCL_OK && best_t < 0.f) st = PSCL_E_UNSUPPORTED;
    if (st == PSCL_OK) *best = cur;
    if (st == PSCL_OK && best_ms) *best_ms = best_t;
    return st;
}

pscl_status pscl_autotune_group(const pscl_plan* const* plans, int n_plans, const pscl_job* jobs,
                                int n_jobs, void* stream, pscl_launch_cfg* cfgs, int* threads,
                                float* best_ms) {
    if (!plans || n_plans < 1 || !jobs || n_jobs < 1 || !cfgs || !threads) return PSCL_E_INVALID;
    for (int i = 0; i < n_plans; ++i)
        if (!plans[i] || plans[i]->dtype != plans[0]->dtype) return PSCL_E_INVALID;
    for (int j = 0; j < n_jobs; ++j)
        if (jobs[j].plan < 0 || jobs[j].plan >= n_plans) return PSCL_E_INVALID;
    const int dtype = plans[0]->dtype;
    int max_L = 1;
    for (int i = 0; i < n_plans; ++i) max_L = std::max(max_L, plans[i]->L);
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    pscl_status st = hip_status(hipEventCreate(&e0));
    if (st == PSCL_OK) st = hip_status(hipEventCreate(&e1));
    float best_t = -1.f;
    pscl_launch_cfg cur{};
    // one configuration for every plan of the group: plans rebuilt from the
    // given plans' codes, a group of them, the jobs decoded once to warm up
    // and twice timed
    auto trial = [&](const pscl_launch_cfg& cfg) {
        if (st != PSCL_OK) return;
        if (cfg.threads < max_L && max_L > 64) return;  // at most 64 paths per wavefront
        std::vector<pscl_plan*> tp(n_plans, nullptr);
        pscl_status cs = PSCL_OK;
        for (int i = 0; i < n_plans && cs == PSCL_OK; ++i) {
            const pscl_plan* p = plans[i];
            cs = pscl_plan_create_cfg(p->N, p->K, p->frozen.data(), p->poly, p->r, p->L, p->dtype,
                                      p->spc_max, p->mode, &cfg, &tp[i]);
        }
        pscl_group* g = nullptr;
        if (cs == PSCL_OK) {
            pscl_launch_cfg gc{cfg.threads, 0, 0, 0, 0, 0};
            cs = pscl_group_create((const pscl_plan* const*)tp.data(), n_plans, n_jobs, 1, &gc, &g);
        }
        float ms = 0.f;
        if (cs == PSCL_OK) cs = pscl_group_decode(g, jobs, n_jobs, stream);
        if (cs == PSCL_OK) cs = hip_status(hipEventRecord(e0, s));
        for (int r = 0; r < 2 && cs == PSCL_OK; ++r) cs = pscl_group_decode(g, jobs, n_jobs, stream);
        if (cs == PSCL_OK) cs = hip_status(hipEventRecord(e1, s));
        if (cs == PSCL_OK) cs = hip_status(hipEventSynchronize(e1));
        if (cs == PSCL_OK) cs = hip_status(hipEventElapsedTime(&ms, e0, e1));
        pscl_group_destroy(g);
        for (pscl_plan* p : tp) pscl_plan_destroy(p);
        if (cs == PSCL_E_UNSUPPORTED || cs == PSCL_E_NOMEM) return;
        if (cs != PSCL_OK) {
            st = cs;
            return;
        }
        ms *= 0.5f;
        if (best_t < 0.f || ms < best_t) {
            best_t = ms;
            cur = cfg;
        }
    };
    for (int t : {64, 128, 256})
        for (int b : {8192, 10240, 12288, 16384, 24576, 32768}) trial(pscl_launch_cfg{t, b, 0, 0, 0, 0});
    const pscl_launch_cfg shape = cur;
    for (int rc = 1; rc <= 3; ++rc) {
        pscl_launch_cfg c = shape;
        c.recompute = rc;
        trial(c);
    }
    if (dtype == PSCL_F32) {
        const pscl_launch_cfg lay = cur;
        for (int fz : {-1, 4, 5}) {
            pscl_launch_cfg c = lay;
            c.fuse_log2 = fz;
            trial(c);
        }
    }
    {
        const pscl_launch_cfg lay = cur;
        for (int u : {1, 2}) {
            pscl_launch_cfg c = lay;
            c.unroll = u;
            trial(c);
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st == PSCL_OK && best_t < 0.f) st = PSCL_E_UNSUPPORTED;
    if (st != PSCL_OK) return st;
    for (int i = 0; i < n_plans; ++i) cfgs[i] = cur;
    *threads = cur.threads;
    if (best_ms) *best_ms = best_t;
    return PSCL_OK;
}

void pscl_group_destroy(pscl_group* g) {
    if (!g) return;
    int cur = 0;
    if (hipGetDevice(&cur) == hipSuccess && cur != g->device) (void)hipSetDevice(g->device);
    for (int i = 0; i < g->slots; ++i)
        if (g->ev[i]) (void)hipEventSynchronize(g->ev[i]);
    for (int i = 0; i < g->slots; ++i) {
        if (g->ev[i]) (void)hipEventDestroy(g->ev[i]);
        (void)hipFree(g->d_jobs[i]);
        (void)hipFree(g->d_counter[i]);
        (void)hipFree(g->d_ws[i]);
        if (g->h_jobs[i]) (void)hipHostFree(g->h_jobs[i]);
    }
    (void)hipFree(g->d_sched);
    (void)hipFree(g->d_plans);
    if (cur != g->device) (void)hipSetDevice(cur);
    delete g;
}

pscl_status pscl_group_create(const pscl_plan* const* plans, int n_plans, int max_jobs,
                              int max_inflight, const pscl_launch_cfg* cfg, pscl_group** out) {
    if (!out || !plans || n_plans < 1 || max_jobs < 1) return PSCL_E_INVALID;
    if (max_inflight < 1 || max_inflight > 8) return PSCL_E_INVALID;
    for (int i = 0; i < n_plans; ++i) {
        if (!plans[i]) return PSCL_E_INVALID;
        if (plans[i]->dtype != plans[0]->dtype || plans[i]->device != plans[0]->device)
            return PSCL_E_UNSUPPORTED;
    }
    const int dtype = plans[0]->dtype;
    int NT = 0, budget = 0, cap_unused = 0, max_L = 1;
    for (int i = 0; i < n_plans; ++i) max_L = std::max(max_L, plans[i]->L);
    default_launch(dtype, max_L, NT, budget, cap_unused);
    if (NT < max_L && !getenv("PSCL_THREADS")) NT = max_L;  // at most 64 paths per wavefront
    if (cfg && cfg->threads) NT = cfg->threads;
    if (NT != 64 && NT != 128 && NT != 256 && NT != 512 && NT != 1024) return PSCL_E_INVALID;
    if (NT < max_L && max_L > 64) return PSCL_E_UNSUPPORTED;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PSCL_E_NODEV;
    if (dev != plans[0]->device) return PSCL_E_INVALID;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return PSCL_E_NODEV;

    pscl_group* g = new pscl_group();
    g->device = dev;
    g->dtype = dtype;
    g->NT = NT;
    g->max_jobs = max_jobs;
    g->slots = max_inflight;
    g->d_ws.assign(max_inflight, nullptr);
    g->d_jobs.assign(max_inflight, nullptr);
    g->h_jobs.assign(max_inflight, nullptr);
    g->d_counter.assign(max_inflight, nullptr);
    g->ev.assign(max_inflight, nullptr);
    g->used.assign(max_inflight, 0);
    int64_t n_rec = 0;
    for (int i = 0; i < n_plans; ++i) {
        const pscl_plan* p = plans[i];
        g->plans.push_back(p);
        g->cost.push_back((double)p->N * p->n * p->L);
        g->lds_bytes = std::max(g->lds_bytes, p->lds_bytes);
        g->ws_frame = std::max<int64_t>(g->ws_frame, p->args.ws_frame);
        n_rec += p->args.n_ops;
    }
    g->wide = wide_list(max_L);
    const void* kern = g->wide ? mixed_kernel_for<true>(dtype) : mixed_kernel_for<false>(dtype);
    pscl_status st = hip_status(
        hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, g->lds_bytes));
    int occ = 0;
    if (st == PSCL_OK)
        st = hip_status(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, NT, g->lds_bytes));
    if (st == PSCL_OK && occ < 1) st = PSCL_E_UNSUPPORTED;
    g->grid = occ * prop.multiProcessorCount;
    // concatenated schedules and the per-plan argument table
    std::vector<DevPlan> dp(n_plans);
    if (st == PSCL_OK) st = hip_status(hipMalloc((void**)&g->d_sched, (size_t)n_rec * 8));
    int64_t base = 0;
    for (int i = 0; i < n_plans && st == PSCL_OK; ++i) {
        const pscl_plan* p = plans[i];
        if (g->wide && p->fuse_k >= 0) {
            // the kernels for lists above 32 paths run no fused forks: a
            // leaf that forms its values from its parent's stage gets its
            // F / G record back
            std::vector<OpRec> r = p->recs;
            for (size_t j = 1; j < r.size(); ++j) {
                const int t = r[j].meta & 7;
                if (r[j].z && (t == OP_REP || t == OP_R1 || t == OP_SPC)) {
                    r[j - 1].meta = (uint16_t)((r[j - 1].meta & ~7u) | (r[j].z == 1 ? OP_F : OP_G));
                    r[j].z = 0;
                }
            }
            st = hip_status(hipMemcpy(g->d_sched + base, r.data(), (size_t)p->args.n_ops * 8,
                                      hipMemcpyHostToDevice));
        } else {
            st = hip_status(hipMemcpy(g->d_sched + base, p->d_ops, (size_t)p->args.n_ops * 8,
                                      hipMemcpyDeviceToDevice));
        }
        dp[i].a = p->args;
        dp[i].a.ws = nullptr;
        dp[i].op_base = base;
        base += p->args.n_ops;
    }
    if (st == PSCL_OK) st = hip_status(hipMalloc((void**)&g->d_plans, sizeof(DevPlan) * n_plans));
    if (st == PSCL_OK)
        st = hip_status(hipMemcpy(g->d_plans, dp.data(), sizeof(DevPlan) * n_plans,
                                  hipMemcpyHostToDevice));
    for (int i = 0; i < max_inflight && st == PSCL_OK; ++i) {
        if (g->ws_frame > 0)
            st = hip_status(hipMalloc((void**)&g->d_ws[i], (size_t)(g->ws_frame * g->grid)));
        if (st != PSCL_OK) break;
        st = hip_status(hipMalloc((void**)&g->d_jobs[i], sizeof(DevJob) * max_jobs));
        if (st == PSCL_OK)
            st = hip_status(hipHostMalloc((void**)&g->h_jobs[i], sizeof(DevJob) * max_jobs));
        if (st == PSCL_OK) st = hip_status(hipMalloc((void**)&g->d_counter[i], 8));
        if (st == PSCL_OK) st = hip_status(hipEventCreateWithFlags(&g->ev[i], hipEventDisableTiming));
    }
    if (st != PSCL_OK) {
        pscl_group_destroy(g);
        return st;
    }
    *out = g;
    return PSCL_OK;
}

pscl_status pscl_group_decode(pscl_group* g, const pscl_job* jobs, int n_jobs, void* stream) {
    if (!g || n_jobs < 0 || (n_jobs > 0 && !jobs)) return PSCL_E_INVALID;
    std::vector<int> idx;
    int64_t total = 0;
    for (int j = 0; j < n_jobs; ++j) {
        const pscl_job& J = jobs[j];
        if (J.plan < 0 || J.plan >= (int)g->plans.size() || J.F < 0) return PSCL_E_INVALID;
        if (J.F == 0) continue;
        if (!J.llr || !J.u_hat || ((uintptr_t)J.llr & 15u) != 0) return PSCL_E_INVALID;
        idx.push_back(j);
        total += J.F;
    }
    if (idx.empty()) return PSCL_OK;
    if ((int)idx.size() > g->max_jobs) return PSCL_E_INVALID;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return PSCL_E_HIP;
    // most expensive frames first, so that the cheap ones fill the tail
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) {
        return g->cost[jobs[x].plan] > g->cost[jobs[y].plan];
    });
    std::lock_guard<std::mutex> lk(g->mu);
    const int slot = g->next_slot;
    g->next_slot = (slot + 1) % g->slots;
    // the slot's previous launch must be done with its job table
    if (g->used[slot] && hipEventSynchronize(g->ev[slot]) != hipSuccess) return PSCL_E_HIP;
    DevJob* h = g->h_jobs[slot];
    int64_t base = 0;
    for (size_t i = 0; i < idx.size(); ++i) {
        const pscl_job& J = jobs[idx[i]];
        h[i].llr = J.llr;
        h[i].u_hat = J.u_hat;
        h[i].crc_ok = J.crc_ok;
        h[i].pm = J.pm;
        h[i].F = J.F;
        h[i].base = base;
        h[i].plan = J.plan;
        h[i].pad = 0;
        base += J.F;
    }
    hipStream_t s = (hipStream_t)stream;
    e = hipMemcpyAsync(g->d_jobs[slot], h, sizeof(DevJob) * idx.size(), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_status(e);
    hipLaunchKernelGGL(zero_counter, dim3(1), dim3(1), 0, s, g->d_counter[slot]);
    const int grid = (int)std::min<int64_t>(total, g->grid);
    const int nj = (int)idx.size();
    if (g->wide) launch_mixed<true>(g, slot, grid, nj, total, s);
    else launch_mixed<false>(g, slot, grid, nj, total, s);
    e = hipGetLastError();
    if (e != hipSuccess) return PSCL_E_HIP;
    e = hipEventRecord(g->ev[slot], s);
    if (e != hipSuccess) return PSCL_E_HIP;
    g->used[slot] = 1;
    return PSCL_OK;
}

}  // extern "C"

// The persistent serving kernel of a group's plans (ring.h): as many
// workgroups as the kernel can keep resident, at most the group's grid (the
// group's first workspace has that many slots).
pscl_status pscl_ring::launch(pscl_group* g, const pscl_ring::Args& r, hipStream_t s) {
    if (!g || !r.ctl || !r.rec || !r.done || !r.count || !r.dev || !r.orphans || !r.cu_rank)
        return PSCL_E_INVALID;
    const void* kern = g->wide ? serve_kernel_for<true>(g->dtype) : serve_kernel_for<false>(g->dtype);
    pscl_status st = hip_status(
        hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, g->lds_bytes));
    int occ = 0, cus = 0;
    if (st == PSCL_OK)
        st = hip_status(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, g->NT, g->lds_bytes));
    if (st == PSCL_OK)
        st = hip_status(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g->device));
    if (st != PSCL_OK) return st;
    if (occ < 1) return PSCL_E_UNSUPPORTED;
    if (r.wg_per_cu > 0) occ = std::min(occ, (int)r.wg_per_cu);
    const int grid = std::min<int>(std::min(g->grid, occ * cus), (int)r.orphan_cap);
    pscl_ring::Args ra = r;
    ra.cus = (uint32_t)cus;
    // this launch's orphan list and the previous one's take count start at 0
    pscl_ring::Dev* dv = r.dev;
    if (hipMemsetAsync(&dv->orphan_n[r.parity], 0, 4, s) != hipSuccess ||
        hipMemsetAsync(&dv->orphan_take[r.parity ^ 1u], 0, 4, s) != hipSuccess ||
        hipMemsetAsync(r.cu_rank, 0, sizeof(uint32_t) * pscl_ring::kCuSlots, s) != hipSuccess)
        return PSCL_E_HIP;
    if (g->wide) launch_serve<true>(g, grid, ra, s);
    else launch_serve<false>(g, grid, ra, s);
    return hip_status(hipGetLastError());
}

extern "C" {

pscl_status pscl_decode_mixed(const pscl_plan* const* plans, int n_plans, const pscl_job* jobs,
                              int n_jobs, void* stream) {
    if (!plans || n_plans < 1 || n_jobs < 0 || (n_jobs > 0 && !jobs)) return PSCL_E_INVALID;
    std::vector<const pscl_plan*> key(plans, plans + n_plans);
    for (const pscl_plan* p : key)
        if (!p) return PSCL_E_INVALID;
    pscl_group* g = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_group_mu);
        auto it = g_groups.find(key);
        if (it != g_groups.end() && it->second->max_jobs >= n_jobs) g = it->second;
    }
    if (!g) {
        pscl_status st = pscl_group_create(plans, n_plans, std::max(64, n_jobs), 4, nullptr, &g);
        if (st != PSCL_OK) return st;
        pscl_group* old = nullptr;
        {
            std::lock_guard<std::mutex> lk(g_group_mu);
            auto it = g_groups.find(key);
            if (it != g_groups.end()) old = it->second;
            g_groups[key] = g;
        }
        if (old) pscl_group_destroy(old);
    }
    return pscl_group_decode(g, jobs, n_jobs, stream);
}

void pscl_adaptive_destroy(pscl_adaptive* ad) {
    if (!ad) return;
    (void)hipDeviceSynchronize();
    (void)hipFree(ad->d_idx);
    (void)hipFree(ad->d_count);
    (void)hipFree(ad->d_next);
    (void)hipFree(ad->d_ok);
    delete ad;
}

pscl_status pscl_adaptive_create(const pscl_plan* fast, const pscl_plan* list, int64_t max_frames,
                                 pscl_adaptive** out) {
    if (!out || !fast || !list || max_frames < 1) return PSCL_E_INVALID;
    if (fast->L != 1 || fast->N != list->N || fast->K != list->K || fast->r != list->r ||
        fast->poly != list->poly || fast->dtype != list->dtype || fast->frozen != list->frozen ||
        fast->device != list->device || fast->r == 0)
        return PSCL_E_INVALID;
    const void* kern = wide_list(list->L) ? gathered_kernel_for<true>(list->dtype)
                                          : gathered_kernel_for<false>(list->dtype);
    pscl_status st = hip_status(
        hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, list->lds_bytes));
    if (st == PSCL_OK) st = ensure_workspace(fast, fast->grid_max);
    if (st == PSCL_OK) st = ensure_workspace(list, list->grid_max);
    if (st != PSCL_OK) return st;
    pscl_adaptive* ad = new pscl_adaptive();
    ad->fast = fast;
    ad->list = list;
    ad->max_frames = max_frames;
    st = hip_status(hipMalloc((void**)&ad->d_idx, sizeof(int64_t) * (size_t)max_frames));
    if (st == PSCL_OK) st = hip_status(hipMalloc((void**)&ad->d_count, 8));
    if (st == PSCL_OK) st = hip_status(hipMalloc((void**)&ad->d_next, 8));
    if (st == PSCL_OK) st = hip_status(hipMalloc((void**)&ad->d_ok, (size_t)max_frames));
    if (st != PSCL_OK) {
        pscl_adaptive_destroy(ad);
        return st;
    }
    *out = ad;
    return PSCL_OK;
}

pscl_status pscl_adaptive_decode(pscl_adaptive* ad, const void* llr, int64_t F, uint8_t* u_hat,
                                 uint8_t* crc_ok, void* pm, int64_t* n_list, void* stream) {
    if (!ad || F < 0 || F > ad->max_frames) return PSCL_E_INVALID;
    hipStream_t s = (hipStream_t)stream;
    if (F == 0) {
        if (n_list) hipLaunchKernelGGL(zero_counter, dim3(1), dim3(1), 0, s,
                                       (unsigned long long*)n_list);
        return hipGetLastError() == hipSuccess ? PSCL_OK : PSCL_E_HIP;
    }
    uint8_t* ok = crc_ok ? crc_ok : ad->d_ok;
    pscl_status st = pscl_decode(ad->fast, llr, F, u_hat, ok, pm, stream);
    if (st != PSCL_OK) return st;
    hipLaunchKernelGGL(zero_counter, dim3(1), dim3(1), 0, s, ad->d_count);
    hipLaunchKernelGGL(zero_counter, dim3(1), dim3(1), 0, s, ad->d_next);
    hipLaunchKernelGGL(gather_failed, dim3((unsigned)((F + 255) / 256)), dim3(256), 0, s, ok, F,
                       ad->d_idx, ad->d_count);
    const pscl_plan* p = ad->list;
    if (wide_list(p->L)) launch_gathered<true>(ad, llr, u_hat, ok, pm, s);
    else launch_gathered<false>(ad, llr, u_hat, ok, pm, s);
    if (n_list) hipLaunchKernelGGL(copy_count, dim3(1), dim3(1), 0, s, ad->d_count, n_list);
    return hipGetLastError() == hipSuccess ? PSCL_OK : PSCL_E_HIP;
}

}  // extern "C"
