/*
 * Test-infrastructure oracle for CRC-aided list decoding of polar codes.
 * THIS IS TEST INFRASTRUCTURE: only the tests, the smoke check and the
 * benchmark's CPU-baseline leg load it.  It shares no code with the HIP path.
 *
 * Everything here is deliberately plain: values are held in double (a float32
 * or integer LLR converts to double exactly), every arithmetic result is
 * rounded back to the domain of the LLR type right after it is formed, paths
 * are copied wholesale when they fork, and candidate metrics are computed from
 * the codeword-metric definition (eq. (pm)) rather than from the per-node
 * shortcut formulas.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no FMA contraction: a G
 * update must be exactly one rounded add).
 */
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_N 8192
#define NEAR_TIE_REL 1e-5

/* ------------------------------------------------------------------------ */
/* CRC (Sec. II-B uses a CRC as the outer code; the paper does not fix its   */
/* bit conventions: register starts at 0, MSB-first, no reflection, no       */
/* final XOR).                                                               */
/* ------------------------------------------------------------------------ */

int orc_crc(const uint8_t* bits, int nbits, uint64_t poly, int r, uint64_t* rem) {
    if (r < 1 || r > 64 || nbits < 0 || !rem || (nbits > 0 && !bits)) return -1;
    uint64_t mask = (r == 64) ? ~0ull : ((1ull << r) - 1);
    uint64_t top = 1ull << (r - 1);
    uint64_t reg = 0;
    for (int i = 0; i < nbits; i++) {
        int fb = ((reg & top) != 0) ^ (bits[i] & 1);
        reg = (reg << 1) & mask;
        if (fb) reg ^= (poly & mask);
    }
    *rem = reg;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Polar transform x = u F^{(x)n} (Sec. II-A).  Written as the two-half      */
/* recursion x = (enc(u_lo) xor enc(u_hi), enc(u_hi)), which is the         */
/* encoder form of the Combine operation, eq. (combine).                      */
/* ------------------------------------------------------------------------ */

static void transform_rec(uint8_t* v, int n) {
    if (n == 1) return;
    int h = n / 2;
    transform_rec(v, h);
    transform_rec(v + h, h);
    for (int i = 0; i < h; i++) v[i] ^= v[i + h];
}

static int is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

int orc_polar_transform(uint8_t* v, int N) {
    if (!v || !is_pow2(N) || N > ORC_MAX_N) return -1;
    transform_rec(v, N);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Candidate selection (Alg. 1): keep the L candidates with the largest      */
/* path metric; equal metrics are ordered by enumeration index (smaller      */
/* first).  The paper's heap leaves the order of the kept paths open; here,  */
/* when candidates are dropped the survivors take slots best first, and when */
/* all are kept they stay in enumeration order.                              */
/* ------------------------------------------------------------------------ */

typedef struct {
    double pm;
    int idx;
} cand_key;

static int cand_cmp(const void* a, const void* b) {
    const cand_key* x = (const cand_key*)a;
    const cand_key* y = (const cand_key*)b;
    if (x->pm > y->pm) return -1;
    if (x->pm < y->pm) return 1;
    return (x->idx < y->idx) ? -1 : (x->idx > y->idx);
}

/* Returns the number kept; *gap = metric of the L-th best minus that of the
 * (L+1)-th best when candidates were dropped, +inf otherwise. */
static int select_best(const double* pm, int n, int L, int* keep, double* gap, double* at) {
    *gap = INFINITY;
    *at = 0.0;
    if (n <= L) {
        for (int i = 0; i < n; i++) keep[i] = i;
        return n;
    }
    cand_key* k = (cand_key*)malloc(sizeof(cand_key) * (size_t)n);
    for (int i = 0; i < n; i++) {
        k[i].pm = pm[i];
        k[i].idx = i;
    }
    qsort(k, (size_t)n, sizeof(cand_key), cand_cmp);
    *gap = k[L - 1].pm - k[L].pm;
    *at = fmax(fabs(k[L - 1].pm), fabs(k[L].pm));
    for (int i = 0; i < L; i++) keep[i] = k[i].idx;
    free(k);
    return L;
}

int orc_select(const double* pm, int n, int L, int* keep) {
    if (!pm || !keep || n < 0 || L < 1) return -1;
    double gap, at;
    return select_best(pm, n, L, keep, &gap, &at);
}

/* ------------------------------------------------------------------------ */
/* Arithmetic of one LLR domain                                              */
/* ------------------------------------------------------------------------ */

typedef struct {
    int dtype;
    double Q; /* saturation bound for integer domains */
} domain;

static domain make_domain(int dtype) {
    domain d;
    d.dtype = dtype;
    d.Q = (dtype == ORC_I16) ? 32767.0 : (dtype == ORC_I8 ? 127.0 : 0.0);
    return d;
}

/* Round a freshly formed sum or difference back into the domain. */
static double dom_round(const domain* d, double x) {
    if (d->dtype == ORC_F32) return (double)(float)x;
    return x;
}

/* Saturate an LLR produced by G (integer domains only). */
static double dom_llr(const domain* d, double x) {
    if (d->dtype == ORC_F32) return (double)(float)x;
    if (x > d->Q) return d->Q;
    if (x < -d->Q) return -d->Q;
    return x;
}

/* Hard decision, eq. (sc:h): 1 iff alpha < 0 (a numeric comparison, so a
 * negative zero decides 0). */
static int h_dec(double a) { return a < 0.0; }

/* F, eq. (f), min-sum form: sgn(a) sgn(b) min(|a|, |b|). */
static double op_f(double a, double b) {
    double m = fmin(fabs(a), fabs(b));
    return ((a < 0.0) != (b < 0.0)) ? -m : m;
}

/* G, eq. (g): b - (2 beta - 1) a, i.e. b + a for beta = 0 and b - a for 1. */
static double op_g(const domain* d, double a, double b, int beta) {
    return dom_llr(d, beta ? (b - a) : (b + a));
}

/* Penalty of codeword cw against the LLRs a, eq. (pm):
 * sum_i |beta_j[i] - h(alpha_i)| |alpha_i|, summed in index order in double and
 * rounded once into the domain. */
static double cw_penalty(const domain* d, const double* a, const uint8_t* cw, int nv) {
    double s = 0.0;
    for (int i = 0; i < nv; i++)
        if ((int)cw[i] != h_dec(a[i])) s += fabs(a[i]);
    return dom_round(d, s);
}

/* A channel value.  An integer domain holds [-Q, Q] (the range G saturates
 * to), so the one input value below it (-128 for int8, -32768 for int16) is
 * saturated to -Q on input like any G result. */
static double llr_at(int dtype, const void* llr, int64_t idx) {
    if (dtype == ORC_F32) return (double)((const float*)llr)[idx];
    double v;
    if (dtype == ORC_I16) v = (double)((const int16_t*)llr)[idx];
    else v = (double)((const int8_t*)llr)[idx];
    domain d = make_domain(dtype);
    return dom_llr(&d, v);
}

/* ------------------------------------------------------------------------ */
/* Decoder A: list decoding on the decoding tree (Sec. III).                 */
/* ------------------------------------------------------------------------ */

enum { NODE_SPLIT = 0, NODE_R0, NODE_R1, NODE_REP, NODE_SPC };

typedef struct {
    int N, K, r, L, spc_max, mode;
    const uint8_t* frozen;
    domain dom;
} tree_code;

typedef struct {
    int near_tie;
} frame_log;

/* Node classes of the Fast-SSC tree restricted to the four node types used by
 * the list decoder (Sec. II-C, Sec. II-D): all frozen -> Rate-0, none frozen
 * -> Rate-1, all but the last frozen -> repetition, only the first frozen and
 * 4 <= Nv <= spc_max -> SPC; otherwise the node is split.  In the
 * size-1-leaves mode every node larger than one is split; in the Rate-0 and
 * repetition mode only those two classes replace sub-trees. */
static int classify(const tree_code* c, int off, int nv) {
    const uint8_t* f = c->frozen + off;
    int nf = 0;
    for (int i = 0; i < nv; i++) nf += f[i] ? 1 : 0;
    if (nv == 1) return nf ? NODE_R0 : NODE_R1;
    if (c->mode == ORC_MODE_SCL_LEAVES) return NODE_SPLIT;
    if (c->mode == ORC_MODE_R0_REP) {
        if (nf == nv) return NODE_R0;
        if (nf == nv - 1 && !f[nv - 1]) return NODE_REP;
        return NODE_SPLIT;
    }
    if (nf == nv) return NODE_R0;
    if (nf == 0) return NODE_R1;
    if (nf == nv - 1 && !f[nv - 1]) return NODE_REP;
    if (nf == 1 && f[0] && nv >= 4 && nv <= c->spc_max) return NODE_SPC;
    return NODE_SPLIT;
}

/* Indices of the m least reliable positions, in order: ascending |alpha|,
 * equal magnitudes to the lower index.  Plain repeated arg-min. */
static void least_reliable(const double* a, int nv, int m, int* out) {
    uint8_t taken[ORC_MAX_N];
    memset(taken, 0, (size_t)nv);
    for (int t = 0; t < m; t++) {
        int best = -1;
        for (int i = 0; i < nv; i++) {
            if (taken[i]) continue;
            if (best < 0 || fabs(a[i]) < fabs(a[best])) best = i;
        }
        out[t] = best;
        taken[best] = 1;
    }
}

/* Candidate codewords of one source path at a leaf node, in rank order (the
 * ML candidate first).  Writes up to 8 codewords of nv bytes into cw and
 * returns how many. */
static int node_candidates(const tree_code* c, int type, const double* a, int nv, uint8_t* cw) {
    int L = c->L;
    if (type == NODE_R0) {
        /* Sec. III-B: the all-zero word is the only codeword. */
        memset(cw, 0, (size_t)nv);
        return 1;
    }
    if (type == NODE_REP) {
        /* Sec. III-E: all-zero and all-one words; the ML one (larger metric,
         * equal metrics -> all-zero, eq. (rep)) is ranked first. */
        uint8_t* z = cw;
        uint8_t* o = cw + nv;
        memset(z, 0, (size_t)nv);
        memset(o, 1, (size_t)nv);
        double pz = cw_penalty(&c->dom, a, z, nv);
        double po = cw_penalty(&c->dom, a, o, nv);
        if (po < pz) {
            memset(z, 1, (size_t)nv);
            memset(o, 0, (size_t)nv);
        }
        return 2;
    }
    /* Threshold detection, eq. (info). */
    uint8_t hd[ORC_MAX_N];
    for (int i = 0; i < nv; i++) hd[i] = (uint8_t)h_dec(a[i]);
    if (type == NODE_R1) {
        if (nv == 1) {
            /* A single information bit: the decision and its complement
             * (eq. (sc-list:info)). */
            cw[0] = hd[0];
            cw[1] = (uint8_t)(1 - hd[0]);
            return 2;
        }
        /* Sec. III-C: Chase-II over the two least reliable bits. */
        int m[2];
        least_reliable(a, nv, 2, m);
        for (int k = 0; k < 4; k++) memcpy(cw + (size_t)k * nv, hd, (size_t)nv);
        cw[1 * nv + m[0]] ^= 1;
        cw[2 * nv + m[1]] ^= 1;
        cw[3 * nv + m[0]] ^= 1;
        cw[3 * nv + m[1]] ^= 1;
        return 4;
    }
    /* SPC, Sec. II-C eq. (spc) and Sec. III-D: the ML word satisfies the
     * parity by flipping the least reliable bit if needed; the other
     * candidates flip an even number of the four least reliable bits of the
     * ML word, in the order {}, {1,2}, {1,3}, {1,4}, {2,3}, {2,4}, {3,4},
     * {1,2,3,4}.  With L = 2 only the first two are generated. */
    static const int flips[8][4] = {{0, 0, 0, 0}, {1, 1, 0, 0}, {1, 0, 1, 0}, {1, 0, 0, 1},
                                     {0, 1, 1, 0}, {0, 1, 0, 1}, {0, 0, 1, 1}, {1, 1, 1, 1}};
    int m[4];
    least_reliable(a, nv, 4, m);
    int parity = 0;
    for (int i = 0; i < nv; i++) parity ^= hd[i];
    uint8_t ml[ORC_MAX_N];
    memcpy(ml, hd, (size_t)nv);
    if (parity) ml[m[0]] ^= 1;
    int ncand = (L == 2) ? 2 : 8;
    for (int k = 0; k < ncand; k++) {
        uint8_t* w = cw + (size_t)k * nv;
        memcpy(w, ml, (size_t)nv);
        for (int t = 0; t < 4; t++)
            if (flips[k][t]) w[m[t]] ^= 1;
    }
    return ncand;
}

/*
 * Decode the constituent code covering positions [off, off + nv) for P paths.
 *   alpha[P][nv], pm[P]: inputs (one row per path).
 *   beta_out[P'][nv], pm_out[P'], parent[P']: outputs; parent indexes the
 *   input rows.  Buffers sized for L rows.  Returns P'.
 * Sec. III: F, G and Combine act on every path independently; paths interact
 * only at leaf nodes, through candidate selection.
 */
static int node_decode(const tree_code* c, int off, int nv, int P, const double* alpha,
                       const double* pm, uint8_t* beta_out, double* pm_out, int* parent,
                       frame_log* log) {
    const domain* d = &c->dom;
    int L = c->L;
    int type = classify(c, off, nv);
    if (type != NODE_SPLIT) {
        int per = 8;
        uint8_t* cw = (uint8_t*)malloc((size_t)P * per * nv);
        double* cpm = (double*)malloc(sizeof(double) * (size_t)P * per);
        int* src = (int*)malloc(sizeof(int) * (size_t)P * per);
        int n = 0;
        /* Candidates enumerated by source path, then by rank. */
        for (int s = 0; s < P; s++) {
            const double* a = alpha + (size_t)s * nv;
            uint8_t* w = cw + (size_t)n * nv;
            int k = node_candidates(c, type, a, nv, w);
            for (int t = 0; t < k; t++) {
                double pen = cw_penalty(d, a, w + (size_t)t * nv, nv);
                cpm[n + t] = dom_round(d, pm[s] - pen);
                src[n + t] = s;
            }
            n += k;
        }
        int* keep = (int*)malloc(sizeof(int) * (size_t)n);
        double gap, at;
        int m = select_best(cpm, n, L, keep, &gap, &at);
        if (d->dtype == ORC_F32 && gap <= NEAR_TIE_REL * at) log->near_tie = 1;
        for (int j = 0; j < m; j++) {
            int e = keep[j];
            memcpy(beta_out + (size_t)j * nv, cw + (size_t)e * nv, (size_t)nv);
            pm_out[j] = cpm[e];
            parent[j] = src[e];
        }
        free(keep);
        free(src);
        free(cpm);
        free(cw);
        return m;
    }

    int h = nv / 2;
    double* al = (double*)malloc(sizeof(double) * (size_t)P * h);
    for (int p = 0; p < P; p++)
        for (int i = 0; i < h; i++)
            al[(size_t)p * h + i] = op_f(alpha[(size_t)p * nv + i], alpha[(size_t)p * nv + i + h]);

    uint8_t* bl = (uint8_t*)malloc((size_t)L * h);
    double* pm1 = (double*)malloc(sizeof(double) * (size_t)L);
    int* par1 = (int*)malloc(sizeof(int) * (size_t)L);
    int P1 = node_decode(c, off, h, P, al, pm, bl, pm1, par1, log);
    free(al);

    double* ar = (double*)malloc(sizeof(double) * (size_t)P1 * h);
    for (int j = 0; j < P1; j++) {
        const double* av = alpha + (size_t)par1[j] * nv;
        for (int i = 0; i < h; i++)
            ar[(size_t)j * h + i] = op_g(d, av[i], av[i + h], bl[(size_t)j * h + i]);
    }

    uint8_t* br = (uint8_t*)malloc((size_t)L * h);
    int* par2 = (int*)malloc(sizeof(int) * (size_t)L);
    int P2 = node_decode(c, off + h, h, P1, ar, pm1, br, pm_out, par2, log);
    free(ar);

    /* Combine, eq. (combine): (beta_l xor beta_r, beta_r). */
    for (int j = 0; j < P2; j++) {
        const uint8_t* l = bl + (size_t)par2[j] * h;
        const uint8_t* rr = br + (size_t)j * h;
        uint8_t* o = beta_out + (size_t)j * nv;
        for (int i = 0; i < h; i++) {
            o[i] = l[i] ^ rr[i];
            o[i + h] = rr[i];
        }
        parent[j] = par1[par2[j]];
    }
    free(par2);
    free(br);
    free(par1);
    free(pm1);
    free(bl);
    return P2;
}

static int check_code(int N, int K, const uint8_t* frozen, int r) {
    if (!is_pow2(N) || N > ORC_MAX_N || !frozen) return -1;
    int k = 0;
    for (int i = 0; i < N; i++) k += frozen[i] ? 0 : 1;
    if (k != K || K < 1) return -1;
    if (r < 0 || r > 64 || r > K) return -1;
    return 0;
}

static void info_positions(int N, const uint8_t* frozen, int* pos) {
    int k = 0;
    for (int i = 0; i < N; i++)
        if (!frozen[i]) pos[k++] = i;
}

/* Final choice (Sec. II-B): the most reliable path that satisfies the
 * CRC; when none does (or there is no CRC) the most reliable path.  Equal
 * metrics go to the lower slot.  u is recovered from the root codeword by the
 * polar transform (an involution).  Returns the chosen slot. */
static int final_pick(int N, int K, const int* pos, uint64_t poly, int r, int dtype, int P,
                      const uint8_t* cws, const double* pms, uint8_t* u_out, uint8_t* ok_out,
                      double* pm_out, frame_log* log) {
    uint8_t* u = (uint8_t*)malloc((size_t)P * N);
    uint8_t* info = (uint8_t*)malloc((size_t)K);
    int* pass = (int*)malloc(sizeof(int) * (size_t)P);
    for (int j = 0; j < P; j++) {
        memcpy(u + (size_t)j * N, cws + (size_t)j * N, (size_t)N);
        transform_rec(u + (size_t)j * N, N);
        for (int t = 0; t < K; t++) info[t] = u[(size_t)j * N + pos[t]];
        pass[j] = 1;
        if (r > 0) {
            uint64_t rem, field = 0;
            orc_crc(info, K - r, poly, r, &rem);
            for (int t = K - r; t < K; t++) field = (field << 1) | info[t];
            pass[j] = (rem == field);
        }
    }
    int any = 0;
    for (int j = 0; j < P; j++) any |= pass[j];
    int best = -1, second = -1;
    for (int j = 0; j < P; j++) {
        if (any && !pass[j]) continue;
        if (best < 0 || pms[j] > pms[best]) {
            second = best;
            best = j;
        } else if (second < 0 || pms[j] > pms[second]) {
            second = j;
        }
    }
    if (dtype == ORC_F32 && second >= 0) {
        double gap = pms[best] - pms[second];
        double at = fmax(fabs(pms[best]), fabs(pms[second]));
        if (gap <= NEAR_TIE_REL * at) log->near_tie = 1;
    }
    for (int t = 0; t < K; t++) u_out[t] = u[(size_t)best * N + pos[t]];
    if (ok_out) *ok_out = (uint8_t)(any ? 1 : 0);
    if (pm_out) *pm_out = pms[best];
    free(pass);
    free(info);
    free(u);
    return best;
}

/* Runs decoder A on one frame; returns the final list size. */
static int tree_frame(const tree_code* c, const double* ch, uint8_t* cws, double* pms,
                      frame_log* log) {
    double pm0 = 0.0;
    int* parent = (int*)malloc(sizeof(int) * (size_t)c->L);
    int P = node_decode(c, 0, c->N, 1, ch, &pm0, cws, pms, parent, log);
    free(parent);
    return P;
}

/* ---- threading over frames ---- */

typedef struct {
    int kind; /* 0 = tree, 1 = scl */
    tree_code tc;
    int N, K, r, L, dtype;
    uint64_t poly;
    const uint8_t* frozen;
    const void* llr;
    int64_t F;
    uint8_t* u_hat;
    uint8_t* crc_ok;
    double* pm;
    uint8_t* near_tie;
    int tid, nthreads;
    const int* pos;
} job;

static int scl_frame(const job* jb, const double* ch, uint8_t* u_paths, double* pms,
                     frame_log* log);

static void* worker(void* arg) {
    const job* jb = (const job*)arg;
    int N = jb->N, L = jb->L;
    double* ch = (double*)malloc(sizeof(double) * (size_t)N);
    uint8_t* cws = (uint8_t*)malloc((size_t)L * N);
    double* pms = (double*)malloc(sizeof(double) * (size_t)L);
    for (int64_t f = jb->tid; f < jb->F; f += jb->nthreads) {
        for (int i = 0; i < N; i++) ch[i] = llr_at(jb->dtype, jb->llr, f * N + i);
        frame_log log = {0};
        uint8_t ok = 0;
        double pmv = 0.0;
        if (jb->kind == 0) {
            int P = tree_frame(&jb->tc, ch, cws, pms, &log);
            final_pick(N, jb->K, jb->pos, jb->poly, jb->r, jb->dtype, P, cws, pms,
                       jb->u_hat + f * jb->K, &ok, &pmv, &log);
        } else {
            int P = scl_frame(jb, ch, cws, pms, &log);
            /* decoder B tracks u directly: pick on u rather than on the
             * codeword */
            int any = 0, best = -1, second = -1;
            uint8_t* info = (uint8_t*)malloc((size_t)jb->K);
            int* pass = (int*)malloc(sizeof(int) * (size_t)P);
            for (int j = 0; j < P; j++) {
                for (int t = 0; t < jb->K; t++) info[t] = cws[(size_t)j * N + jb->pos[t]];
                pass[j] = 1;
                if (jb->r > 0) {
                    uint64_t rem, field = 0;
                    orc_crc(info, jb->K - jb->r, jb->poly, jb->r, &rem);
                    for (int t = jb->K - jb->r; t < jb->K; t++) field = (field << 1) | info[t];
                    pass[j] = (rem == field);
                }
                any |= pass[j];
            }
            for (int j = 0; j < P; j++) {
                if (any && !pass[j]) continue;
                if (best < 0 || pms[j] > pms[best]) {
                    second = best;
                    best = j;
                } else if (second < 0 || pms[j] > pms[second]) {
                    second = j;
                }
            }
            if (jb->dtype == ORC_F32 && second >= 0) {
                double gap = pms[best] - pms[second];
                if (gap <= NEAR_TIE_REL * fmax(fabs(pms[best]), fabs(pms[second])))
                    log.near_tie = 1;
            }
            for (int t = 0; t < jb->K; t++)
                jb->u_hat[f * jb->K + t] = cws[(size_t)best * N + jb->pos[t]];
            ok = (uint8_t)(any ? 1 : 0);
            pmv = pms[best];
            free(pass);
            free(info);
        }
        if (jb->crc_ok) jb->crc_ok[f] = ok;
        if (jb->pm) jb->pm[f] = pmv;
        if (jb->near_tie) jb->near_tie[f] = (uint8_t)log.near_tie;
    }
    free(pms);
    free(cws);
    free(ch);
    return NULL;
}

static int run_jobs(job* proto, int threads) {
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    pthread_t th[256];
    job jobs[256];
    for (int t = 0; t < threads; t++) {
        jobs[t] = *proto;
        jobs[t].tid = t;
        jobs[t].nthreads = threads;
    }
    if (threads == 1) {
        worker(&jobs[0]);
        return 0;
    }
    for (int t = 0; t < threads; t++) pthread_create(&th[t], NULL, worker, &jobs[t]);
    for (int t = 0; t < threads; t++) pthread_join(th[t], NULL);
    return 0;
}

static int valid_L(int L) { return L >= 1 && L <= 4096; }

int orc_decode_tree(int N, int K, const uint8_t* frozen_mask, uint64_t poly, int r, int L,
                    int dtype, int spc_max, int mode, const void* llr, int64_t F,
                    uint8_t* u_hat, uint8_t* crc_ok, double* pm, uint8_t* near_tie,
                    int threads) {
    if (check_code(N, K, frozen_mask, r) || !valid_L(L) || F < 0 || (F > 0 && (!llr || !u_hat)))
        return -1;
    if (dtype < ORC_F32 || dtype > ORC_I8 || (mode < ORC_MODE_TREE || mode > ORC_MODE_R0_REP))
        return -1;
    int* pos = (int*)malloc(sizeof(int) * (size_t)K);
    info_positions(N, frozen_mask, pos);
    job jb;
    memset(&jb, 0, sizeof(jb));
    jb.kind = 0;
    jb.tc.N = N;
    jb.tc.K = K;
    jb.tc.r = r;
    jb.tc.L = L;
    jb.tc.spc_max = spc_max;
    jb.tc.mode = mode;
    jb.tc.frozen = frozen_mask;
    jb.tc.dom = make_domain(dtype);
    jb.N = N;
    jb.K = K;
    jb.r = r;
    jb.L = L;
    jb.dtype = dtype;
    jb.poly = poly;
    jb.frozen = frozen_mask;
    jb.llr = llr;
    jb.F = F;
    jb.u_hat = u_hat;
    jb.crc_ok = crc_ok;
    jb.pm = pm;
    jb.near_tie = near_tie;
    jb.pos = pos;
    run_jobs(&jb, threads);
    free(pos);
    return 0;
}

int orc_decode_tree_list(int N, int K, const uint8_t* frozen_mask, int L, int dtype, int spc_max,
                         int mode, const void* llr, int* n_paths, uint8_t* codewords,
                         double* pms) {
    if (check_code(N, K, frozen_mask, 0) || !valid_L(L) || !llr || !n_paths || !codewords || !pms)
        return -1;
    if (dtype < ORC_F32 || dtype > ORC_I8) return -1;
    tree_code tc;
    tc.N = N;
    tc.K = K;
    tc.r = 0;
    tc.L = L;
    tc.spc_max = spc_max;
    tc.mode = mode;
    tc.frozen = frozen_mask;
    tc.dom = make_domain(dtype);
    double* ch = (double*)malloc(sizeof(double) * (size_t)N);
    for (int i = 0; i < N; i++) ch[i] = llr_at(dtype, llr, i);
    frame_log log = {0};
    *n_paths = tree_frame(&tc, ch, codewords, pms, &log);
    free(ch);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Decoder B: bit-by-bit LLR SC-list decoding (Sec. II-B).                   */
/*                                                                           */
/* Phase i estimates u_i.  Each path keeps, for every level k = 0..n, the    */
/* LLRs a[k][0..2^k) entering the size-2^k node that contains u_i (a[n] is   */
/* the channel) and, for every level k < n, the partial sums s[k][0..2^k)    */
/* returned by the most recent left child of size 2^k.  Moving from phase    */
/* i-1 to phase i recomputes the levels below the lowest common ancestor of  */
/* the two leaves: one G at the ancestor, then F down to the leaf.  Paths    */
/* are copied wholesale on a fork.                                           */
/* ------------------------------------------------------------------------ */

typedef struct {
    double pm;
    double* a;  /* (2N-1) LLRs: level k at offset (2^k - 1) */
    uint8_t* s; /* (N-1) partial sums: level k at offset (2^k - 1), k < n */
    uint8_t* u; /* N decided bits */
} scl_path;

static int lvl_off(int k) { return (1 << k) - 1; }

static void scl_path_alloc(scl_path* p, int N) {
    p->a = (double*)malloc(sizeof(double) * (size_t)(2 * N - 1));
    p->s = (uint8_t*)malloc((size_t)(N > 1 ? N - 1 : 1));
    p->u = (uint8_t*)calloc((size_t)N, 1);
}

static void scl_path_free(scl_path* p) {
    free(p->a);
    free(p->s);
    free(p->u);
}

static void scl_path_copy(scl_path* dst, const scl_path* src, int N) {
    dst->pm = src->pm;
    memcpy(dst->a, src->a, sizeof(double) * (size_t)(2 * N - 1));
    memcpy(dst->s, src->s, (size_t)(N > 1 ? N - 1 : 1));
    memcpy(dst->u, src->u, (size_t)N);
}

static int ctz_int(int x) {
    int c = 0;
    while (!(x & 1)) {
        x >>= 1;
        c++;
    }
    return c;
}

/* Bring a[0][0] (the LLR of u_i) up to date for phase i. */
static void scl_llrs(const domain* d, scl_path* p, int n, int i) {
    int top;
    if (i == 0) {
        top = n; /* every level below the root is computed by F */
        for (int k = n; k >= 1; k--) {
            int h = 1 << (k - 1);
            double* in = p->a + lvl_off(k);
            double* out = p->a + lvl_off(k - 1);
            for (int t = 0; t < h; t++) out[t] = op_f(in[t], in[t + h]);
        }
        return;
    }
    /* leaves i-1 and i first part at level t+1, t = number of trailing zeros
     * of i: u_i is in the right child there. */
    top = ctz_int(i) + 1;
    {
        int k = top;
        int h = 1 << (k - 1);
        double* in = p->a + lvl_off(k);
        double* out = p->a + lvl_off(k - 1);
        const uint8_t* sl = p->s + lvl_off(k - 1);
        for (int t = 0; t < h; t++) out[t] = op_g(d, in[t], in[t + h], sl[t]);
    }
    for (int k = top - 1; k >= 1; k--) {
        int h = 1 << (k - 1);
        double* in = p->a + lvl_off(k);
        double* out = p->a + lvl_off(k - 1);
        for (int t = 0; t < h; t++) out[t] = op_f(in[t], in[t + h]);
    }
}

/* Record u_i = b and propagate the partial sums upward (eq. (combine)). */
static void scl_sums(scl_path* p, int n, int i, int b) {
    p->u[i] = (uint8_t)b;
    uint8_t cur[ORC_MAX_N];
    cur[0] = (uint8_t)b;
    int len = 1;
    int k = 0;
    while (k < n && ((i >> k) & 1)) {
        /* the node of size 2^k just finished is a right child: combine with
         * its left sibling's partial sums */
        const uint8_t* l = p->s + lvl_off(k);
        uint8_t nxt[ORC_MAX_N];
        for (int t = 0; t < len; t++) {
            nxt[t] = l[t] ^ cur[t];
            nxt[t + len] = cur[t];
        }
        len *= 2;
        memcpy(cur, nxt, (size_t)len);
        k++;
    }
    if (k < n) memcpy(p->s + lvl_off(k), cur, (size_t)len); /* a left child */
}

static int scl_frame(const job* jb, const double* ch, uint8_t* u_paths, double* pms,
                     frame_log* log) {
    int N = jb->N, L = jb->L;
    int n = 0;
    while ((1 << n) < N) n++;
    domain d = make_domain(jb->dtype);
    scl_path* cur = (scl_path*)malloc(sizeof(scl_path) * (size_t)L);
    scl_path* nxt = (scl_path*)malloc(sizeof(scl_path) * (size_t)L);
    for (int j = 0; j < L; j++) {
        scl_path_alloc(&cur[j], N);
        scl_path_alloc(&nxt[j], N);
    }
    int P = 1;
    cur[0].pm = 0.0;
    memcpy(cur[0].a + lvl_off(n), ch, sizeof(double) * (size_t)N);
    double* cpm = (double*)malloc(sizeof(double) * 2 * (size_t)L);
    int* keep = (int*)malloc(sizeof(int) * 2 * (size_t)L);
    for (int i = 0; i < N; i++) {
        for (int j = 0; j < P; j++) scl_llrs(&d, &cur[j], n, i);
        if (jb->frozen[i]) {
            /* frozen bit: u_i = 0, metric penalised when h(alpha) = 1,
             * eq. (sc-list:info) */
            for (int j = 0; j < P; j++) {
                double a = cur[j].a[0];
                if (h_dec(a)) cur[j].pm = dom_round(&d, cur[j].pm - fabs(a));
                scl_sums(&cur[j], n, i, 0);
            }
            continue;
        }
        /* information bit: each path forks into its decision h(alpha) and
         * the complement, penalised by |alpha| */
        for (int j = 0; j < P; j++) {
            double a = cur[j].a[0];
            cpm[2 * j] = cur[j].pm;
            cpm[2 * j + 1] = dom_round(&d, cur[j].pm - fabs(a));
        }
        double gap, at;
        int m = select_best(cpm, 2 * P, L, keep, &gap, &at);
        if (d.dtype == ORC_F32 && gap <= NEAR_TIE_REL * at) log->near_tie = 1;
        for (int t = 0; t < m; t++) {
            int e = keep[t];
            int src = e / 2;
            int b = h_dec(cur[src].a[0]) ^ (e & 1);
            scl_path_copy(&nxt[t], &cur[src], N);
            nxt[t].pm = cpm[e];
            scl_sums(&nxt[t], n, i, b);
        }
        scl_path* tmp = cur;
        cur = nxt;
        nxt = tmp;
        P = m;
    }
    for (int j = 0; j < P; j++) {
        memcpy(u_paths + (size_t)j * N, cur[j].u, (size_t)N);
        pms[j] = cur[j].pm;
    }
    free(keep);
    free(cpm);
    for (int j = 0; j < L; j++) {
        scl_path_free(&cur[j]);
        scl_path_free(&nxt[j]);
    }
    free(cur);
    free(nxt);
    return P;
}

int orc_decode_scl(int N, int K, const uint8_t* frozen_mask, uint64_t poly, int r, int L,
                   int dtype, const void* llr, int64_t F, uint8_t* u_hat, uint8_t* crc_ok,
                   double* pm, uint8_t* near_tie, int threads) {
    if (check_code(N, K, frozen_mask, r) || !valid_L(L) || F < 0 || (F > 0 && (!llr || !u_hat)))
        return -1;
    if (dtype < ORC_F32 || dtype > ORC_I8) return -1;
    int* pos = (int*)malloc(sizeof(int) * (size_t)K);
    info_positions(N, frozen_mask, pos);
    job jb;
    memset(&jb, 0, sizeof(jb));
    jb.kind = 1;
    jb.N = N;
    jb.K = K;
    jb.r = r;
    jb.L = L;
    jb.dtype = dtype;
    jb.poly = poly;
    jb.frozen = frozen_mask;
    jb.llr = llr;
    jb.F = F;
    jb.u_hat = u_hat;
    jb.crc_ok = crc_ok;
    jb.pm = pm;
    jb.near_tie = near_tie;
    jb.pos = pos;
    run_jobs(&jb, threads);
    free(pos);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Decoder C: exhaustive ML over CRC-valid codewords.                        */
/* ------------------------------------------------------------------------ */

int orc_decode_ml(int N, int K, const uint8_t* frozen_mask, uint64_t poly, int r, int dtype,
                  const void* llr, int64_t F, uint8_t* u_hat, double* dist) {
    if (check_code(N, K, frozen_mask, r) || F < 0 || K - r > 20 || (F > 0 && (!llr || !u_hat)))
        return -1;
    if (dtype < ORC_F32 || dtype > ORC_I8) return -1;
    int* pos = (int*)malloc(sizeof(int) * (size_t)K);
    info_positions(N, frozen_mask, pos);
    int kp = K - r;
    uint8_t* info = (uint8_t*)malloc((size_t)K);
    uint8_t* x = (uint8_t*)malloc((size_t)N);
    for (int64_t f = 0; f < F; f++) {
        double best = INFINITY;
        for (long msg = 0; msg < (1L << kp); msg++) {
            for (int t = 0; t < kp; t++) info[t] = (uint8_t)((msg >> (kp - 1 - t)) & 1);
            if (r > 0) {
                uint64_t rem;
                orc_crc(info, kp, poly, r, &rem);
                for (int t = 0; t < r; t++) info[kp + t] = (uint8_t)((rem >> (r - 1 - t)) & 1);
            }
            memset(x, 0, (size_t)N);
            for (int t = 0; t < K; t++) x[pos[t]] = info[t];
            transform_rec(x, N);
            double dd = 0.0;
            for (int i = 0; i < N; i++) {
                double a = llr_at(dtype, llr, f * N + i);
                if ((int)x[i] != h_dec(a)) dd += fabs(a);
            }
            if (dd < best) {
                best = dd;
                memcpy(u_hat + f * K, info, (size_t)K);
            }
        }
        if (dist) dist[f] = best;
    }
    free(x);
    free(info);
    free(pos);
    return 0;
}
