/*
 * CPU oracle for the multilinear ZeroCheck SumCheck prover, in plain C.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests (parity at full size) and by
 * the benchmark's CPU-baseline leg.  It shares no code with the HIP library
 * and is itself checked against the Python oracle (oracle/zc_oracle.py).
 *
 * It computes exactly what the Python oracle computes (same readings of the
 * paper, listed there): the algorithm of Fig. 2 (right) of "When Proofs Meet
 * Hardware" -- build eq_r (Sec. 3.3), then for i = 1..mu the round
 * polynomial G_i at X = 0..d+1 over the remaining hypercube, the SHA-256
 * Fiat-Shamir challenge alpha_i, and the fold of every table (eq included)
 * with alpha_i (Sec. 4.1); the openings are the folded single values.
 *
 * Field: BN254 scalar field, elements as 4 x 64-bit little-endian limbs,
 * held in Montgomery form (R = 2^256) inside, canonical at the interface.
 * Only p is written down; -p^-1 mod 2^64 and R^2 mod p are derived at start.
 * Parallelism: OpenMP over hypercube pairs, per-thread partial sums (field
 * addition is exact, so the order of the sums does not matter).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>
#include <openssl/sha.h>

typedef unsigned __int128 u128;
typedef struct { uint64_t v[4]; } fe;

static const fe FP = {{0x43e1f593f0000001ULL, 0x2833e84879b97091ULL,
                       0xb85045b68181585dULL, 0x30644e72e131a029ULL}};
static uint64_t NINV;  /* -p^-1 mod 2^64 */
static fe R2;          /* 2^512 mod p */
static fe ONE_M;       /* R mod p (Montgomery form of 1) */
static int inited;

static int geq(const fe *a, const fe *b) {
    for (int i = 3; i >= 0; --i) {
        if (a->v[i] != b->v[i]) return a->v[i] > b->v[i];
    }
    return 1;
}

static fe sub_raw(fe a, fe b, uint64_t *borrow) {
    fe r;
    uint64_t br = 0;
    for (int i = 0; i < 4; ++i) {
        u128 d = (u128)a.v[i] - b.v[i] - br;
        r.v[i] = (uint64_t)d;
        br = (uint64_t)(d >> 64) ? 1 : 0;
    }
    *borrow = br;
    return r;
}

static fe add_raw(fe a, fe b, uint64_t *carry) {
    fe r;
    uint64_t c = 0;
    for (int i = 0; i < 4; ++i) {
        u128 s = (u128)a.v[i] + b.v[i] + c;
        r.v[i] = (uint64_t)s;
        c = (uint64_t)(s >> 64);
    }
    *carry = c;
    return r;
}

static fe fadd(fe a, fe b) {
    uint64_t c, br;
    fe r = add_raw(a, b, &c);
    if (c || geq(&r, &FP)) r = sub_raw(r, FP, &br);
    return r;
}

static fe fsub(fe a, fe b) {
    uint64_t br, c;
    fe r = sub_raw(a, b, &br);
    if (br) r = add_raw(r, FP, &c);
    return r;
}

/* Montgomery product a*b*R^-1 mod p (CIOS, 64-bit words). */
static fe fmul(fe a, fe b) {
    uint64_t t[6] = {0, 0, 0, 0, 0, 0};
    for (int i = 0; i < 4; ++i) {
        u128 c = 0;
        for (int j = 0; j < 4; ++j) {
            c = (u128)a.v[j] * b.v[i] + t[j] + (uint64_t)(c >> 64);
            t[j] = (uint64_t)c;
        }
        c = (u128)t[4] + (uint64_t)(c >> 64);
        t[4] = (uint64_t)c;
        t[5] = (uint64_t)(c >> 64);
        uint64_t m = t[0] * NINV;
        c = (u128)m * FP.v[0] + t[0];
        for (int j = 1; j < 4; ++j) {
            c = (u128)m * FP.v[j] + t[j] + (uint64_t)(c >> 64);
            t[j - 1] = (uint64_t)c;
        }
        c = (u128)t[4] + (uint64_t)(c >> 64);
        t[3] = (uint64_t)c;
        t[4] = t[5] + (uint64_t)(c >> 64);
    }
    fe r = {{t[0], t[1], t[2], t[3]}};
    uint64_t br;
    if (t[4] || geq(&r, &FP)) r = sub_raw(r, FP, &br);
    return r;
}

static void init_consts(void) {
    if (inited) return;
    /* Newton iteration for p^-1 mod 2^64 (p odd): x <- x (2 - p x). */
    uint64_t x = 1;
    for (int i = 0; i < 7; ++i) x *= 2 - FP.v[0] * x;
    NINV = (uint64_t)0 - x;
    /* R mod p and R^2 mod p by repeated modular doubling of 1. */
    fe one = {{1, 0, 0, 0}};
    fe v = one;
    for (int i = 0; i < 512; ++i) {
        v = fadd(v, v);
        if (i == 255) ONE_M = v;
    }
    R2 = v;
    inited = 1;
}

static fe to_mont(fe a) { return fmul(a, R2); }
static fe from_mont(fe a) { fe one = {{1, 0, 0, 0}}; return fmul(a, one); }
static fe small(uint64_t k) { fe a = {{k, 0, 0, 0}}; return to_mont(a); }

/* ------------------------------------------------------------------ gate */
enum { GATE_VANILLA = 0, GATE_PROD = 1, GATE_SUMPROD = 2 };

/* Table 1 shapes g1..gP + gP+1..gP+A, m = P + 16 A. */
static int sumprod_ok(uint32_t m) {
    uint32_t pp = m & 15, aa = m >> 4;
    return (pp == 2 && aa <= 3) || ((pp == 3 || pp == 4) && aa == 0);
}

static int gate_ntables(uint32_t gate, uint32_t m) {
    if (gate == GATE_VANILLA) return 8;
    if (gate == GATE_PROD && m >= 1 && m <= 8) return (int)m + 2;
    if (gate == GATE_SUMPROD && sumprod_ok(m)) return (int)((m & 15) + (m >> 4));
    return -1;
}

static int gate_degree(uint32_t gate, uint32_t m) {
    if (gate == GATE_VANILLA) return 3;
    if (gate == GATE_SUMPROD) return (int)(m & 15);
    return (int)m + 1;
}

/* f_M on one value per witness table, Montgomery form in and out. */
static fe gate_value(uint32_t gate, uint32_t m, const fe *v) {
    if (gate == GATE_VANILLA) {
        /* qM*a*b + qL*a + qR*b + qO*c + qC; columns a b c qM qL qR qO qC */
        fe t = fmul(fmul(v[3], v[0]), v[1]);
        t = fadd(t, fmul(v[4], v[0]));
        t = fadd(t, fmul(v[5], v[1]));
        t = fadd(t, fmul(v[6], v[2]));
        return fadd(t, v[7]);
    }
    if (gate == GATE_SUMPROD) {
        /* g1*...*gP + gP+1 + ... + gP+A */
        uint32_t pp = m & 15, aa = m >> 4;
        fe t = v[0];
        for (uint32_t k = 1; k < pp; ++k) t = fmul(t, v[k]);
        for (uint32_t k = 0; k < aa; ++k) t = fadd(t, v[pp + k]);
        return t;
    }
    fe prod = v[0];
    for (uint32_t k = 1; k <= m; ++k) prod = fmul(prod, v[k]);
    return fsub(prod, v[m + 1]);
}

/* Gate degree d, or -1 for an unknown gate (exported for the wrapper). */
int zco_degree(uint32_t gate, uint32_t m) {
    return gate_ntables(gate, m) < 0 ? -1 : gate_degree(gate, m);
}

/* ------------------------------------------------------------ transcript */
static void put_canon(uint8_t *out, fe mont) {
    fe c = from_mont(mont);
    for (int i = 0; i < 4; ++i)
        for (int b = 0; b < 8; ++b) out[8 * i + b] = (uint8_t)(c.v[i] >> (8 * b));
}

static fe digest_to_field(const uint8_t *dg) {
    fe a;
    for (int i = 0; i < 4; ++i) {
        uint64_t w = 0;
        for (int b = 7; b >= 0; --b) w = (w << 8) | dg[8 * i + b];
        a.v[i] = w;
    }
    uint64_t br;
    while (geq(&a, &FP)) a = sub_raw(a, FP, &br);
    return a;
}

/* ------------------------------------------------------------------ prove */
/*
 * tables: k x 2^mu x 4 u64, canonical little-endian, gate column order.
 * r: mu x 4 u64 canonical.  Outputs canonical: evals mu x (d+2) x 4,
 * alphas mu x 4, openings (k+1) x 4 (eq last).  nthreads <= 0: OpenMP default.
 * Returns 0, or -1 (bad shape), -4 (an input >= p), -3 (out of memory).
 */
int zco_prove(uint32_t mu, uint32_t gate, uint32_t m, const uint64_t *tables,
              const uint64_t *r, uint64_t *evals, uint64_t *alphas, uint64_t *openings,
              int nthreads) {
    init_consts();
    int kw = gate_ntables(gate, m);
    if (kw < 0 || mu < 1 || mu > 30 || !tables || !r || !evals || !alphas || !openings)
        return -1;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    const int d = gate_degree(gate, m);
    const int k = kw + 1;
    const uint64_t n = (uint64_t)1 << mu;

    fe *rm = (fe *)malloc(sizeof(fe) * mu);
    fe **tab = (fe **)calloc((size_t)k, sizeof(fe *));
    if (!rm || !tab) { free(rm); free(tab); return -3; }
    for (int t = 0; t < k; ++t) {
        tab[t] = (fe *)malloc(sizeof(fe) * n);
        if (!tab[t]) {
            for (int u = 0; u < t; ++u) free(tab[u]);
            free(tab); free(rm);
            return -3;
        }
    }
    int bad = 0;
    for (uint32_t i = 0; i < mu; ++i) {
        fe a;
        memcpy(a.v, r + 4 * i, 32);
        if (geq(&a, &FP)) bad = 1;
        rm[i] = to_mont(a);
    }
    for (int t = 0; t < kw; ++t) {
        const uint64_t *src = tables + (uint64_t)t * n * 4;
        int tbad = 0;
#pragma omp parallel for reduction(| : tbad)
        for (int64_t b = 0; b < (int64_t)n; ++b) {
            fe a;
            memcpy(a.v, src + 4 * b, 32);
            if (geq(&a, &FP)) tbad = 1;
            tab[t][b] = to_mont(a);
        }
        bad |= tbad;
    }
    if (bad) {
        for (int t = 0; t < k; ++t) free(tab[t]);
        free(tab); free(rm);
        return -4;
    }

    /* Build MLE (definition): E[b] = prod_i (x_i ? r_i : 1 - r_i), x_1 = MSB. */
    {
        fe *E = tab[kw];
        const fe one = ONE_M;
#pragma omp parallel for
        for (int64_t b = 0; b < (int64_t)n; ++b) {
            fe acc = one;
            for (uint32_t i = 0; i < mu; ++i) {
                int xi = (int)((b >> (mu - 1 - i)) & 1);
                acc = fmul(acc, xi ? rm[i] : fsub(one, rm[i]));
            }
            E[b] = acc;
        }
    }

    /* Transcript T_0 = SHA-256("ZCv1" || mu || gate || m || enc(r_1..r_mu)). */
    uint8_t ts[32];
    {
        size_t len = 16 + 32 * (size_t)mu;
        uint8_t *msg = (uint8_t *)malloc(len);
        memcpy(msg, "ZCv1", 4);
        uint32_t hdr[3] = {mu, gate, m};
        for (int i = 0; i < 3; ++i)
            for (int b = 0; b < 4; ++b) msg[4 + 4 * i + b] = (uint8_t)(hdr[i] >> (8 * b));
        for (uint32_t i = 0; i < mu; ++i) put_canon(msg + 16 + 32 * i, rm[i]);
        SHA256(msg, len, ts);
        free(msg);
    }

    fe xs[12];
    for (int x = 0; x < 12; ++x) xs[x] = small((uint64_t)x);

    uint64_t len = n;
    for (uint32_t i = 1; i <= mu; ++i) {
        const uint64_t h = len / 2;
        fe G[12];
        for (int x = 0; x < d + 2; ++x) memset(&G[x], 0, sizeof(fe));
#pragma omp parallel
        {
            fe part[12];
            for (int x = 0; x < d + 2; ++x) memset(&part[x], 0, sizeof(fe));
            fe ext[12];
#pragma omp for
            for (int64_t j = 0; j < (int64_t)h; ++j) {
                for (int x = 0; x < d + 2; ++x) {
                    for (int t = 0; t < k; ++t) {
                        fe lo = tab[t][j], hi = tab[t][j + h];
                        ext[t] = fadd(lo, fmul(xs[x], fsub(hi, lo)));
                    }
                    part[x] = fadd(part[x], fmul(gate_value(gate, m, ext), ext[kw]));
                }
            }
#pragma omp critical
            for (int x = 0; x < d + 2; ++x) G[x] = fadd(G[x], part[x]);
        }
        /* T_i = SHA-256(T_{i-1} || enc(G_i(0)) .. enc(G_i(d+1))); alpha_i = T_i mod p. */
        uint8_t msg[32 + 32 * 12];
        memcpy(msg, ts, 32);
        for (int x = 0; x < d + 2; ++x) {
            put_canon(msg + 32 + 32 * x, G[x]);
            memcpy(evals + ((uint64_t)(i - 1) * (d + 2) + x) * 4, msg + 32 + 32 * x, 32);
        }
        SHA256(msg, 32 + 32 * (size_t)(d + 2), ts);
        fe alpha_c = digest_to_field(ts);
        memcpy(alphas + (uint64_t)(i - 1) * 4, alpha_c.v, 32);
        fe alpha = to_mont(alpha_c);
        /* fold every table: t'[j] = t[j] + alpha (t[j+h] - t[j]) */
        for (int t = 0; t < k; ++t) {
            fe *T = tab[t];
#pragma omp parallel for
            for (int64_t j = 0; j < (int64_t)h; ++j) T[j] = fadd(T[j], fmul(alpha, fsub(T[j + h], T[j])));
        }
        len = h;
    }
    for (int t = 0; t < k; ++t) {
        fe c = from_mont(tab[t][0]);
        memcpy(openings + 4 * t, c.v, 32);
        free(tab[t]);
    }
    free(tab);
    free(rm);
    return 0;
}

/* Number of OpenMP threads the oracle would use. */
int zco_max_threads(void) { return omp_get_max_threads(); }
