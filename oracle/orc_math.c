/*
 * Oracle elementary functions and random numbers.  TEST INFRASTRUCTURE ONLY.
 *
 * The method's results must not depend on which libm evaluates log, exp,
 * cbrt, sin and cos, because the Monte-Carlo collision map amplifies last-bit
 * differences from step to step.  The method is therefore defined with the
 * specific function algorithms below, built only from IEEE-754 correctly
 * rounded +, -, *, / and sqrt (no contraction into fused multiply-add).  Each
 * is pinned against the C library's function in the tests (a few ulp).
 *
 *   log  : x = m 2^e, m in (sqrt(1/2), sqrt(2)]; f = m - 1, s = f / (2 + f),
 *          log(1+f) = f - s (f - V) with V the atanh series in s^2 to s^22
 *          (2 atanh s = 2s + 2s^3/3 + ...; 2s = f - s f); ln 2 split hi + lo.
 *   exp  : k = nearest integer to x / ln 2, r = (x - k ln2_hi) - k ln2_lo,
 *          Taylor polynomial of degree 13 by Horner, scaled by 2^k.
 *   cbrt : exponent split by 3, start 1 + (m' - 1)/7 on m' in [1, 8), six
 *          Newton steps y <- y + (m'/y^2 - y)/3.
 *   sincos of 2 pi (k + 1/2) / 2^52 for a 52-bit integer k: exact reduction to
 *          the nearest quarter turn in integers, then Taylor polynomials in
 *          theta = f pi/2, |theta| <= pi/4 (sine to theta^17, cosine to theta^16).
 *
 * Philox4x32-10 follows Salmon, Moraes, Dror, Shaw, "Parallel random numbers:
 * as easy as 1, 2, 3" (SC'11): multipliers 0xD2511F53 and 0xCD9E8D57, Weyl key
 * increments 0x9E3779B9 and 0xBB67AE85, ten rounds.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "orc.h"

static const double LN2_HI = 0x1.62e42p-1;            /* ln 2 with 21 significant bits */
static const double LN2_LO = 0x1.fdf473de6af28p-22;   /* ln 2 - LN2_HI */
static const double INV_LN2 = 0x1.71547652b82fep+0;
static const double SQRT2 = 0x1.6a09e667f3bcdp+0;
static const double PIO2 = 0x1.921fb54442d18p+0;

static double from_bits(uint64_t b) { double d; memcpy(&d, &b, 8); return d; }
static uint64_t to_bits(double d) { uint64_t b; memcpy(&b, &d, 8); return b; }

/* 2^n for -1022 <= n <= 1023 */
static double pow2i(int n) { return from_bits((uint64_t)(n + 1023) << 52); }

double orc_log(double x)
{
    if (x != x || x < 0.0) return NAN;
    if (x == 0.0) return -INFINITY;
    if (x == INFINITY) return INFINITY;
    int e_adj = 0;
    uint64_t b = to_bits(x);
    if (((b >> 52) & 0x7ff) == 0) {          /* subnormal: scale into normal range */
        x = x * 0x1p54;
        e_adj = -54;
        b = to_bits(x);
    }
    int e = (int)((b >> 52) & 0x7ff) - 1023 + e_adj;
    double m = from_bits((b & 0x000fffffffffffffULL) | 0x3ff0000000000000ULL);
    if (m > SQRT2) { m = m * 0.5; e = e + 1; }
    double f = m - 1.0;
    double s = f / (2.0 + f);
    double s2 = s * s;
    double v = 2.0 / 23.0;
    v = 2.0 / 21.0 + s2 * v;
    v = 2.0 / 19.0 + s2 * v;
    v = 2.0 / 17.0 + s2 * v;
    v = 2.0 / 15.0 + s2 * v;
    v = 2.0 / 13.0 + s2 * v;
    v = 2.0 / 11.0 + s2 * v;
    v = 2.0 / 9.0 + s2 * v;
    v = 2.0 / 7.0 + s2 * v;
    v = 2.0 / 5.0 + s2 * v;
    v = 2.0 / 3.0 + s2 * v;
    v = s2 * v;
    double lg = f - s * (f - v);
    double de = (double)e;
    return de * LN2_HI + (lg + de * LN2_LO);
}

double orc_exp(double x)
{
    if (x != x) return x;
    if (x > 709.78) return INFINITY;
    if (x < -745.14) return 0.0;
    double k = floor(x * INV_LN2 + 0.5);
    double hi = x - k * LN2_HI;
    double lo = k * LN2_LO;
    double r = hi - lo;
    double p = 1.0 / 6227020800.0;           /* 1/13! */
    p = 1.0 / 479001600.0 + r * p;           /* 1/12! */
    p = 1.0 / 39916800.0 + r * p;
    p = 1.0 / 3628800.0 + r * p;
    p = 1.0 / 362880.0 + r * p;
    p = 1.0 / 40320.0 + r * p;
    p = 1.0 / 5040.0 + r * p;
    p = 1.0 / 720.0 + r * p;
    p = 1.0 / 120.0 + r * p;
    p = 1.0 / 24.0 + r * p;
    p = 1.0 / 6.0 + r * p;
    p = 0.5 + r * p;
    p = 1.0 + r * p;
    p = 1.0 + r * p;
    int ki = (int)k;
    if (ki > 1023) return (p * 2.0) * pow2i(ki - 1);
    if (ki < -1022) return (p * pow2i(ki + 600)) * pow2i(-600);
    return p * pow2i(ki);
}

double orc_cbrt(double x)
{
    if (x != x) return x;
    if (x == 0.0) return x;
    if (x < 0.0) return -orc_cbrt(-x);
    if (x == INFINITY) return x;
    double post = 1.0;
    uint64_t b = to_bits(x);
    if (((b >> 52) & 0x7ff) == 0) {
        x = x * 0x1p54;
        post = 0x1p-18;
        b = to_bits(x);
    }
    int e = (int)((b >> 52) & 0x7ff) - 1023;
    int r = ((e % 3) + 3) % 3;
    int e3 = (e - r) / 3;
    double m = from_bits((b & 0x000fffffffffffffULL) | 0x3ff0000000000000ULL);
    if (r == 1) m = m * 2.0;
    if (r == 2) m = m * 4.0;
    double y = 1.0 + (m - 1.0) * (1.0 / 7.0);
    for (int it = 0; it < 6; ++it) {
        double t = m / (y * y);
        y = y + (t - y) / 3.0;
    }
    return (y * pow2i(e3)) * post;
}

void orc_sincos2pi(uint64_t k, double *s_out, double *c_out)
{
    k &= 0x000fffffffffffffULL;
    int64_t q = (int64_t)((k + (1ULL << 49)) >> 50);     /* nearest quarter turn, 0..4 */
    int64_t rem = (int64_t)k - (q << 50);                 /* in [-2^49, 2^49) */
    double f = ((double)rem + 0.5) * 0x1p-50;             /* exact, in [-1/2, 1/2) */
    double th = f * PIO2;
    double t2 = th * th;
    double sp = 1.0 / 355687428096000.0;                 /* 1/17! */
    sp = -1.0 / 1307674368000.0 + t2 * sp;               /* -1/15! */
    sp = 1.0 / 6227020800.0 + t2 * sp;
    sp = -1.0 / 39916800.0 + t2 * sp;
    sp = 1.0 / 362880.0 + t2 * sp;
    sp = -1.0 / 5040.0 + t2 * sp;
    sp = 1.0 / 120.0 + t2 * sp;
    sp = -1.0 / 6.0 + t2 * sp;
    double sn = th + th * (t2 * sp);
    double cp = 1.0 / 20922789888000.0;                  /* 1/16! */
    cp = -1.0 / 87178291200.0 + t2 * cp;                 /* -1/14! */
    cp = 1.0 / 479001600.0 + t2 * cp;
    cp = -1.0 / 3628800.0 + t2 * cp;
    cp = 1.0 / 40320.0 + t2 * cp;
    cp = -1.0 / 720.0 + t2 * cp;
    cp = 1.0 / 24.0 + t2 * cp;
    cp = -0.5 + t2 * cp;
    double cs = 1.0 + t2 * cp;
    switch (q & 3) {
    case 0: *s_out = sn; *c_out = cs; break;
    case 1: *s_out = cs; *c_out = -sn; break;
    case 2: *s_out = -sn; *c_out = -cs; break;
    default: *s_out = -cs; *c_out = sn; break;
    }
}

void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void orc_philox_many(int64_t n, const uint32_t *ctr, const uint32_t *key, uint32_t *out)
{
    for (int64_t i = 0; i < n; ++i) orc_philox(ctr + 4 * i, key + 2 * i, out + 4 * i);
}

/* Uniform on the open interval (0, 1) from a 32-bit word. */
double orc_u32(uint32_t x)
{
    return ((double)x + 0.5) * 0x1p-32;
}

/* Uniform on the open interval (0, 1) from the top 52 bits of (hi, lo). */
double orc_u52(uint32_t hi, uint32_t lo)
{
    uint64_t a = ((uint64_t)hi << 32) | lo;
    return ((double)(a >> 12) + 0.5) * 0x1p-52;
}

/*
 * Random permutation of [0, n): the slots sorted by (key[slot], slot), i.e. a
 * stable sort on 32-bit random keys.  Pairing is defined on this permutation.
 */
typedef struct { uint32_t key; int32_t slot; } keyed;

static int cmp_keyed(const void *a, const void *b)
{
    const keyed *x = (const keyed *)a, *y = (const keyed *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->slot < y->slot ? -1 : (x->slot > y->slot ? 1 : 0);
}

void orc_perm(int32_t n, const uint32_t *keys, int32_t *out)
{
    if (n <= 0) return;
    keyed *t = malloc(sizeof(keyed) * (size_t)n);
    for (int32_t i = 0; i < n; ++i) { t[i].key = keys[i]; t[i].slot = i; }
    qsort(t, (size_t)n, sizeof(keyed), cmp_keyed);
    for (int32_t i = 0; i < n; ++i) out[i] = t[i].slot;
    free(t);
}
