/*
 * exsum_oracle.c -- CPU oracle for exact floating-point summation.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plainly correct
 * reference that the GPU library is checked against.  Only the tests, the
 * smoke check and the benchmark's CPU-baseline leg may load it; the GPU
 * library never links, calls or includes anything from here, and this file
 * includes nothing from the library.
 *
 * What it computes (Neal 2015, abstract and Introduction): the exact sum of
 * a set of binary64 values, rounded once to the nearest binary64 value with
 * ties to even.  The paper's superaccumulators are a fast route to that
 * value; this oracle does not follow them.  It uses the plain definition:
 *
 *   1. Decode each term as the format section defines it: sign s, exponent
 *      field e, mantissa field m; for 0 < e < 2047 the value is
 *      (-1)^s 2^(e-1023) (1 + m 2^-52); for e == 0 it is (-1)^s 2^-1022 m 2^-52;
 *      e == 2047 is an infinity (m == 0) or a NaN (m != 0).
 *   2. Every finite value is an integer multiple of 2^-1074 (the smallest
 *      denormal): M * 2^(e_eff - 1) units, with e_eff = max(e, 1) and
 *      M = m + 2^52 when e != 0 (the implicit bit), M = m otherwise.
 *   3. Positive and negative terms are added into two separate unsigned
 *      wide integers (34 limbs of 64 bits, 2176 bits; one term needs at
 *      most 2098 bits, leaving room for more than 2^77 terms).  Additions
 *      only, no borrows.
 *   4. The difference of the two is rounded to nearest, ties to even
 *      (section "Exact summation using a small superaccumulator", on
 *      obtaining the correctly rounded value), overflowing to an infinity
 *      when the rounded magnitude needs a biased exponent of 2047.
 *
 * Readings where the paper is silent (they fix the convention; the GPU
 * library follows the same ones):
 *   - an exact-zero sum (including n == 0 and sums of -0.0) is +0.0;
 *   - any NaN input gives a NaN whose bits are the largest (bits & ~sign)
 *     over the NaN inputs, with the quiet bit set (order independent);
 *   - +Inf together with -Inf (and no NaN) gives 0x7FF8000000000000;
 *   - an infinite input dominates any finite part, even one that would
 *     itself round to the opposite infinity.
 *
 * The same decode/accumulate/round definition, with the binary32 field
 * widths (8 exponent bits, 23 mantissa bits, units of 2^-149), gives the
 * single-precision sum the paper mentions as a smaller variant (Introduction).
 * The dot product and squared norm follow the Performance evaluations
 * section: each product is first rounded to binary64 by ordinary IEEE
 * multiplication, then the products are summed exactly.  The mean follows
 * the Discussion: the exact sum divided by n, rounded once.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#define LIMBS 34

typedef struct {
    uint64_t w[LIMBS];
} wide_t;

typedef struct {
    wide_t pos;            /* sum of positive finite terms */
    wide_t neg;            /* sum of magnitudes of negative finite terms */
    int pos_inf;
    int neg_inf;
    uint64_t nan_bits;     /* max over NaN inputs of (bits with sign cleared); 0 = none */
} acc_t;

/* ---- wide unsigned integer helpers ---------------------------------- */

/* w += M * 2^shift.  M < 2^64.  Carries ripple to the top limb. */
static void wide_add_shifted(wide_t *a, uint64_t M, int shift)
{
    int limb = shift / 64;
    int off = shift % 64;
    uint64_t lo = M << off;
    uint64_t hi = off ? (M >> (64 - off)) : 0;
    uint64_t old = a->w[limb];
    a->w[limb] = old + lo;
    uint64_t carry = a->w[limb] < old;
    int i = limb + 1;
    /* add hi + carry into the next limb, then ripple */
    uint64_t add = hi;
    while (i < LIMBS && (add != 0 || carry != 0)) {
        uint64_t o = a->w[i];
        uint64_t t = o + add;
        uint64_t c1 = t < o;
        uint64_t t2 = t + carry;
        uint64_t c2 = t2 < t;
        a->w[i] = t2;
        carry = c1 + c2;
        add = 0;
        i++;
    }
}

/* a += b */
static void wide_add(wide_t *a, const wide_t *b)
{
    uint64_t carry = 0;
    for (int i = 0; i < LIMBS; i++) {
        uint64_t t = a->w[i] + b->w[i];
        uint64_t c1 = t < a->w[i];
        uint64_t t2 = t + carry;
        uint64_t c2 = t2 < t;
        a->w[i] = t2;
        carry = c1 + c2;
    }
}

/* -1, 0, +1 for a <, ==, > b */
static int wide_cmp(const wide_t *a, const wide_t *b)
{
    for (int i = LIMBS - 1; i >= 0; i--) {
        if (a->w[i] != b->w[i]) return a->w[i] > b->w[i] ? 1 : -1;
    }
    return 0;
}

/* r = a - b, requires a >= b */
static void wide_sub(wide_t *r, const wide_t *a, const wide_t *b)
{
    uint64_t borrow = 0;
    for (int i = 0; i < LIMBS; i++) {
        uint64_t t = a->w[i] - b->w[i];
        uint64_t b1 = a->w[i] < b->w[i];
        uint64_t t2 = t - borrow;
        uint64_t b2 = t < borrow;
        r->w[i] = t2;
        borrow = b1 + b2;
    }
}

/* number of significant bits (0 for zero) */
static int wide_bitlen(const wide_t *a)
{
    for (int i = LIMBS - 1; i >= 0; i--) {
        if (a->w[i]) return 64 * i + (64 - __builtin_clzll(a->w[i]));
    }
    return 0;
}

static int wide_bit(const wide_t *a, int pos)
{
    return (int)((a->w[pos / 64] >> (pos % 64)) & 1u);
}

/* (a >> pos) truncated to 64 bits */
static uint64_t wide_bits_at(const wide_t *a, int pos)
{
    int limb = pos / 64, off = pos % 64;
    uint64_t v = a->w[limb] >> off;
    if (off && limb + 1 < LIMBS) v |= a->w[limb + 1] << (64 - off);
    return v;
}

/* any bit set strictly below position pos */
static int wide_any_below(const wide_t *a, int pos)
{
    int limb = pos / 64, off = pos % 64;
    for (int i = 0; i < limb; i++) if (a->w[i]) return 1;
    if (off && (a->w[limb] & ((1ull << off) - 1))) return 1;
    return 0;
}

/* r = a >> s (s >= 1), with every discarded bit ORed into bit 0 of r. */
static void wide_shr_sticky(wide_t *r, const wide_t *a, int s)
{
    for (int i = 0; i < LIMBS; i++) {
        int pos = i * 64 + s;
        r->w[i] = pos < LIMBS * 64 ? wide_bits_at(a, pos) : 0;
    }
    if (wide_any_below(a, s)) r->w[0] |= 1;
}

/* q = a / d, returns a % d.  d > 0. */
static uint64_t wide_divmod_u64(wide_t *q, const wide_t *a, uint64_t d)
{
    unsigned __int128 rem = 0;
    for (int i = LIMBS - 1; i >= 0; i--) {
        unsigned __int128 cur = (rem << 64) | a->w[i];
        q->w[i] = (uint64_t)(cur / d);
        rem = cur % d;
    }
    return (uint64_t)rem;
}

/* ---- decode and accumulate -------------------------------------------- */

static void acc_init(acc_t *acc) { memset(acc, 0, sizeof *acc); }

/* Add one binary64 term, decoded per the format definitions. */
static void acc_add_f64(acc_t *acc, double v)
{
    uint64_t b;
    memcpy(&b, &v, sizeof b);
    uint64_t s = b >> 63;
    uint64_t e = (b >> 52) & 2047u;
    uint64_t m = b & ((1ull << 52) - 1);
    if (e == 2047) {
        if (m == 0) {
            if (s) acc->neg_inf = 1; else acc->pos_inf = 1;
        } else {
            uint64_t payload = b & 0x7FFFFFFFFFFFFFFFull;
            if (payload > acc->nan_bits) acc->nan_bits = payload;
        }
        return;
    }
    if (e == 0 && m == 0) return;                 /* +0 or -0 adds nothing */
    uint64_t e_eff = e ? e : 1;                   /* denormals: exponent 1, no implicit bit */
    uint64_t M = e ? (m | (1ull << 52)) : m;
    wide_add_shifted(s ? &acc->neg : &acc->pos, M, (int)(e_eff - 1));
}

/* Same for binary32 (8 exponent bits, 23 mantissa bits, units 2^-149). */
static void acc_add_f32(acc_t *acc, float v)
{
    uint32_t b;
    memcpy(&b, &v, sizeof b);
    uint32_t s = b >> 31;
    uint32_t e = (b >> 23) & 255u;
    uint32_t m = b & ((1u << 23) - 1);
    if (e == 255) {
        if (m == 0) {
            if (s) acc->neg_inf = 1; else acc->pos_inf = 1;
        } else {
            uint64_t payload = b & 0x7FFFFFFFu;
            if (payload > acc->nan_bits) acc->nan_bits = payload;
        }
        return;
    }
    if (e == 0 && m == 0) return;
    uint32_t e_eff = e ? e : 1;
    uint64_t M = e ? (m | (1u << 23)) : m;
    wide_add_shifted(s ? &acc->neg : &acc->pos, M, (int)(e_eff - 1));
}

static void acc_merge(acc_t *a, const acc_t *b)
{
    wide_add(&a->pos, &b->pos);
    wide_add(&a->neg, &b->neg);
    a->pos_inf |= b->pos_inf;
    a->neg_inf |= b->neg_inf;
    if (b->nan_bits > a->nan_bits) a->nan_bits = b->nan_bits;
}

/* ---- rounding ---------------------------------------------------------- */

/*
 * Round (A / d) * 2^(units) to the nearest value of a binary format with
 * `mbits` stored mantissa bits and all-ones exponent `emax`, ties to even.
 * A is a non-negative wide integer counting units of the smallest denormal;
 * d >= 1 is an exact divisor (1 for a plain sum, n for a mean).
 * Returns the magnitude bits (sign not included).
 */
static uint64_t round_quotient(const wide_t *A, uint64_t d, int mbits, uint64_t emax)
{
    wide_t Q;
    uint64_t R;
    if (d == 1) { Q = *A; R = 0; }
    else R = wide_divmod_u64(&Q, A, d);

    const uint64_t hidden = 1ull << mbits;       /* 2^52 for binary64 */
    int b = wide_bitlen(&Q);
    uint64_t q;
    int sh;
    int up;
    if (b <= mbits + 1) {
        /* Q < 2^(mbits+1): the unit of the last place is one unit; only the
         * fraction R/d is discarded. */
        sh = 0;
        q = Q.w[0];
        unsigned __int128 twoR = (unsigned __int128)R * 2;
        up = (twoR > d) || (twoR == d && (q & 1));
    } else {
        sh = b - (mbits + 1);
        q = wide_bits_at(&Q, sh) & ((hidden << 1) - 1);
        int round_bit = wide_bit(&Q, sh - 1);
        int sticky = wide_any_below(&Q, sh - 1) || R != 0;
        up = round_bit && (sticky || (q & 1));
    }
    if (up) q += 1;
    if (q < hidden) {
        /* denormal (or zero): the bits are the count of smallest units */
        return q;
    }
    if (q == (hidden << 1)) { q = hidden; sh += 1; }
    uint64_t E = (uint64_t)sh + 1;               /* biased exponent */
    if (E >= emax) return emax << mbits;         /* overflow to infinity */
    return (E << mbits) | (q - hidden);
}

/* Finish an accumulator: specials first, then the rounded difference. */
static uint64_t acc_result(const acc_t *acc, uint64_t d, int mbits, uint64_t emax, int width)
{
    const uint64_t sign_bit = 1ull << (width - 1);
    const uint64_t quiet = 1ull << (mbits - 1);
    if (acc->nan_bits) return acc->nan_bits | quiet;
    if (acc->pos_inf && acc->neg_inf) return (emax << mbits) | quiet;
    if (acc->pos_inf) return emax << mbits;
    if (acc->neg_inf) return sign_bit | (emax << mbits);
    int c = wide_cmp(&acc->pos, &acc->neg);
    if (c == 0) return 0;                        /* exact zero -> +0 */
    wide_t A;
    uint64_t s;
    if (c > 0) { wide_sub(&A, &acc->pos, &acc->neg); s = 0; }
    else       { wide_sub(&A, &acc->neg, &acc->pos); s = sign_bit; }
    uint64_t mag = round_quotient(&A, d, mbits, emax);
    if (mag == 0) return 0;                      /* a mean that rounds to zero -> +0 */
    return s | mag;
}

/* ---- exported entry points -------------------------------------------- */

uint64_t exo_sum_f64(const double *x, int64_t n)
{
    acc_t acc;
    acc_init(&acc);
    for (int64_t i = 0; i < n; i++) acc_add_f64(&acc, x[i]);
    return acc_result(&acc, 1, 52, 2047, 64);
}

void exo_segmented_f64(const double *x, const int64_t *offsets, int64_t nseg, uint64_t *out)
{
    for (int64_t s = 0; s < nseg; s++) {
        acc_t acc;
        acc_init(&acc);
        for (int64_t i = offsets[s]; i < offsets[s + 1]; i++) acc_add_f64(&acc, x[i]);
        out[s] = acc_result(&acc, 1, 52, 2047, 64);
    }
}

/* Sum of x[idx[j]] for j < m: used to check sampled requests of a pool. */
void exo_sum_ranges_f64(const double *x, const int64_t *starts, const int64_t *lens,
                        int64_t nr, uint64_t *out)
{
    for (int64_t r = 0; r < nr; r++) {
        acc_t acc;
        acc_init(&acc);
        for (int64_t i = 0; i < lens[r]; i++) acc_add_f64(&acc, x[starts[r] + i]);
        out[r] = acc_result(&acc, 1, 52, 2047, 64);
    }
}

uint64_t exo_mean_f64(const double *x, int64_t n)
{
    acc_t acc;
    acc_init(&acc);
    for (int64_t i = 0; i < n; i++) acc_add_f64(&acc, x[i]);
    if (n <= 0) return 0;
    return acc_result(&acc, (uint64_t)n, 52, 2047, 64);
}

uint64_t exo_dot_f64(const double *x, const double *y, int64_t n)
{
    acc_t acc;
    acc_init(&acc);
    for (int64_t i = 0; i < n; i++) {
        volatile double p = x[i] * y[i];          /* rounded to binary64 */
        acc_add_f64(&acc, p);
    }
    return acc_result(&acc, 1, 52, 2047, 64);
}

uint64_t exo_sqnorm_f64(const double *x, int64_t n)
{
    acc_t acc;
    acc_init(&acc);
    for (int64_t i = 0; i < n; i++) {
        volatile double p = x[i] * x[i];
        acc_add_f64(&acc, p);
    }
    return acc_result(&acc, 1, 52, 2047, 64);
}

uint32_t exo_sum_f32(const float *x, int64_t n)
{
    acc_t acc;
    acc_init(&acc);
    for (int64_t i = 0; i < n; i++) acc_add_f32(&acc, x[i]);
    return (uint32_t)acc_result(&acc, 1, 23, 255, 32);
}

/*
 * Exact dot product of binary32 vectors (Introduction: the single-precision
 * variant; Performance evaluations: the dot product).  Each product of two
 * binary32 values is exact as a binary64 value (24-bit by 24-bit mantissas
 * fit in 53 bits, and the exponents stay inside the binary64 range), so the
 * products are formed in binary64, summed exactly, and the sum is rounded
 * once to binary32.  The accumulator counts units of 2^-1074; binary32's
 * smallest unit is 2^-149, 2^925 of them.  Two more bits are kept (units of
 * 2^-151) with everything below folded into a sticky bit, and the quotient
 * by 4 is rounded in binary32.  A nonzero sum that rounds to zero gives +0,
 * as for the mean.  A NaN product maps back to binary32 by dropping the 29
 * low payload bits.
 */
uint32_t exo_dot_f32(const float *x, const float *y, int64_t n)
{
    acc_t acc;
    acc_init(&acc);
    for (int64_t i = 0; i < n; i++) {
        volatile double p = (double)x[i] * (double)y[i];   /* exact */
        acc_add_f64(&acc, p);
    }
    if (acc.nan_bits) return 0x7FC00000u | (uint32_t)((acc.nan_bits >> 29) & 0x7FFFFFu);
    if (acc.pos_inf && acc.neg_inf) return 0x7FC00000u;
    if (acc.pos_inf) return 0x7F800000u;
    if (acc.neg_inf) return 0xFF800000u;
    int c = wide_cmp(&acc.pos, &acc.neg);
    if (c == 0) return 0;
    wide_t A, B;
    uint32_t s;
    if (c > 0) { wide_sub(&A, &acc.pos, &acc.neg); s = 0; }
    else       { wide_sub(&A, &acc.neg, &acc.pos); s = 0x80000000u; }
    wide_shr_sticky(&B, &A, 923);
    uint64_t mag = round_quotient(&B, 4, 23, 255);
    if (mag == 0) return 0;
    return s | (uint32_t)mag;
}

/* Multi-threaded variant, for timing the CPU baseline only: contiguous
 * parts are accumulated separately, their wide integers added exactly,
 * and the total rounded once. */
typedef struct {
    const double *x;
    int64_t lo, hi;
    acc_t acc;
} part_t;

static void *part_run(void *arg)
{
    part_t *p = (part_t *)arg;
    acc_init(&p->acc);
    for (int64_t i = p->lo; i < p->hi; i++) acc_add_f64(&p->acc, p->x[i]);
    return NULL;
}

uint64_t exo_sum_f64_mt(const double *x, int64_t n, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
    part_t *parts = (part_t *)calloc((size_t)nthreads, sizeof(part_t));
    pthread_t *tids = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    for (int t = 0; t < nthreads; t++) {
        parts[t].x = x;
        parts[t].lo = n * t / nthreads;
        parts[t].hi = n * (t + 1) / nthreads;
        pthread_create(&tids[t], NULL, part_run, &parts[t]);
    }
    acc_t total;
    acc_init(&total);
    for (int t = 0; t < nthreads; t++) {
        pthread_join(tids[t], NULL);
        acc_merge(&total, &parts[t].acc);
    }
    free(parts);
    free(tids);
    return acc_result(&total, 1, 52, 2047, 64);
}

/*
 * Exact sums of many ranges of one finite pool through exact prefix sums, so
 * that a long trace of requests (slices of one resident pool) can be checked
 * in full.  Integer addition is exact and associative (Discussion: parts of a
 * sum are summed separately and added), so with P(k) = the positive and
 * negative wide sums of x[0 .. k*stride), the sum of x[a .. b) is
 *     P(kb) - P(ka) + (the terms x[a .. ka*stride) and x[kb*stride .. b)),
 * where ka = ceil(a / stride) and kb = floor(b / stride); when ka > kb the
 * range lies inside one stride and its terms are summed directly.  Each of
 * the two wide sums only grows with k, so both subtractions are of a smaller
 * unsigned integer from a larger one.  Infinities and NaNs cannot be
 * differenced: the pool must be finite.
 * Returns 0, or -1 (writing nothing) if the pool holds an infinity or NaN,
 * -2 for a range outside [0, n) or stride < 1.
 */
typedef struct {
    wide_t pos, neg;
} prefix_t;

typedef struct {
    const double *x;
    const prefix_t *cp;
    int64_t stride;
    const int64_t *starts, *lens;
    int64_t lo, hi;
    uint64_t *out;
} ranges_job_t;

static void *ranges_run(void *arg)
{
    ranges_job_t *j = (ranges_job_t *)arg;
    for (int64_t r = j->lo; r < j->hi; r++) {
        int64_t a = j->starts[r], b = a + j->lens[r];
        int64_t ka = (a + j->stride - 1) / j->stride, kb = b / j->stride;
        acc_t acc;
        acc_init(&acc);
        if (ka > kb) {
            for (int64_t i = a; i < b; i++) acc_add_f64(&acc, j->x[i]);
        } else {
            wide_sub(&acc.pos, &j->cp[kb].pos, &j->cp[ka].pos);
            wide_sub(&acc.neg, &j->cp[kb].neg, &j->cp[ka].neg);
            for (int64_t i = a; i < ka * j->stride; i++) acc_add_f64(&acc, j->x[i]);
            for (int64_t i = kb * j->stride; i < b; i++) acc_add_f64(&acc, j->x[i]);
        }
        j->out[r] = acc_result(&acc, 1, 52, 2047, 64);
    }
    return NULL;
}

int exo_ranges_by_prefix_f64(const double *x, int64_t n, const int64_t *starts, const int64_t *lens,
                             int64_t nr, int64_t stride, int nthreads, uint64_t *out)
{
    if (stride < 1 || n < 0) return -2;
    for (int64_t r = 0; r < nr; r++)
        if (starts[r] < 0 || lens[r] < 0 || starts[r] > n - lens[r]) return -2;
    int64_t K = n / stride;
    prefix_t *cp = (prefix_t *)calloc((size_t)K + 1, sizeof(prefix_t));
    if (!cp) return -2;
    acc_t run;
    acc_init(&run);
    for (int64_t k = 1; k <= K; k++) {
        for (int64_t i = (k - 1) * stride; i < k * stride; i++) acc_add_f64(&run, x[i]);
        cp[k].pos = run.pos;
        cp[k].neg = run.neg;
    }
    for (int64_t i = K * stride; i < n; i++) acc_add_f64(&run, x[i]);
    if (run.pos_inf || run.neg_inf || run.nan_bits) {
        free(cp);
        return -1;
    }
    if (nthreads < 1) nthreads = 1;
    ranges_job_t *jobs = (ranges_job_t *)calloc((size_t)nthreads, sizeof(ranges_job_t));
    pthread_t *tids = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    for (int t = 0; t < nthreads; t++) {
        jobs[t] = (ranges_job_t){x, cp, stride, starts, lens, nr * t / nthreads, nr * (t + 1) / nthreads, out};
        pthread_create(&tids[t], NULL, ranges_run, &jobs[t]);
    }
    for (int t = 0; t < nthreads; t++) pthread_join(tids[t], NULL);
    free(jobs);
    free(tids);
    free(cp);
    return 0;
}
