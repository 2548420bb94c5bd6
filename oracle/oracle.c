/*
 * CPU oracle for Ozaki-scheme multi-component matrix multiplication.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is loaded by the tests, by the
 * smoke check and by the CPU-baseline leg of the benchmark.  The product
 * library never links, loads or calls it, and it shares no code with it.
 *
 * Plain, slow and written to be read against the paper (Utsugiri & Kouya,
 * "Acceleration of Multiple Precision Matrix Multiplication using Ozaki
 * scheme", arXiv 2301.09960):
 *
 *   - Section 3, Algorithm 1: the split loop (row/column maxima mu, power-of-
 *     two shifts tau = 2^(ceil(log2 mu) + ceil((S + log2 l)/2)), extraction
 *     A_alpha = (A^(S) + S_A) - S_A, L-bit residual update), the triangular
 *     set of slice products C_ab = A_a B_b with a + b <= D + 1, and the L-bit
 *     accumulation C := C + sum_b C_ab taken alpha by alpha.
 *   - Section 3 (discussion after Fig. 1): every C_ab is computed without
 *     error; here each one is computed by exact integer arithmetic.
 *   - Section 4.1: the "simple matrix multiplication" (a triple loop in the
 *     multi-component format) is oracle_gemm_naive.
 *   - Section 1, eq. (1) and below it: the error measure is the maximum
 *     relative error over the elements of C; the exact product needed for it
 *     is oracle_gemm_exact_check (a long fixed-point accumulator).
 *
 * Readings where the paper is silent:
 *   - Layout: component-planar, column-major.  Matrix X with `rows` rows and
 *     `cols` columns stores component r of element (i, p) at
 *     X[r*rows*cols + i + p*rows].
 *   - A^(S) is the leading component of the current residual.  Before the
 *     first pass this is the input's component 0 as given (inputs are taken to
 *     be normalized expansions); after each update the residual is renormalized
 *     by renorm() below, an exact procedure, and its component 0 is taken.
 *   - D passes of the loop are made (D slices extracted); the remainder left
 *     after D passes is dropped, so every slice product is exact.  (Taking the
 *     rounded remainder as the last slice, literally A_D := A^(S), would make
 *     products with it inexact.)
 *   - mu = 0 (an all-zero row or column) gives an all-zero slice; its exponent
 *     is reported as INT_MIN.
 *   - ceil((S + log2 l)/2) is computed in integers as (S + ceil(log2 l) + 1)/2.
 *   - INT8 slices (not in the paper): E = 1 + max ilogb(x_0) over the row (or
 *     column); digit s (s = 1..D) is Algorithm 1's extraction (x + tau) - tau
 *     on the fixed grid u_s = 2^(E - 6 - 7 (s - 1)) instead of a grid set by
 *     the residual's maximum, applied to the exact residual (the whole
 *     expansion, not its leading component): the residual rounded to nearest
 *     on that grid; |digit| <= 64; the rest is dropped.
 *
 * Built with: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC
 * (IEEE binary64/binary32, round to nearest, no contraction, SSE2 evaluation).
 */
#include <float.h>
#include <limits.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_ENOMEM 2
#define ORC_ENOTEXACT 3 /* a slice was off its grid or a product sum too large */

#define ZERO_EXP INT_MIN
#define ORC_MAXC 16 /* longest expansion handled (components of binary64) */

/* ------------------------------------------------------------------------- */
/* Error-free transformations.                                                */
/* ------------------------------------------------------------------------- */

/* Knuth's TwoSum: s + e == a + b exactly, s = fl(a + b).  No precondition. */
static double two_sum(double a, double b, double *e)
{
    double s = a + b;
    double bb = s - a;
    *e = (a - (s - bb)) + (b - bb);
    return s;
}

static float two_sum_f(float a, float b, float *e)
{
    float s = a + b;
    float bb = s - a;
    *e = (a - (s - bb)) + (b - bb);
    return s;
}

/* TwoProd with a fused multiply-add: p + e == a * b exactly (no underflow). */
static double two_prod(double a, double b, double *e)
{
    double p = a * b;
    *e = fma(a, b, -p);
    return p;
}

double oracle_two_sum(double a, double b, double *e) { return two_sum(a, b, e); }
float oracle_two_sum_f(float a, float b, float *e) { return two_sum_f(a, b, e); }
double oracle_two_prod(double a, double b, double *e) { return two_prod(a, b, e); }

/*
 * Renormalization of an n-term expansion, in place (n <= 80).
 *   1. bottom-up pass: s = x[n-1]; for i = n-2 .. 0: (s, e[i+1]) = TwoSum(x[i], s).
 *   2. top-down pass over (s, e[1], .., e[n-1]): t = s; for i = 1 .. n-1:
 *      (t, err) = TwoSum(t, e[i]); if err != 0 emit t and continue with t = err.
 *      Finally emit t and pad with zeros.
 * Only TwoSum is used, so the sum of the terms is unchanged exactly; the first
 * output is nonzero whenever the sum is nonzero.
 */
static void renorm(double *x, int n)
{
    double e[80];
    double s = x[n - 1];
    for (int i = n - 2; i >= 0; --i)
        s = two_sum(x[i], s, &e[i + 1]);
    double t = s;
    int w = 0;
    for (int i = 1; i < n; ++i) {
        double err;
        t = two_sum(t, e[i], &err);
        if (err != 0.0) {
            x[w++] = t;
            t = err;
        }
    }
    x[w++] = t;
    while (w < n)
        x[w++] = 0.0;
}

static void renorm_f(float *x, int n)
{
    float e[80];
    float s = x[n - 1];
    for (int i = n - 2; i >= 0; --i)
        s = two_sum_f(x[i], s, &e[i + 1]);
    float t = s;
    int w = 0;
    for (int i = 1; i < n; ++i) {
        float err;
        t = two_sum_f(t, e[i], &err);
        if (err != 0.0f) {
            x[w++] = t;
            t = err;
        }
    }
    x[w++] = t;
    while (w < n)
        x[w++] = 0.0f;
}

void oracle_renorm(double *x, int n) { renorm(x, n); }
void oracle_renorm_f(float *x, int n) { renorm_f(x, n); }

/* ------------------------------------------------------------------------- */
/* Split constants (Algorithm 1).                                             */
/* ------------------------------------------------------------------------- */

/* ceil(log2 k) for k >= 1. */
static int ceil_log2_int(long k)
{
    int r = 0;
    while ((1L << r) < k)
        ++r;
    return r;
}

/* The shift ceil((S + log2 l) / 2) of tau in Algorithm 1, for l = k >= 1. */
int oracle_rho(int S, long k)
{
    if (k < 1)
        return 0;
    return (S + ceil_log2_int(k) + 1) / 2;
}

/* ceil(log2 mu) for finite mu > 0. */
static int ceil_log2_pos(double mu)
{
    int e = ilogb(mu);
    if (ldexp(1.0, e) != mu)
        e += 1;
    return e;
}

/* ------------------------------------------------------------------------- */
/* Plain split: Algorithm 1 with binary64 slices (S = 53) or binary32 (S = 24)*/
/* ------------------------------------------------------------------------- */

/*
 * Split `nvec` vectors of `len` c-component elements.  Element p of vector v,
 * component r, is X[r*s_comp + v*s_vec + p*s_elt] (rows of A: s_vec = 1,
 * s_elt = m; columns of B: s_vec = k, s_elt = 1).
 * Outputs (same element strides): slice a at slices[a*nvec*len + ...],
 * exponent ceil(log2 mu_a) of vector v at exps[a*nvec + v] (ZERO_EXP if
 * mu_a = 0), and optionally the final residual (c components) at
 * resid[r*nvec*len + ...] when resid != NULL.
 *
 * last_remainder = 0: all D slices are extracted on the grid of tau and the
 * remainder is dropped, so every slice product is exact (the reading this
 * library uses).  last_remainder = 1: Algorithm 1 as printed, where the last
 * slice is the leading component of the residual left by the first D - 1
 * passes (A_D := A^(S)); its exponent entry is still ceil(log2 mu_D).
 */
int oracle_split_plain(int nvec, int len, int c, const double *X, long s_vec, long s_elt, long s_comp,
                       int D, int rho, int last_remainder, double *slices, int *exps, double *resid)
{
    if (nvec < 0 || len < 0 || c < 1 || c > 8 || D < 1)
        return ORC_EINVAL;
    const long plane = (long)nvec * len;
    int status = ORC_OK;
#pragma omp parallel for schedule(dynamic, 4)
    for (int v = 0; v < nvec; ++v) {
        double *R = malloc(sizeof(double) * (size_t)(len > 0 ? len : 1) * c);
        if (!R) {
            status = ORC_ENOMEM;
            continue;
        }
        for (int p = 0; p < len; ++p)
            for (int r = 0; r < c; ++r)
                R[(long)p * c + r] = X[r * s_comp + v * s_vec + p * s_elt];
        for (int a = 0; a < D; ++a) {
            double mu = 0.0;
            for (int p = 0; p < len; ++p)
                mu = fmax(mu, fabs(R[(long)p * c]));
            double *out = slices + a * plane + v * s_vec;
            if (mu == 0.0) {
                exps[a * nvec + v] = ZERO_EXP;
                for (int p = 0; p < len; ++p)
                    out[p * s_elt] = 0.0;
                continue;
            }
            int e = ceil_log2_pos(mu);
            exps[a * nvec + v] = e;
            double tau = ldexp(1.0, e + rho);
            const int literal = last_remainder && a == D - 1;
            for (int p = 0; p < len; ++p) {
                double lead = R[(long)p * c];
                double sl = literal ? lead : (lead + tau) - tau;
                out[p * s_elt] = sl;
                R[(long)p * c] = lead - sl; /* exact */
                renorm(&R[(long)p * c], c);
            }
        }
        if (resid)
            for (int p = 0; p < len; ++p)
                for (int r = 0; r < c; ++r)
                    resid[r * plane + v * s_vec + p * s_elt] = R[(long)p * c + r];
        free(R);
    }
    return status;
}

int oracle_split_plain_f(int nvec, int len, int c, const float *X, long s_vec, long s_elt, long s_comp,
                         int D, int rho, int last_remainder, float *slices, int *exps, float *resid)
{
    if (nvec < 0 || len < 0 || c < 1 || c > 8 || D < 1)
        return ORC_EINVAL;
    const long plane = (long)nvec * len;
    int status = ORC_OK;
#pragma omp parallel for schedule(dynamic, 4)
    for (int v = 0; v < nvec; ++v) {
        float *R = malloc(sizeof(float) * (size_t)(len > 0 ? len : 1) * c);
        if (!R) {
            status = ORC_ENOMEM;
            continue;
        }
        for (int p = 0; p < len; ++p)
            for (int r = 0; r < c; ++r)
                R[(long)p * c + r] = X[r * s_comp + v * s_vec + p * s_elt];
        for (int a = 0; a < D; ++a) {
            float mu = 0.0f;
            for (int p = 0; p < len; ++p)
                mu = fmaxf(mu, fabsf(R[(long)p * c]));
            float *out = slices + a * plane + v * s_vec;
            if (mu == 0.0f) {
                exps[a * nvec + v] = ZERO_EXP;
                for (int p = 0; p < len; ++p)
                    out[p * s_elt] = 0.0f;
                continue;
            }
            int e = ceil_log2_pos((double)mu);
            exps[a * nvec + v] = e;
            float tau = ldexpf(1.0f, e + rho);
            const int literal = last_remainder && a == D - 1;
            for (int p = 0; p < len; ++p) {
                float lead = R[(long)p * c];
                float sl = literal ? lead : (lead + tau) - tau;
                out[p * s_elt] = sl;
                R[(long)p * c] = lead - sl;
                renorm_f(&R[(long)p * c], c);
            }
        }
        if (resid)
            for (int p = 0; p < len; ++p)
                for (int r = 0; r < c; ++r)
                    resid[r * plane + v * s_vec + p * s_elt] = R[(long)p * c + r];
        free(R);
    }
    return status;
}

/* ------------------------------------------------------------------------- */
/* Exact slice products C_ab = A_a B_b.                                       */
/* ------------------------------------------------------------------------- */

/*
 * Slice entry x of a vector with exponent e lies on the grid 2^(e + rho - S)
 * with |x| <= 2^e (the extraction lemma); its integer on that grid is found
 * with ldexp and checked.  Returns 0 and sets *q on success.
 */
static int slice_to_int(double x, int e, int rho, int S, int64_t *q)
{
    *q = 0;
    if (x == 0.0)
        return 1;
    if (e == ZERO_EXP)
        return 0;
    double y = ldexp(x, -(e + rho - S));
    if (y != nearbyint(y) || fabs(y) > ldexp(1.0, S - rho))
        return 0;
    *q = (int64_t)y;
    return 1;
}

/*
 * Cab (n x m column-major: Cab[i + j*m]) = Aa (k x m col-major, exponents ea[m])
 * times Bb (n x k col-major, exponents eb[n]), by exact int64 dot products on
 * the slice grids.  S = 53 for binary64 slices, 24 for binary32 (then the
 * result is also exact as a binary32 value; it is stored as binary64 here).
 */
int oracle_slice_product(int m, int n, int k, const double *Aa, const int *ea, const double *Bb, const int *eb,
                         int rho, int S, double *Cab)
{
    int status = ORC_OK;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i < m; ++i) {
            int64_t acc = 0;
            int ok = 1;
            for (int p = 0; p < k; ++p) {
                int64_t qa, qb;
                ok &= slice_to_int(Aa[i + (long)p * m], ea[i], rho, S, &qa);
                ok &= slice_to_int(Bb[p + (long)j * k], eb[j], rho, S, &qb);
                acc += qa * qb;
            }
            if (!ok || llabs(acc) > (1LL << S)) {
                status = ORC_ENOTEXACT;
                Cab[i + (long)j * m] = NAN;
                continue;
            }
            Cab[i + (long)j * m] =
                (acc == 0 || ea[i] == ZERO_EXP || eb[j] == ZERO_EXP) ? 0.0
                                                                    : ldexp((double)acc, ea[i] + eb[j] + 2 * (rho - S));
        }
    }
    return status;
}

/* ------------------------------------------------------------------------- */
/* Long fixed-point accumulator (exact sums of binary64 values and products). */
/* ------------------------------------------------------------------------- */

/*
 * value = sum_i d[i] * 2^(32 i - BIAS).  Deposits add at most 32 bits per
 * limb, so limbs hold a long run of deposits before carries are propagated.
 * Bit positions from 2^-2304 upward cover every product of two finite binary64
 * values (subnormal mantissas included) and sums of up to 2^40 of them.
 */
#define SA_NL 140
#define SA_BIAS 2304

typedef struct {
    int64_t d[SA_NL];
    long ndep;
} sacc;

static void sa_clear(sacc *s) { memset(s, 0, sizeof *s); }

static void sa_norm(sacc *s)
{
    for (int i = 0; i < SA_NL - 1; ++i) {
        int64_t low = s->d[i] & 0xffffffffLL;
        int64_t carry = (s->d[i] - low) / 4294967296LL;
        s->d[i] = low;
        s->d[i + 1] += carry;
    }
    s->ndep = 0;
}

/* add sign * u * 2^q, u < 2^64 */
static void sa_dep_u64(sacc *s, int neg, uint64_t u, int q)
{
    if (u == 0)
        return;
    int pos = q + SA_BIAS;
    int idx = pos >> 5, sh = pos & 31;
    unsigned __int128 v = (unsigned __int128)u << sh;
    for (int t = 0; t < 3; ++t) {
        int64_t chunk = (int64_t)(uint64_t)(v & 0xffffffffu);
        s->d[idx + t] += neg ? -chunk : chunk;
        v >>= 32;
    }
    if (++s->ndep > (1L << 28))
        sa_norm(s);
}

/* x = mant * 2^q with |mant| < 2^53 */
static void split_double(double x, int64_t *mant, int *q)
{
    int ex;
    double f = frexp(x, &ex);
    *mant = (int64_t)ldexp(f, 53);
    *q = ex - 53;
}

static void sa_add(sacc *s, double x)
{
    if (x == 0.0)
        return;
    int64_t m;
    int q;
    split_double(x, &m, &q);
    sa_dep_u64(s, m < 0, (uint64_t)llabs(m), q);
}

static void sa_add_prod(sacc *s, double a, double b)
{
    if (a == 0.0 || b == 0.0)
        return;
    int64_t ma, mb;
    int qa, qb;
    split_double(a, &ma, &qa);
    split_double(b, &mb, &qb);
    int neg = (ma < 0) != (mb < 0);
    unsigned __int128 P = (unsigned __int128)(uint64_t)llabs(ma) * (uint64_t)llabs(mb);
    sa_dep_u64(s, neg, (uint64_t)P, qa + qb);
    sa_dep_u64(s, neg, (uint64_t)(P >> 64), qa + qb + 64);
}

/* After sa_norm: sign of the value (-1, 0, 1). */
static int sa_sign(const sacc *s)
{
    if (s->d[SA_NL - 1] < 0)
        return -1;
    for (int i = SA_NL - 1; i >= 0; --i)
        if (s->d[i] != 0)
            return 1;
    return 0;
}

/* |value| as normalized nonnegative limbs (input must be normalized). */
static void sa_abs(const sacc *s, sacc *out)
{
    *out = *s;
    if (s->d[SA_NL - 1] < 0) {
        for (int i = 0; i < SA_NL; ++i)
            out->d[i] = -out->d[i];
        sa_norm(out);
    }
}

/* bit b (as exponent, value bit 2^b) of a nonnegative normalized magnitude */
static int sa_bit(const sacc *mag, int b)
{
    int pos = b + SA_BIAS;
    if (pos < 0 || pos >= 32 * SA_NL)
        return 0;
    return (int)((mag->d[pos >> 5] >> (pos & 31)) & 1);
}

/* exponent of the leading 1 bit of a nonnegative normalized magnitude, or INT_MIN */
static int sa_lead(const sacc *mag)
{
    for (int i = SA_NL - 1; i >= 0; --i)
        if (mag->d[i] != 0) {
            int b = 31;
            while (!((mag->d[i] >> b) & 1))
                --b;
            return 32 * i + b - SA_BIAS;
        }
    return INT_MIN;
}

/* any bit strictly below exponent b set? */
static int sa_sticky_below(const sacc *mag, int b)
{
    int pos = b + SA_BIAS;
    if (pos <= 0)
        return 0;
    int idx = pos >> 5, sh = pos & 31;
    for (int i = 0; i < idx && i < SA_NL; ++i)
        if (mag->d[i] != 0)
            return 1;
    if (idx < SA_NL && sh > 0 && (mag->d[idx] & ((1LL << sh) - 1)) != 0)
        return 1;
    return 0;
}

/*
 * Round the (normalized) value to the nearest binary floating-point number with
 * p significand bits and minimum exponent emin (binary64: p = 53, emin = -1074;
 * binary32: p = 24, emin = -149), ties to even.  Overflow is not handled (the
 * oracle's inputs are bounded far below it).
 */
static double sa_round(const sacc *s, int p, int emin)
{
    int sg = sa_sign(s);
    if (sg == 0)
        return 0.0;
    sacc mag;
    sa_abs(s, &mag);
    int lead = sa_lead(&mag);
    int lsb = lead - (p - 1);
    if (lsb < emin)
        lsb = emin;
    uint64_t m = 0;
    for (int b = lead; b >= lsb; --b)
        m = (m << 1) | (uint64_t)sa_bit(&mag, b);
    int rbit = sa_bit(&mag, lsb - 1);
    int sticky = sa_sticky_below(&mag, lsb - 1);
    if (rbit && (sticky || (m & 1)))
        m += 1;
    double r = ldexp((double)m, lsb);
    return sg < 0 ? -r : r;
}

/* Greedy expansion: x_r = RN(v - x_0 - .. - x_{r-1}); the accumulator is consumed. */
static void sa_to_expansion(sacc *s, double *x, int c, int p, int emin)
{
    for (int r = 0; r < c; ++r) {
        sa_norm(s);
        x[r] = sa_round(s, p, emin);
        sa_add(s, -x[r]);
    }
}

/* ------------------------------------------------------------------------- */
/* Exact product, bound check and the paper's relative error.                 */
/* ------------------------------------------------------------------------- */

/*
 * For the listed rows of C = A B (all rows if rows == NULL, nrows = m):
 *   diff[u*n*nrows + t + j*nrows] = RN(|C_u - A B|) for each of the nc
 *                       matrices under test (exact difference, rounded once),
 *   absab[...]        = sum_p |a_ip0| |b_pj0| in binary64 (leading components;
 *                       relative error below (k + 2) 2^-52 of sum |a||b|),
 *   cex[...]          = RN(A B), the exact product rounded once.
 * A: c planes of k x m (col-major), B: c planes of n x k, each C_u (Cs[u]): c
 * planes of n x ldc.  is_f32 selects binary32 component arrays.  The exact
 * product is formed once per entry and compared with every C_u.
 */
int oracle_gemm_exact_check_many(int c, int is_f32, int m, int n, int k, const void *Av, const void *Bv, int nc,
                                 const void *const *Cs, int ldc, const int *rows, int nrows, double *diff,
                                 double *absab, double *cex)
{
    if (c < 1 || c > ORC_MAXC || m < 0 || n < 0 || k < 0 || nc < 0 || (nc > 0 && (!Cs || !diff)))
        return ORC_EINVAL;
    const long pa = (long)m * k, pb = (long)k * n, pc = (long)ldc * n;
    int status = ORC_OK;
#pragma omp parallel
    {
        sacc *s = malloc(sizeof(sacc));
        sacc *w = malloc(sizeof(sacc));
        if (!s || !w)
            status = ORC_ENOMEM;
#pragma omp for schedule(dynamic, 1) collapse(2)
        for (int t = 0; t < nrows; ++t) {
            for (int j = 0; j < n; ++j) {
                if (!s || !w)
                    continue;
                int i = rows ? rows[t] : t;
                sa_clear(s);
                double ab = 0.0;
                for (int p = 0; p < k; ++p) {
                    for (int ra = 0; ra < c; ++ra) {
                        double a = is_f32 ? (double)((const float *)Av)[ra * pa + i + (long)p * m]
                                          : ((const double *)Av)[ra * pa + i + (long)p * m];
                        if (a == 0.0)
                            continue;
                        for (int rb = 0; rb < c; ++rb) {
                            double b = is_f32 ? (double)((const float *)Bv)[rb * pb + p + (long)j * k]
                                              : ((const double *)Bv)[rb * pb + p + (long)j * k];
                            sa_add_prod(s, a, b);
                        }
                    }
                    double a0 = is_f32 ? (double)((const float *)Av)[i + (long)p * m]
                                       : ((const double *)Av)[i + (long)p * m];
                    double b0 = is_f32 ? (double)((const float *)Bv)[p + (long)j * k]
                                       : ((const double *)Bv)[p + (long)j * k];
                    ab += fabs(a0) * fabs(b0);
                }
                sa_norm(s);
                if (cex)
                    cex[t + (long)j * nrows] = sa_round(s, 53, -1074);
                for (int u = 0; u < nc; ++u) {
                    const void *Cv = Cs[u];
                    *w = *s;
                    for (int r = 0; r < c; ++r) {
                        double cv = is_f32 ? (double)((const float *)Cv)[r * pc + i + (long)j * ldc]
                                           : ((const double *)Cv)[r * pc + i + (long)j * ldc];
                        sa_add(w, -cv);
                    }
                    sa_norm(w);
                    diff[(long)u * n * nrows + t + (long)j * nrows] = fabs(sa_round(w, 53, -1074));
                }
                if (absab)
                    absab[t + (long)j * nrows] = ab;
            }
        }
        free(s);
        free(w);
    }
    return status;
}

/* The single-matrix form: diff (if not NULL) for C_test = Cv. */
int oracle_gemm_exact_check(int c, int is_f32, int m, int n, int k, const void *Av, const void *Bv, const void *Cv,
                            int ldc, const int *rows, int nrows, double *diff, double *absab, double *cex)
{
    const void *cs[1] = {Cv};
    return oracle_gemm_exact_check_many(c, is_f32, m, n, k, Av, Bv, diff ? 1 : 0, cs, ldc, rows, nrows, diff, absab,
                                        cex);
}

/* Exact sum of a list of binary64 values, returned as a c-term greedy expansion. */
int oracle_exact_sum(const double *x, long nx, int c, int is_f32, double *out)
{
    sacc *s = malloc(sizeof(sacc));
    if (!s)
        return ORC_ENOMEM;
    sa_clear(s);
    for (long t = 0; t < nx; ++t)
        sa_add(s, x[t]);
    sa_to_expansion(s, out, c, is_f32 ? 24 : 53, is_f32 ? -149 : -1074);
    free(s);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Ozaki GEMM (Algorithm 1) in the oracle's arithmetic.                       */
/* ------------------------------------------------------------------------- */

/* One L-bit addition: out = expansion of (x + y), both c-term, rounded to c
 * terms (the exact sum, then greedy nearest rounding). */
static void lbit_add(sacc *s, const double *x, const double *y, int c, int p, int emin, double *out)
{
    sa_clear(s);
    for (int r = 0; r < c; ++r) {
        sa_add(s, x[r]);
        sa_add(s, y[r]);
    }
    sa_to_expansion(s, out, c, p, emin);
}

/*
 * C = Ozaki product of A (c planes, k x m) and B (c planes, n x k) with D
 * slices, for the listed rows of C (all if rows == NULL; row t of the outputs
 * is row rows[t] of C).  Follows Algorithm 1 with the readings in the file
 * header.  Outputs (nrows x n column-major planes, c of them):
 *   C_tri:   the exact sum over the triangle a + b <= D + 1 of the exact slice
 *            products, rounded once to a c-term expansion;
 *   C_paper: (nullable) the same terms accumulated as Algorithm 1 writes it:
 *            for a = 1..D: T = sum_b C_ab in L-bit, then C := C + T in L-bit,
 *            each L-bit addition rounding the exact sum to c terms.
 * is_f32 selects binary32 components and slices (S = 24), else S = 53.
 */
int oracle_ozaki_gemm(int c, int is_f32, int m, int n, int k, const void *Av, const void *Bv, int D,
                      const int *rows, int nrows, double *C_tri, double *C_paper)
{
    if (c < 1 || c > 8 || D < 1 || m < 0 || n < 0 || k < 0)
        return ORC_EINVAL;
    const int S = is_f32 ? 24 : 53;
    const int prec = S, emin = is_f32 ? -149 : -1074;
    const int rho = oracle_rho(S, k);
    int status = ORC_OK;

    /* Gather the requested rows of A into a compact (c, k, nrows) block. */
    double *Ar = malloc(sizeof(double) * (size_t)c * k * (nrows > 0 ? nrows : 1));
    double *Bd = malloc(sizeof(double) * (size_t)c * k * (n > 0 ? n : 1));
    double *As = malloc(sizeof(double) * (size_t)D * k * (nrows > 0 ? nrows : 1));
    double *Bs = malloc(sizeof(double) * (size_t)D * k * (n > 0 ? n : 1));
    int *ea = malloc(sizeof(int) * (size_t)D * (nrows > 0 ? nrows : 1));
    int *eb = malloc(sizeof(int) * (size_t)D * (n > 0 ? n : 1));
    if (!Ar || !Bd || !As || !Bs || !ea || !eb) {
        status = ORC_ENOMEM;
        goto done;
    }
    for (int r = 0; r < c; ++r)
        for (int p = 0; p < k; ++p) {
            for (int t = 0; t < nrows; ++t) {
                int i = rows ? rows[t] : t;
                long src = (long)r * m * k + i + (long)p * m;
                Ar[(long)r * nrows * k + t + (long)p * nrows] =
                    is_f32 ? (double)((const float *)Av)[src] : ((const double *)Av)[src];
            }
            for (int j = 0; j < n; ++j) {
                long src = (long)r * k * n + p + (long)j * k;
                Bd[src] = is_f32 ? (double)((const float *)Bv)[src] : ((const double *)Bv)[src];
            }
        }

    if (is_f32) {
        /* binary32 split on binary32 copies, widened back for the products */
        float *Af = malloc(sizeof(float) * (size_t)c * k * (nrows > 0 ? nrows : 1));
        float *Bf = malloc(sizeof(float) * (size_t)c * k * (n > 0 ? n : 1));
        float *Asf = malloc(sizeof(float) * (size_t)D * k * (nrows > 0 ? nrows : 1));
        float *Bsf = malloc(sizeof(float) * (size_t)D * k * (n > 0 ? n : 1));
        if (!Af || !Bf || !Asf || !Bsf) {
            free(Af), free(Bf), free(Asf), free(Bsf);
            status = ORC_ENOMEM;
            goto done;
        }
        for (long t = 0; t < (long)c * k * nrows; ++t)
            Af[t] = (float)Ar[t];
        for (long t = 0; t < (long)c * k * n; ++t)
            Bf[t] = (float)Bd[t];
        status = oracle_split_plain_f(nrows, k, c, Af, 1, nrows, (long)nrows * k, D, rho, 0, Asf, ea, NULL);
        if (status == ORC_OK)
            status = oracle_split_plain_f(n, k, c, Bf, k, 1, (long)k * n, D, rho, 0, Bsf, eb, NULL);
        for (long t = 0; t < (long)D * k * nrows; ++t)
            As[t] = Asf[t];
        for (long t = 0; t < (long)D * k * n; ++t)
            Bs[t] = Bsf[t];
        free(Af), free(Bf), free(Asf), free(Bsf);
    } else {
        status = oracle_split_plain(nrows, k, c, Ar, 1, nrows, (long)nrows * k, D, rho, 0, As, ea, NULL);
        if (status == ORC_OK)
            status = oracle_split_plain(n, k, c, Bd, k, 1, (long)k * n, D, rho, 0, Bs, eb, NULL);
    }
    if (status != ORC_OK)
        goto done;

    /* Slice products of the triangle a + b <= D + 1, then accumulation. */
    const long plane = (long)nrows * n;
#pragma omp parallel
    {
        sacc *s = malloc(sizeof(sacc));
        double *prod = malloc(sizeof(double) * (size_t)D * D);
        if (!s || !prod)
            status = ORC_ENOMEM;
#pragma omp for schedule(dynamic, 1) collapse(2)
        for (int j = 0; j < n; ++j) {
            for (int t = 0; t < nrows; ++t) {
                if (!s || !prod)
                    continue;
                /* C_ab(t, j) for a + b <= D + 1 (0-based: a + b <= D - 1) */
                for (int a = 0; a < D; ++a) {
                    for (int b = 0; a + b <= D - 1; ++b) {
                        int e1 = ea[a * nrows + t], e2 = eb[b * n + j];
                        int64_t acc = 0;
                        int ok = 1;
                        for (int p = 0; p < k; ++p) {
                            int64_t qa, qb;
                            ok &= slice_to_int(As[(long)a * nrows * k + t + (long)p * nrows], e1, rho, S, &qa);
                            ok &= slice_to_int(Bs[(long)b * k * n + p + (long)j * k], e2, rho, S, &qb);
                            acc += qa * qb;
                        }
                        if (!ok || llabs(acc) > (1LL << S))
                            status = ORC_ENOTEXACT;
                        prod[a * D + b] = (acc == 0) ? 0.0 : ldexp((double)acc, e1 + e2 + 2 * (rho - S));
                    }
                }
                double out[8];
                sa_clear(s);
                for (int a = 0; a < D; ++a)
                    for (int b = 0; a + b <= D - 1; ++b)
                        sa_add(s, prod[a * D + b]);
                sa_to_expansion(s, out, c, prec, emin);
                for (int r = 0; r < c; ++r)
                    C_tri[r * plane + t + (long)j * nrows] = out[r];
                if (C_paper) {
                    double Cacc[8] = {0}, T[8], term[8], tmp[8];
                    for (int a = 0; a < D; ++a) {
                        for (int r = 0; r < c; ++r)
                            T[r] = 0.0;
                        for (int b = 0; a + b <= D - 1; ++b) {
                            term[0] = prod[a * D + b];
                            for (int r = 1; r < c; ++r)
                                term[r] = 0.0;
                            lbit_add(s, T, term, c, prec, emin, tmp);
                            memcpy(T, tmp, sizeof(double) * c);
                        }
                        lbit_add(s, Cacc, T, c, prec, emin, tmp);
                        memcpy(Cacc, tmp, sizeof(double) * c);
                    }
                    for (int r = 0; r < c; ++r)
                        C_paper[r * plane + t + (long)j * nrows] = Cacc[r];
                }
            }
        }
        free(s);
        free(prod);
    }
done:
    free(Ar), free(Bd), free(As), free(Bs), free(ea), free(eb);
    return status;
}

/* ------------------------------------------------------------------------- */
/* INT8 slices (the precision form; not in the paper).                        */
/* ------------------------------------------------------------------------- */

/*
 * RNE(R / 2^e) for the normalized accumulator R with |R| <= 64.5 * 2^e: the
 * nearest integer, ties to even (symmetric in the sign).
 */
static int rne_quotient(const sacc *R, int e)
{
    int sg = sa_sign(R);
    if (sg == 0)
        return 0;
    sacc mag;
    sa_abs(R, &mag);
    int q = 0;
    for (int b = e + 7; b >= e; --b)
        q = 2 * q + sa_bit(&mag, b);
    if (sa_bit(&mag, e - 1) && (sa_sticky_below(&mag, e - 1) || (q & 1)))
        q += 1;
    return sg < 0 ? -q : q;
}

/*
 * Split `nvec` vectors (strides as in oracle_split_plain) into D int8 digit
 * planes.  E_v = 1 + max_p ilogb(x_p0) over nonzero leading components
 * (ZERO_EXP if none), so |x| < 2^E_v for a normalized expansion.  Digit s
 * (s = 1..D) uses the unit u_s = 2^(E_v - 6 - 7 (s - 1)) and is the
 * extraction step of Algorithm 1 on that fixed grid applied to the exact
 * residual: with R the exact value of the element (the sum of its components)
 * at s = 1, d_s = RN(R / u_s) (nearest, ties to even) and R := R - d_s u_s.
 * Hence sum_{t <= s} d_t u_t = RN(x / u_s) u_s for every s, |d_s| <= 64 and
 * the remainder after D digits is at most u_D / 2.  The residual is held
 * exactly in the long accumulator.  Returns ORC_ENOTEXACT if a digit falls
 * outside [-64, 64] (an input that is not a normalized expansion).
 */
int oracle_split_int8(int nvec, int len, int c, const double *X, long s_vec, long s_elt, long s_comp, int D,
                      int8_t *digits, int *exps)
{
    if (nvec < 0 || len < 0 || c < 1 || c > ORC_MAXC || D < 1)
        return ORC_EINVAL;
    const long plane = (long)nvec * len;
    int status = ORC_OK;
#pragma omp parallel for schedule(dynamic, 4)
    for (int v = 0; v < nvec; ++v) {
        int E = ZERO_EXP;
        for (int p = 0; p < len; ++p) {
            double x0 = X[v * s_vec + p * s_elt];
            if (x0 != 0.0 && ilogb(x0) + 1 > E)
                E = ilogb(x0) + 1;
        }
        exps[v] = E;
        sacc R;
        for (int p = 0; p < len; ++p) {
            int8_t *dst = digits + v * s_vec + p * s_elt;
            sa_clear(&R);
            for (int r = 0; r < c; ++r)
                sa_add(&R, X[r * s_comp + v * s_vec + p * s_elt]);
            for (int d = 1; d <= D; ++d) {
                int val = 0;
                if (E != ZERO_EXP) {
                    const int ue = E - 6 - 7 * (d - 1);
                    sa_norm(&R);
                    val = rne_quotient(&R, ue);
                    if (val < -64 || val > 64) {
#pragma omp atomic write
                        status = ORC_ENOTEXACT;
                        val = 0;
                    }
                    sa_dep_u64(&R, val > 0, (uint64_t)(val < 0 ? -val : val), ue); /* R -= val u_s, exact */
                }
                dst[(d - 1) * plane] = (int8_t)val;
            }
        }
    }
    return status;
}

/*
 * Diagonal sums of INT8 digit products: for g = 1..D,
 *   S_g = sum over s + t = g + 1 of A_s B_t  (exact, int64),
 * A digits (D planes of k x m), B digits (D planes of n x k); output
 * Sg[(g-1)*m*n + i + j*m].
 */
int oracle_int8_diag_sums(int m, int n, int k, int D, const int8_t *Ad, const int8_t *Bd, int64_t *Sg)
{
    const long pa = (long)m * k, pb = (long)k * n, pc = (long)m * n;
#pragma omp parallel for schedule(static) collapse(2)
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < m; ++i)
            for (int g = 1; g <= D; ++g) {
                int64_t acc = 0;
                for (int s = 1; s <= g; ++s) {
                    int t = g + 1 - s;
                    const int8_t *a = Ad + (s - 1) * pa + i;
                    const int8_t *b = Bd + (t - 1) * pb + (long)j * k;
                    for (int p = 0; p < k; ++p)
                        acc += (int64_t)a[(long)p * m] * (int64_t)b[p];
                }
                Sg[(g - 1) * pc + i + (long)j * m] = acc;
            }
    return ORC_OK;
}

/*
 * INT8-form result: digit s of A's row i has unit 2^(E_i - 6 - 7 (s - 1)) and
 * digit t of B's column j 2^(F_j - 6 - 7 (t - 1)), so every product on the
 * diagonal s + t = g + 1 has unit 2^(E_i + F_j + 2 - 7 (g + 1)):
 * C = sum_g S_g 2^(E_i + F_j + 2 - 7 (g + 1)), summed exactly and rounded once
 * to a c-term binary64 expansion (planes of m x n).
 */
int oracle_int8_combine(int m, int n, int D, int c, const int64_t *Sg, const int *EA, const int *EB, double *C)
{
    if (c < 1 || c > ORC_MAXC || m < 0 || n < 0 || D < 1)
        return ORC_EINVAL;
    const long pc = (long)m * n;
    int status = ORC_OK;
#pragma omp parallel
    {
        sacc *s = malloc(sizeof(sacc));
        if (!s)
            status = ORC_ENOMEM;
#pragma omp for schedule(static) collapse(2)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < m; ++i) {
                if (!s)
                    continue;
                sa_clear(s);
                if (EA[i] != ZERO_EXP && EB[j] != ZERO_EXP)
                    for (int g = 1; g <= D; ++g) {
                        int64_t v = Sg[(g - 1) * pc + i + (long)j * m];
                        if (v != 0)
                            sa_dep_u64(s, v < 0, (uint64_t)llabs(v), EA[i] + EB[j] + 2 - 7 * (g + 1));
                    }
                double out[ORC_MAXC];
                sa_to_expansion(s, out, c, 53, -1074);
                for (int r = 0; r < c; ++r)
                    C[r * pc + i + (long)j * m] = out[r];
            }
        free(s);
    }
    return status;
}

/* ------------------------------------------------------------------------- */
/* The paper's "simple matrix multiplication" (Section 4.1): a triple loop in */
/* multi-component arithmetic written from the published error-free methods.  */
/* ------------------------------------------------------------------------- */

/*
 * c-term product a*b: the products a_r b_s with r + s < c, the low halves of
 * those with r + s < c - 1 kept exactly by TwoProd, gathered and renormalized;
 * terms of order c and beyond are dropped (the usual truncated multi-component
 * multiplication).  c-term sum acc + y: all 2c terms are ordered by decreasing
 * magnitude and renormalized, keeping c terms.
 */
static void sort_desc(double *t, int n)
{
    for (int i = 1; i < n; ++i) {
        double v = t[i];
        int j = i - 1;
        while (j >= 0 && fabs(t[j]) < fabs(v)) {
            t[j + 1] = t[j];
            --j;
        }
        t[j + 1] = v;
    }
}

static void mc_mul(const double *a, const double *b, int c, double *out)
{
    double t[80];
    int n = 0;
    for (int r = 0; r < c; ++r)
        for (int s = 0; r + s < c; ++s) {
            double e;
            double p = two_prod(a[r], b[s], &e);
            t[n++] = p;
            if (r + s < c - 1)
                t[n++] = e;
        }
    sort_desc(t, n);
    renorm(t, n);
    for (int r = 0; r < c; ++r)
        out[r] = t[r];
}

static void mc_add(double *acc, const double *y, int c)
{
    double t[16];
    for (int r = 0; r < c; ++r) {
        t[r] = acc[r];
        t[c + r] = y[r];
    }
    sort_desc(t, 2 * c);
    renorm(t, 2 * c);
    for (int r = 0; r < c; ++r)
        acc[r] = t[r];
}

static void mc_mul_f(const float *a, const float *b, int c, float *out)
{
    float t[80];
    int n = 0;
    for (int r = 0; r < c; ++r)
        for (int s = 0; r + s < c; ++s) {
            float p = a[r] * b[s];
            t[n++] = p;
            if (r + s < c - 1)
                t[n++] = fmaf(a[r], b[s], -p);
        }
    for (int i = 1; i < n; ++i) {
        float v = t[i];
        int j = i - 1;
        while (j >= 0 && fabsf(t[j]) < fabsf(v)) {
            t[j + 1] = t[j];
            --j;
        }
        t[j + 1] = v;
    }
    renorm_f(t, n);
    for (int r = 0; r < c; ++r)
        out[r] = t[r];
}

static void mc_add_f(float *acc, const float *y, int c)
{
    float t[16];
    for (int r = 0; r < c; ++r) {
        t[r] = acc[r];
        t[c + r] = y[r];
    }
    for (int i = 1; i < 2 * c; ++i) {
        float v = t[i];
        int j = i - 1;
        while (j >= 0 && fabsf(t[j]) < fabsf(v)) {
            t[j + 1] = t[j];
            --j;
        }
        t[j + 1] = v;
    }
    renorm_f(t, 2 * c);
    for (int r = 0; r < c; ++r)
        acc[r] = t[r];
}

/* C (c planes, nrows x n) = A B for the listed rows, by the naive triple loop. */
int oracle_gemm_naive(int c, int is_f32, int m, int n, int k, const void *Av, const void *Bv, const int *rows,
                      int nrows, void *Cv)
{
    if (c < 1 || c > 4 || m < 0 || n < 0 || k < 0)
        return ORC_EINVAL;
    const long pa = (long)m * k, pb = (long)k * n, pc = (long)nrows * n;
#pragma omp parallel for schedule(static) collapse(2)
    for (int j = 0; j < n; ++j)
        for (int t = 0; t < nrows; ++t) {
            int i = rows ? rows[t] : t;
            if (is_f32) {
                const float *A = Av, *B = Bv;
                float acc[8] = {0}, a[8], b[8], pr[8];
                for (int p = 0; p < k; ++p) {
                    for (int r = 0; r < c; ++r) {
                        a[r] = A[r * pa + i + (long)p * m];
                        b[r] = B[r * pb + p + (long)j * k];
                    }
                    mc_mul_f(a, b, c, pr);
                    mc_add_f(acc, pr, c);
                }
                for (int r = 0; r < c; ++r)
                    ((float *)Cv)[r * pc + t + (long)j * nrows] = acc[r];
            } else {
                const double *A = Av, *B = Bv;
                double acc[8] = {0}, a[8], b[8], pr[8];
                for (int p = 0; p < k; ++p) {
                    for (int r = 0; r < c; ++r) {
                        a[r] = A[r * pa + i + (long)p * m];
                        b[r] = B[r * pb + p + (long)j * k];
                    }
                    mc_mul(a, b, c, pr);
                    mc_add(acc, pr, c);
                }
                for (int r = 0; r < c; ++r)
                    ((double *)Cv)[r * pc + t + (long)j * nrows] = acc[r];
            }
        }
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* D+S (a binary64 leading part and a binary32 trailing part; Section 4.4's   */
/* GPU comparison of D+S, DD and TS simple matrix multiplication).            */
/* ------------------------------------------------------------------------- */

/*
 * D+S rounding of exact sums: for each of `count` values given as c binary64
 * components (planes `stride` apart), hi = RN53(v) and lo = RN24(v - hi), both
 * from the exact value (a long fixed-point accumulator), ties to even.
 */
int oracle_ds_round(int c, long count, long stride, const double *x, double *hi, float *lo)
{
    if (c < 1 || c > ORC_MAXC || count < 0)
        return ORC_EINVAL;
    int status = ORC_OK;
#pragma omp parallel
    {
        sacc *s = malloc(sizeof(sacc));
        if (!s)
            status = ORC_ENOMEM;
#pragma omp for schedule(static)
        for (long t = 0; t < count; ++t) {
            if (!s)
                continue;
            sa_clear(s);
            for (int r = 0; r < c; ++r)
                sa_add(s, x[r * stride + t]);
            sa_norm(s);
            const double h = sa_round(s, 53, -1074);
            sa_add(s, -h);
            sa_norm(s);
            hi[t] = h;
            lo[t] = (float)sa_round(s, 24, -149);
        }
        free(s);
    }
    return status;
}

/*
 * The simple matrix multiplication in D+S: each D+S input is read as the DD
 * number (hi, (double)lo) (exact), the triple loop runs in the DD arithmetic
 * of oracle_gemm_naive (c = 2), and each entry of C is rounded to D+S once
 * at the end (oracle_ds_round of the DD accumulator).  Planes: A (k x m),
 * B (n x k), C (n x nrows), leading dimension = rows.
 */
int oracle_gemm_naive_ds(int m, int n, int k, const double *Ahi, const float *Alo, const double *Bhi,
                         const float *Blo, const int *rows, int nrows, double *Chi, float *Clo)
{
    if (m < 0 || n < 0 || k < 0)
        return ORC_EINVAL;
    const long pc = (long)nrows * n;
    double *acc2 = malloc(sizeof(double) * (size_t)(2 * pc + 1));
    if (!acc2)
        return ORC_ENOMEM;
#pragma omp parallel for schedule(static) collapse(2)
    for (int j = 0; j < n; ++j)
        for (int t = 0; t < nrows; ++t) {
            const int i = rows ? rows[t] : t;
            double acc[2] = {0.0, 0.0}, a[2], b[2], pr[2];
            for (int p = 0; p < k; ++p) {
                a[0] = Ahi[i + (long)p * m];
                a[1] = (double)Alo[i + (long)p * m];
                b[0] = Bhi[p + (long)j * k];
                b[1] = (double)Blo[p + (long)j * k];
                mc_mul(a, b, 2, pr);
                mc_add(acc, pr, 2);
            }
            acc2[t + (long)j * nrows] = acc[0];
            acc2[pc + t + (long)j * nrows] = acc[1];
        }
    const int st = oracle_ds_round(2, pc, pc, acc2, Chi, Clo);
    free(acc2);
    return st;
}

int oracle_omp_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the oracle's later parallel loops (for timing on one core). */
int oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
