/*
 * oracle.c -- plain CPU reference for the data-parallel hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library includes, links or
 * calls this file; it shares no header, helper, table or constant generator
 * with it.  Only the test-suite, the benchmark's CPU baseline and the smoke
 * check load it (through oracle/__init__.py).
 *
 * Every function is the plain definition of the result, written as a single
 * sequential loop, so that it can be checked against the paper by eye:
 *
 *   - reduce      : exact int64 sum of int32 values   (Sec. 5, "block-wide
 *                   parallel reduction"; read as the full sum of the array)
 *   - scan        : inclusive prefix sum, wrapping modulo 2^32 (Sec. 5,
 *                   "scan"; the paper fixes neither the kind of scan nor
 *                   its overflow behaviour: inclusive, int32 in and out,
 *                   two's-complement wrap is the reading taken here);
 *                   the exclusive form shifts it by one place, from 0
 *   - transpose   : out[c][r] = in[r][c] as a 32-bit pattern move (Sec. 1,
 *                   Listings 1 and 2; Sec. 5 "matrix transposition")
 *   - GEMM        : C = A*B, reference entries in FP64 with the absolute
 *                   value sum D = sum_k |a_ik||b_kj| that scales the error
 *                   bound (Sec. 5 "matrix multiplication")
 *   - split-BF16  : h = bf16_rne(a), l = bf16_rne(a - h), the operands of
 *                   the three-product GEMM C ~ Ah*Bh + Ah*Bl + Al*Bh
 *   - FP8 e4m3    : per-row / per-column absmax scaling, OCP e4m3fn encoding
 *                   with round-to-nearest-even and saturation to +-448
 *   - segmented   : the reduce / scan definitions restarted at every segment
 *                   offset
 *   - min/max     : smallest and largest int32 value (identities when empty)
 *   - float sum   : the exact sum of FP32 values, rounded once to a double
 *   - float scan  : the exact inclusive prefixes, each rounded once
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -shared -fPIC
 * (contraction off so that every FP32 multiply rounds on its own).
 */
#include <stdint.h>
#include <string.h>
#include <math.h>
#include <limits.h>

/* ------------------------------------------------------------------ */
/* Reduce: s = sum_i x_i, exact in int64 (|x_i| < 2^31, n < 2^32).     */
/* ------------------------------------------------------------------ */
int64_t oracle_reduce_i32(const int32_t *x, int64_t n)
{
    int64_t s = 0;
    for (int64_t i = 0; i < n; ++i)
        s += (int64_t)x[i];
    return s;
}

/* ------------------------------------------------------------------ */
/* Inclusive scan: y_i = (x_0 + ... + x_i) mod 2^32, stored as int32.   */
/* Returns 1 when the exact running total left the int32 range (so the */
/* stored values are the wrapped ones), else 0.  *max_abs receives the  */
/* largest |exact prefix| seen.                                         */
/* ------------------------------------------------------------------ */
int oracle_scan_i32(const int32_t *x, int32_t *y, int64_t n, int64_t *max_abs)
{
    uint32_t acc = 0;          /* modular running total */
    int64_t exact = 0, m = 0;  /* exact running total, for the wrap report */
    for (int64_t i = 0; i < n; ++i) {
        acc += (uint32_t)x[i];
        y[i] = (int32_t)acc;
        exact += (int64_t)x[i];
        int64_t a = exact < 0 ? -exact : exact;
        if (a > m) m = a;
    }
    if (max_abs) *max_abs = m;
    return m > INT32_MAX ? 1 : 0;
}

/* ------------------------------------------------------------------ */
/* Exclusive scan: y_0 = 0, y_i = (x_0 + ... + x_(i-1)) mod 2^32.       */
/* ------------------------------------------------------------------ */
void oracle_scan_exclusive_i32(const int32_t *x, int32_t *y, int64_t n)
{
    uint32_t acc = 0;          /* modular total of the elements before i */
    for (int64_t i = 0; i < n; ++i) {
        y[i] = (int32_t)acc;
        acc += (uint32_t)x[i];
    }
}

/* ------------------------------------------------------------------ */
/* Transpose of a rows x cols row-major matrix of 32-bit words:         */
/* out (cols x rows) has out[c][r] = in[r][c].  A byte move: NaN        */
/* payloads, signed zeros and subnormals pass through untouched.        */
/* ------------------------------------------------------------------ */
void oracle_transpose_u32(const uint32_t *in, uint32_t *out, int64_t rows, int64_t cols)
{
    for (int64_t r = 0; r < rows; ++r)
        for (int64_t c = 0; c < cols; ++c)
            memcpy(&out[c * rows + r], &in[r * cols + c], 4);
}

/* ------------------------------------------------------------------ */
/* The same transposition for elements of `elem` bytes (1, 2, 4 or 8):  */
/* element (r, c) of `in` is copied to element (c, r) of `out`.         */
/* ------------------------------------------------------------------ */
void oracle_transpose_bytes(const uint8_t *in, uint8_t *out, int64_t rows, int64_t cols,
                            int64_t elem)
{
    for (int64_t r = 0; r < rows; ++r)
        for (int64_t c = 0; c < cols; ++c)
            memcpy(&out[(c * rows + r) * elem], &in[(r * cols + c) * elem], (size_t)elem);
}

/* ------------------------------------------------------------------ */
/* Reversal of n 32-bit words: out[i] = in[n - 1 - i] (a byte move).    */
/* ------------------------------------------------------------------ */
void oracle_reverse_u32(const uint32_t *in, uint32_t *out, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        memcpy(&out[i], &in[n - 1 - i], 4);
}

/* ------------------------------------------------------------------ */
/* GEMM reference on sampled entries.                                   */
/* A is M x K (row stride lda), B is K x N (row stride ldb), row-major. */
/* For each sample s: R[s] = sum_k a[i][k]*b[k][j] in FP64 (every FP32  */
/* product is exact in FP64), D[s] = sum_k |a[i][k]|*|b[k][j]|.         */
/* ------------------------------------------------------------------ */
void oracle_gemm_ref_sampled(const float *A, int64_t lda, const float *B, int64_t ldb,
                             int64_t K, const int64_t *ii, const int64_t *jj, int64_t ns,
                             double *R, double *D)
{
    for (int64_t s = 0; s < ns; ++s) {
        double r = 0.0, d = 0.0;
        for (int64_t k = 0; k < K; ++k) {
            double p = (double)A[ii[s] * lda + k] * (double)B[k * ldb + jj[s]];
            r += p;
            d += fabs(p);
        }
        R[s] = r;
        if (D) D[s] = d;
    }
}

/* ------------------------------------------------------------------ */
/* bfloat16: the upper 16 bits of an IEEE binary32, rounded to nearest  */
/* with ties to even on the 16 dropped bits.  A NaN stays a NaN (quiet  */
/* bit forced); infinities and zeros keep their sign.                   */
/* ------------------------------------------------------------------ */
static uint32_t f32_bits(float a) { uint32_t u; memcpy(&u, &a, 4); return u; }
static float bits_f32(uint32_t u) { float a; memcpy(&a, &u, 4); return a; }

uint16_t oracle_bf16_rne(float a)
{
    uint32_t u = f32_bits(a);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu) != 0)
        return (uint16_t)((u >> 16) | 0x0040u);           /* quiet NaN */
    uint32_t upper = u >> 16, lower = u & 0xffffu;
    if (lower > 0x8000u || (lower == 0x8000u && (upper & 1u)))
        upper += 1u;                                       /* carries into the exponent */
    return (uint16_t)upper;
}

float oracle_bf16_to_f32(uint16_t h) { return bits_f32((uint32_t)h << 16); }

/* h = bf16(a); l = bf16(a - h) (a - h is exact in FP32). */
void oracle_split_bf16(const float *a, uint16_t *hi, uint16_t *lo, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) {
        uint16_t h = oracle_bf16_rne(a[i]);
        float rest = a[i] - oracle_bf16_to_f32(h);
        hi[i] = h;
        lo[i] = oracle_bf16_rne(rest);
    }
}

/* Reference of the three-product GEMM on its own operands, in FP64:     */
/* R3 = sum_k ah*bh + ah*bl + al*bh (each product exact in FP64);        */
/* D3 = the same sum of absolute values.                                 */
void oracle_gemm_bf16x3_sampled(const float *A, int64_t lda, const float *B, int64_t ldb,
                                int64_t K, const int64_t *ii, const int64_t *jj, int64_t ns,
                                double *R3, double *D3)
{
    for (int64_t s = 0; s < ns; ++s) {
        double r = 0.0, d = 0.0;
        for (int64_t k = 0; k < K; ++k) {
            float a = A[ii[s] * lda + k], b = B[k * ldb + jj[s]];
            uint16_t ah16 = oracle_bf16_rne(a), bh16 = oracle_bf16_rne(b);
            double ah = oracle_bf16_to_f32(ah16), bh = oracle_bf16_to_f32(bh16);
            double al = oracle_bf16_to_f32(oracle_bf16_rne(a - (float)ah));
            double bl = oracle_bf16_to_f32(oracle_bf16_rne(b - (float)bh));
            double p1 = ah * bh, p2 = ah * bl, p3 = al * bh;
            r += p1; r += p2; r += p3;
            d += fabs(p1) + fabs(p2) + fabs(p3);
        }
        R3[s] = r;
        if (D3) D3[s] = d;
    }
}

/* ------------------------------------------------------------------ */
/* OCP 8-bit floating point E4M3 ("e4m3fn"): 1 sign, 4 exponent bits    */
/* with bias 7, 3 mantissa bits; no infinities; S.1111.111 is NaN, so   */
/* the largest finite magnitude is 1.110b x 2^8 = 448; subnormals are   */
/* m x 2^-9, m = 1..7.                                                  */
/* ------------------------------------------------------------------ */

/* Round a non-negative double to the nearest integer, ties to even.   */
static double rne_int(double v)
{
    double f = floor(v), frac = v - f;
    if (frac > 0.5) return f + 1.0;
    if (frac < 0.5) return f;
    return fmod(f, 2.0) == 0.0 ? f : f + 1.0;
}

/* Encode with round-to-nearest-even; magnitudes that round above 448   */
/* (including infinity) saturate to 448; NaN maps to the NaN code.      */
uint8_t oracle_e4m3_encode(float x)
{
    uint32_t u = f32_bits(x);
    uint8_t sign = (uint8_t)((u >> 24) & 0x80u);
    if (isnan(x)) return (uint8_t)(sign | 0x7f);
    if (isinf(x)) return (uint8_t)(sign | 0x7e);  /* no infinities: saturate */
    double a = fabs((double)x);
    if (a == 0.0) return sign;
    if (a < ldexp(1.0, -6)) {                     /* subnormal range: quantum 2^-9 */
        double m = rne_int(a * 512.0);            /* exact scaling by a power of two */
        if (m >= 8.0) return (uint8_t)(sign | 0x08);      /* rounds up to 2^-6 */
        return (uint8_t)(sign | (uint8_t)m);
    }
    int e;                                        /* a = f * 2^e, f in [0.5, 1) */
    frexp(a, &e);
    int E = e - 1;                                /* a in [2^E, 2^(E+1)) */
    if (E > 8) return (uint8_t)(sign | 0x7e);     /* saturate */
    double m = rne_int(ldexp(a, 3 - E));          /* 8 <= m <= 16 */
    if (m >= 16.0) { m = 8.0; E += 1; }
    if (E > 8 || (E == 8 && m > 14.0)) return (uint8_t)(sign | 0x7e);
    return (uint8_t)(sign | (uint8_t)((E + 7) << 3) | (uint8_t)(m - 8.0));
}

void oracle_e4m3_encode_n(const float *x, uint8_t *q, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        q[i] = oracle_e4m3_encode(x[i]);
}

double oracle_e4m3_decode(uint8_t q)
{
    double s = (q & 0x80) ? -1.0 : 1.0;
    int ef = (q >> 3) & 0xf, mf = q & 0x7;
    if (ef == 0xf && mf == 0x7) return NAN;
    if (ef == 0) return s * ldexp((double)mf, -9);
    return s * ldexp(8.0 + mf, ef - 7 - 3);
}

/* Row scaling of A (M x K): alpha_i = max_k |a_ik| (exact),              */
/* inv = 448/alpha_i in FP32 (1 if the row is all zero),                  */
/* q_ik = e4m3(a_ik * inv) with one FP32 multiply, scale_i = alpha_i/448. */
void oracle_quant_rows_e4m3(const float *A, int64_t M, int64_t K, int64_t lda,
                            uint8_t *q, int64_t ldq, float *alpha, float *scale)
{
    for (int64_t i = 0; i < M; ++i) {
        float m = 0.0f;
        for (int64_t k = 0; k < K; ++k) {
            float v = fabsf(A[i * lda + k]);
            if (v > m) m = v;
        }
        float inv = (m > 0.0f) ? 448.0f / m : 1.0f;
        for (int64_t k = 0; k < K; ++k) {
            float t = A[i * lda + k] * inv;
            q[i * ldq + k] = oracle_e4m3_encode(t);
        }
        if (alpha) alpha[i] = m;
        if (scale) scale[i] = m / 448.0f;
    }
}

/* Column scaling of B (K x N): beta_j = max_k |b_kj|, same encoding. */
void oracle_quant_cols_e4m3(const float *B, int64_t K, int64_t N, int64_t ldb,
                            uint8_t *q, int64_t ldq, float *beta, float *scale)
{
    for (int64_t j = 0; j < N; ++j) {
        float m = 0.0f;
        for (int64_t k = 0; k < K; ++k) {
            float v = fabsf(B[k * ldb + j]);
            if (v > m) m = v;
        }
        float inv = (m > 0.0f) ? 448.0f / m : 1.0f;
        for (int64_t k = 0; k < K; ++k) {
            float t = B[k * ldb + j] * inv;
            q[k * ldq + j] = oracle_e4m3_encode(t);
        }
        if (beta) beta[j] = m;
        if (scale) scale[j] = m / 448.0f;
    }
}

/* Reference of the scaled FP8 GEMM on its own codes, in FP64:            */
/* Rq = sa_i * sb_j * sum_k deq(qa_ik) * deq(qb_kj); Dq with |.| terms.   */
void oracle_gemm_fp8_sampled(const uint8_t *qa, int64_t ldqa, const uint8_t *qb, int64_t ldqb,
                             const float *sa, const float *sb, int64_t K,
                             const int64_t *ii, const int64_t *jj, int64_t ns,
                             double *Rq, double *Dq)
{
    for (int64_t s = 0; s < ns; ++s) {
        double r = 0.0, d = 0.0;
        for (int64_t k = 0; k < K; ++k) {
            double p = oracle_e4m3_decode(qa[ii[s] * ldqa + k]) *
                       oracle_e4m3_decode(qb[k * ldqb + jj[s]]);
            r += p;
            d += fabs(p);
        }
        double sc = (double)sa[ii[s]] * (double)sb[jj[s]];
        Rq[s] = sc * r;
        if (Dq) Dq[s] = fabs(sc) * d;
    }
}

/* ------------------------------------------------------------------ */
/* Segmented forms: segment s covers [off[s], off[s+1]).               */
/* ------------------------------------------------------------------ */
void oracle_reduce_segmented_i32(const int32_t *x, const int64_t *off, int64_t S, int64_t *out)
{
    for (int64_t s = 0; s < S; ++s) {
        int64_t acc = 0;
        for (int64_t i = off[s]; i < off[s + 1]; ++i)
            acc += (int64_t)x[i];
        out[s] = acc;
    }
}

void oracle_scan_segmented_i32(const int32_t *x, int32_t *y, const int64_t *off, int64_t S)
{
    for (int64_t s = 0; s < S; ++s) {
        uint32_t acc = 0;
        for (int64_t i = off[s]; i < off[s + 1]; ++i) {
            acc += (uint32_t)x[i];
            y[i] = (int32_t)acc;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Min and max of int32 values: out[0] = min, out[1] = max.  An empty  */
/* array gives the identities out = {INT32_MAX, INT32_MIN}.  (A further */
/* reduction operator over the same block-wide structure, Sec. 5.)     */
/* ------------------------------------------------------------------ */
void oracle_minmax_i32(const int32_t *x, int64_t n, int32_t *out)
{
    int32_t lo = INT32_MAX, hi = INT32_MIN;
    for (int64_t i = 0; i < n; ++i) {
        if (x[i] < lo) lo = x[i];
        if (x[i] > hi) hi = x[i];
    }
    out[0] = lo;
    out[1] = hi;
}

/* ------------------------------------------------------------------ */
/* Sum of FP32 values, exactly, returned rounded once to the nearest    */
/* double (ties to even).  Every finite float is an integer multiple of */
/* 2^-149 below 2^128, so x * 2^149 is an integer of at most 277 bits;   */
/* the sum of n < 2^40 of them fits 317 bits.  The integers are added   */
/* into eleven 32-bit limbs (bits 32k .. 32k+31 of sum * 2^149), held   */
/* in int64 so that carries can wait, and the total is rounded at the  */
/* end.  Non-finite inputs follow IEEE addition, which for a sum is     */
/* order-free: any NaN, or +inf together with -inf, gives NaN; else an  */
/* infinity gives that infinity.  A zero total is returned as +0.      */
/* (The float reduction is the                                          */
/* block-wide reduction of Sec. 5 over another element type; the paper  */
/* fixes no order, so the exact sum is the reference.)                  */
/* ------------------------------------------------------------------ */
#define ORACLE_LIMBS 11

typedef struct {
    int64_t L[ORACLE_LIMBS];   /* sum * 2^149 in 32-bit limbs, carries pending */
    int64_t pending;           /* additions since the last carry pass */
    int nan, pinf, ninf;
} exact_acc;

static void limbs_carry(int64_t *L)
{
    for (int k = 0; k < ORACLE_LIMBS - 1; ++k) {
        int64_t c = L[k] >> 32;               /* floor division by 2^32 */
        L[k] -= c * ((int64_t)1 << 32);
        L[k + 1] += c;
    }
}

static void exact_add(exact_acc *a, float xf)
{
    uint32_t u;
    memcpy(&u, &xf, 4);
    const uint32_t ef = (u >> 23) & 0xFF, frac = u & 0x7FFFFF;
    if (ef == 0xFF) {
        if (frac) a->nan = 1;
        else if (u >> 31) a->ninf = 1;
        else a->pinf = 1;
        return;
    }
    /* value = m * 2^(s - 149) with m < 2^24, s in [0, 253] */
    const int64_t m = ef ? (int64_t)(frac | 0x800000u) : (int64_t)frac;
    const int s = ef ? (int)ef - 1 : 0;
    const int64_t v = (u >> 31) ? -(m << (s % 32)) : (m << (s % 32));   /* |v| < 2^55 */
    const int k = s / 32;
    a->L[k] += v & 0xFFFFFFFF;     /* low 32 bits, as a non-negative number */
    a->L[k + 1] += v >> 32;        /* the rest, floor-shifted */
    if (++a->pending == (1 << 20)) {
        limbs_carry(a->L);
        a->pending = 0;
    }
}

/* The accumulated value rounded once to the nearest double, ties to even. */
static double exact_round(exact_acc *a)
{
    if (a->nan || (a->pinf && a->ninf)) return NAN;
    if (a->pinf) return INFINITY;
    if (a->ninf) return -INFINITY;
    limbs_carry(a->L);             /* value-preserving */
    a->pending = 0;
    /* limbs 0..9 now lie in [0, 2^32); the top limb carries the sign */
    const int neg = a->L[ORACLE_LIMBS - 1] < 0;
    uint32_t mag[ORACLE_LIMBS];
    if (neg) {                      /* two's-complement negation over the limbs */
        uint64_t borrow = 1;
        for (int k = 0; k < ORACLE_LIMBS; ++k) {
            uint64_t w = (uint64_t)(~(uint32_t)a->L[k]) + borrow;
            mag[k] = (uint32_t)w;
            borrow = w >> 32;
        }
    } else {
        for (int k = 0; k < ORACLE_LIMBS; ++k) mag[k] = (uint32_t)a->L[k];
    }
    int top = -1;                   /* highest set bit of the magnitude */
    for (int k = ORACLE_LIMBS - 1; k >= 0 && top < 0; --k)
        for (int b = 31; b >= 0; --b)
            if ((mag[k] >> b) & 1u) { top = 32 * k + b; break; }
    if (top < 0) return 0.0;
#define BIT(b) ((b) >= 0 && ((mag[(b) / 32] >> ((b) % 32)) & 1u))
    const int lo = top - 52 > 0 ? top - 52 : 0;   /* keep bits lo..top: at most 53 */
    uint64_t mant = 0;
    for (int b = top; b >= lo; --b) mant = (mant << 1) | (uint64_t)BIT(b);
    if (lo > 0) {                   /* round to nearest, ties to even */
        int round = BIT(lo - 1), sticky = 0;
        for (int b = lo - 2; b >= 0 && !sticky; --b) sticky = BIT(b);
        if (round && (sticky || (mant & 1))) mant += 1;
    }
#undef BIT
    const double r = ldexp((double)mant, lo - 149);
    return neg ? -r : r;
}

double oracle_sum_f32(const float *x, int64_t n)
{
    exact_acc a;
    memset(&a, 0, sizeof a);
    for (int64_t i = 0; i < n; ++i) exact_add(&a, x[i]);
    return exact_round(&a);
}

/* ------------------------------------------------------------------ */
/* Inclusive scan of FP32 values, exactly: out[k] = x[0] + ... + x[i]  */
/* for i = idx[k], rounded once to the nearest double (idx ascending,   */
/* each below n).  The same exact accumulator as the sum, read at the   */
/* requested positions; idx = 0, 1, ..., n-1 gives the whole scan.      */
/* (The scan of Sec. 5 over float values; the paper fixes no order, so  */
/* the exact prefix is the reference.)                                  */
/* ------------------------------------------------------------------ */
int oracle_scan_f32_at(const float *x, int64_t n, const int64_t *idx, int64_t m, double *out)
{
    exact_acc a;
    memset(&a, 0, sizeof a);
    int64_t i = 0;
    for (int64_t k = 0; k < m; ++k) {
        if (idx[k] < i - 1 || idx[k] >= n) return -1;   /* not ascending or out of range */
        for (; i <= idx[k]; ++i) exact_add(&a, x[i]);
        out[k] = exact_round(&a);
    }
    return 0;
}
