/*
 * TEST INFRASTRUCTURE ONLY -- the oracle's number formats for the
 * mixed-precision forms (bfloat16, OCP FP8 E4M3, three-term bfloat16 splits).
 *
 * Paper, Sec. 5: the fused packing is expected to carry over to other
 * precisions, and the packing stage may encode a transformation of the data
 * on its way into the packed buffer (the 1m method rewrites complex operands
 * while packing).  Here the pack converts: FP32 to bfloat16, or FP32 to a sum
 * of three bfloat16 terms.  The paper fixes none of the formats below; each
 * function states the definition it implements, written from the format's
 * specification (IEEE-style fields, round to nearest, ties to even), and
 * shares no code with the GPU library.
 *
 * Formats:
 *   bfloat16: the upper 16 bits of a binary32 (1 sign, 8 exponent, 7 fraction
 *     bits).  FP32 -> bfloat16 rounds to nearest, ties to even; a NaN stays a
 *     NaN (quiet bit set).
 *   OCP FP8 E4M3 ("E4M3FN"): 1 sign, 4 exponent (bias 7), 3 fraction bits; no
 *     infinities; S.1111.111 is NaN; largest finite 448 (0x7E); subnormals
 *     m/8 * 2^-6.  Encoding rounds to nearest, ties to even, and saturates
 *     finite values (and infinities) beyond 448 to +-448.
 *   FP8 scale of a line (row of op(A) or column of op(B)) with largest
 *     magnitude amax: the largest power of two s with amax * s <= 448
 *     (s = 1 when amax == 0); its exponent is clamped to [-126, 126].
 *   Three-term split of a binary32 x: x0 = bf16(x), x1 = bf16(x - x0),
 *     x2 = bf16(x - x0 - x1), each difference exact in binary32, so that
 *     x0 + x1 + x2 == x for every finite x whose bfloat16 rounding is finite.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

static uint32_t f32_bits(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    return u;
}

static float bits_f32(uint32_t u)
{
    float f;
    memcpy(&f, &u, 4);
    return f;
}

/* Round a binary32 to bfloat16 bits: nearest, ties to even. */
static uint16_t bf16_of(float f)
{
    const uint32_t u = f32_bits(f);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu) != 0)
        return (uint16_t)((u >> 16) | 0x0040u); /* NaN stays NaN */
    const uint32_t lower = u & 0xFFFFu, upper = u >> 16;
    uint32_t r = upper;
    if (lower > 0x8000u || (lower == 0x8000u && (upper & 1u))) r += 1; /* carries into the exponent */
    return (uint16_t)r;
}

static float bf16_value(uint16_t h) { return bits_f32((uint32_t)h << 16); }

void oracle_bf16_round(const float* x, int64_t n, uint16_t* out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = bf16_of(x[i]);
}

void oracle_bf16_decode(const uint16_t* h, int64_t n, double* out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = (double)bf16_value(h[i]);
}

/* x = x0 + x1 + x2 (three bfloat16 planes, plane-major in out: out[t*n + i]). */
void oracle_split3(const float* x, int64_t n, uint16_t* out)
{
    for (int64_t i = 0; i < n; ++i) {
        const float v = x[i];
        const uint16_t h0 = bf16_of(v);
        const float r1 = v - bf16_value(h0);
        const uint16_t h1 = bf16_of(r1);
        const float r2 = r1 - bf16_value(h1);
        out[i] = h0;
        out[n + i] = h1;
        out[2 * n + i] = bf16_of(r2);
    }
}

/* Value of an E4M3 code (NaN codes give NaN). */
static double e4m3_value(uint8_t q)
{
    const int s = q >> 7, e = (q >> 3) & 15, m = q & 7;
    double v;
    if (e == 15 && m == 7) return NAN;
    if (e == 0) v = ldexp((double)m, -9);      /* m/8 * 2^-6 */
    else v = ldexp(8.0 + m, e - 10);             /* (1 + m/8) * 2^(e-7) */
    return s ? -v : v;
}

void oracle_e4m3_decode(const uint8_t* q, int64_t n, double* out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = e4m3_value(q[i]);
}

/* Encode one value (given exactly as a double) to E4M3: nearest, ties to
   even, saturating.  Works by exact scaling: the representable magnitudes
   in [2^e, 2^(e+1)) are multiples of 2^(e-3) (normals, e >= -6); below
   2^-6 they are multiples of 2^-9. */
static uint8_t e4m3_of(double v)
{
    if (isnan(v)) return 0x7F;
    const uint8_t sign = signbit(v) ? 0x80 : 0x00;
    double a = fabs(v);
    if (a > 448.0) return sign | 0x7E;  /* saturate (also +-inf) */
    int e;
    if (a < ldexp(1.0, -6)) e = -6;      /* subnormal range: unit 2^-9 */
    else { frexp(a, &e); e -= 1; }      /* a in [2^e, 2^(e+1)) */
    const double unit = ldexp(1.0, e - 3);
    const double t = a / unit;           /* exact: power-of-two division */
    double r = floor(t);
    const double frac = t - r;
    if (frac > 0.5 || (frac == 0.5 && fmod(r, 2.0) != 0.0)) r += 1.0;
    double q = r * unit;                 /* the rounded magnitude */
    if (q > 448.0) q = 448.0;
    /* find the code of q by decoding all positive codes (monotone) */
    for (int c = 0; c <= 0x7E; ++c)
        if (e4m3_value((uint8_t)c) == q) return sign | (uint8_t)c;
    return sign | 0x7E; /* unreachable for finite inputs */
}

void oracle_e4m3_encode(const double* x, int64_t n, uint8_t* out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = e4m3_of(x[i]);
}

/* Exponent of the FP8 scale of a line with largest magnitude amax. */
static int fp8_scale_exp(double amax)
{
    if (!(amax > 0.0) || isinf(amax)) return 0;
    int best = -126;
    for (int e = 126; e >= -126; --e)
        if (ldexp(amax, e) <= 448.0) { best = e; break; }
    return best;
}

int oracle_fp8_scale_exponent(double amax) { return fp8_scale_exp(amax); }

/*
 * Quantize a binary32 matrix X (rows x cols, stored column-major (layout 0)
 * or row-major (1) with leading dimension ld) to E4M3 with one power-of-two
 * scale per row (axis 0) or per column (axis 1): Q = e4m3(X * s_line), stored
 * in the same layout with leading dimension ldq; scales[line] = s_line.
 */
void oracle_quantize_fp8(int layout, int64_t rows, int64_t cols, const float* X, int64_t ld,
                         int axis, uint8_t* Q, int64_t ldq, float* scales)
{
    const int64_t lines = axis == 0 ? rows : cols;
    for (int64_t l = 0; l < lines; ++l) {
        double amax = 0.0;
        const int64_t len = axis == 0 ? cols : rows;
        for (int64_t t = 0; t < len; ++t) {
            const int64_t r = axis == 0 ? l : t, c = axis == 0 ? t : l;
            const double v = fabs((double)X[layout == 0 ? r + c * ld : r * ld + c]);
            if (v > amax) amax = v;  /* NaN never compares greater */
        }
        const int e = fp8_scale_exp(amax);
        scales[l] = (float)ldexp(1.0, e);
        for (int64_t t = 0; t < len; ++t) {
            const int64_t r = axis == 0 ? l : t, c = axis == 0 ? t : l;
            const double v = (double)X[layout == 0 ? r + c * ld : r * ld + c];
            Q[layout == 0 ? r + c * ldq : r * ldq + c] = e4m3_of(ldexp(v, e));
        }
    }
}
