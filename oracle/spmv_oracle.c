/*
 * CPU oracle for the CB-SpMV hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the package's smoke check and the benchmark's CPU
 * baseline may load this library.  It shares no code, header, table or helper
 * with the GPU library: it is the plain definition of what the CB method
 * computes, written for a reader to check by eye against the paper.
 *
 * What it computes
 *   The CB method re-orders the summation of the ordinary sparse
 *   matrix-vector product and nothing else (Section 2.2, Algorithm 1 gives the
 *   product; Algorithms 3 and 4 sum the same products tile by tile).  So the
 *   oracle is that product over the input's COO triplets (Section 2.1):
 *       S_i  = sum over stored entries t with row_t = i of val_t * x[col_t]
 *       y_i  = alpha * S_i + beta * y0_i      (beta term dropped when beta == 0)
 *   and, for k right-hand sides stored row-major, the same for every column.
 *   The BLAS alpha/beta convention (beta == 0 means y0 is never read) is the
 *   library contract, not a statement of the paper.
 *
 *   Checking variants accumulate S_i with Neumaier's compensated summation so
 *   that the reference error is far below every tolerance used in the tests.
 *
 *   The value-rounding helpers give the storage values of the FP32 and BF16
 *   variants: round-to-nearest, ties-to-even, straight from the FP64 value
 *   (no intermediate FP32 step for BF16), NaN kept as a quiet NaN with the top
 *   payload bits, overflow to +-Inf.
 *
 * Precision: everything in IEEE double, compiled without -ffast-math.
 */
#include <stdint.h>
#include <string.h>
#include <math.h>

/* ---- Section 2.1 / 2.2: plain product over COO triplets ---------------- */

/* y[i] = alpha * sum_{t: row[t]=i} val[t]*x[col[t]] + beta*y0[i]; the triplets
 * are visited in the order given.  y0 may alias y.  y0 is not read when
 * beta == 0. */
void oracle_spmv_coo(int64_t m, int64_t nnz, const int32_t *row, const int32_t *col,
                     const double *val, const double *x, double alpha, double beta,
                     const double *y0, double *y, double *work /* m doubles */)
{
    for (int64_t i = 0; i < m; ++i) work[i] = 0.0;
    for (int64_t t = 0; t < nnz; ++t) work[row[t]] += val[t] * x[col[t]];
    for (int64_t i = 0; i < m; ++i) {
        double r = alpha * work[i];
        if (beta != 0.0) r += beta * y0[i];
        y[i] = r;
    }
}

/* The same product over CSR rows with the rows split over `threads` OpenMP threads: the
 * all-core CPU reference the benchmark times.  Each row is summed in entry order, exactly as
 * oracle_spmv_coo forms it (beta = 0). */
void oracle_spmv_csr_par(int64_t m, const int64_t *row_ptr, const int32_t *col, const double *val,
                         const double *x, double alpha, double *y, int threads)
{
#pragma omp parallel for num_threads(threads) schedule(static, 1024)
    for (int64_t i = 0; i < m; ++i) {
        double s = 0.0;
        for (int64_t t = row_ptr[i]; t < row_ptr[i + 1]; ++t) s += val[t] * x[col[t]];
        y[i] = alpha * s;
    }
}

/* Neumaier-compensated variant of oracle_spmv_coo (checking reference). */
void oracle_spmv_coo_comp(int64_t m, int64_t nnz, const int32_t *row, const int32_t *col,
                          const double *val, const double *x, double alpha, double beta,
                          const double *y0, double *y, double *s, double *c /* m each */)
{
    for (int64_t i = 0; i < m; ++i) { s[i] = 0.0; c[i] = 0.0; }
    for (int64_t t = 0; t < nnz; ++t) {
        const int32_t i = row[t];
        const double p = val[t] * x[col[t]];
        const double sum = s[i] + p;
        /* the compensation is defined for finite partial sums only; once a sum
         * is Inf or NaN the result is the plain IEEE sum */
        if (isfinite(sum)) {
            if (fabs(s[i]) >= fabs(p)) c[i] += (s[i] - sum) + p;
            else                       c[i] += (p - sum) + s[i];
        }
        s[i] = sum;
    }
    for (int64_t i = 0; i < m; ++i) {
        double r = alpha * (isfinite(s[i]) ? s[i] + c[i] : s[i]);
        if (beta != 0.0) r += beta * y0[i];
        y[i] = r;
    }
}

/* scale[i] = |alpha| * sum |val_t| |x[col_t]| + |beta| |y0_i| -- the
 * normalisation of the accuracy metric (|A||x| term of a forward error bound).
 * The beta term is dropped when beta == 0. */
void oracle_scale_coo(int64_t m, int64_t nnz, const int32_t *row, const int32_t *col,
                      const double *val, const double *x, double alpha, double beta,
                      const double *y0, double *scale)
{
    for (int64_t i = 0; i < m; ++i) scale[i] = 0.0;
    for (int64_t t = 0; t < nnz; ++t) scale[row[t]] += fabs(val[t]) * fabs(x[col[t]]);
    for (int64_t i = 0; i < m; ++i) {
        double r = fabs(alpha) * scale[i];
        if (beta != 0.0) r += fabs(beta) * fabs(y0[i]);
        scale[i] = r;
    }
}

/* k right-hand sides, row-major: X is n x k with leading dimension ldx,
 * Y and Y0 are m x k with leading dimension ldy.
 * Y[i][j] = alpha * sum_t val_t X[col_t][j] + beta * Y0[i][j].
 * comp != 0 selects Neumaier accumulation.  work holds 2*m*k doubles. */
void oracle_spmm_coo(int64_t m, int64_t nnz, int32_t k, const int32_t *row, const int32_t *col,
                     const double *val, const double *X, int64_t ldx, double alpha, double beta,
                     const double *Y0, double *Y, int64_t ldy, int comp, double *work)
{
    double *s = work, *c = work + (size_t)m * (size_t)k;
    for (int64_t q = 0; q < m * (int64_t)k; ++q) { s[q] = 0.0; c[q] = 0.0; }
    for (int64_t t = 0; t < nnz; ++t) {
        const int64_t i = row[t];
        for (int32_t j = 0; j < k; ++j) {
            const double p = val[t] * X[(int64_t)col[t] * ldx + j];
            double *si = &s[i * k + j];
            if (!comp) { *si += p; continue; }
            const double sum = *si + p;
            if (isfinite(sum)) {
                if (fabs(*si) >= fabs(p)) c[i * k + j] += (*si - sum) + p;
                else                      c[i * k + j] += (p - sum) + *si;
            }
            *si = sum;
        }
    }
    for (int64_t i = 0; i < m; ++i)
        for (int32_t j = 0; j < k; ++j) {
            const double sij = s[i * k + j];
            double r = alpha * (isfinite(sij) ? sij + c[i * k + j] : sij);
            if (beta != 0.0) r += beta * Y0[i * ldy + j];
            Y[i * ldy + j] = r;
        }
}

/* ---- storage-value rounding (FP64 -> FP32 / BF16, RNE) ------------------ */

/* Round the non-negative integer sig / 2^shift to the nearest integer, ties to
 * even.  shift >= 1. */
static uint64_t rne_shift_right(uint64_t sig, int shift)
{
    if (shift >= 64) return 0; /* sig < 2^53 here, so the quotient is < 1/2 */
    const uint64_t q = sig >> shift;
    const uint64_t rem = sig & ((1ull << shift) - 1ull);
    const uint64_t half = 1ull << (shift - 1);
    if (rem > half || (rem == half && (q & 1ull))) return q + 1;
    return q;
}

/* Shared rounding of a finite non-zero double to a binary format with
 * `mant` stored significand bits and the IEEE single exponent range
 * (bias 127, min normal exponent -126).  Returns the encoded bits without sign. */
static uint32_t round_to_single_range(uint64_t bits, int mant)
{
    const int E = (int)((bits >> 52) & 0x7FF);
    if (E == 0) return 0; /* double subnormals are far below half the smallest target subnormal */
    const int e = E - 1023;                                  /* value = sig * 2^(e-52) */
    const uint64_t sig = (1ull << 52) | (bits & ((1ull << 52) - 1ull));
    const int qexp = (e < -126 ? -126 : e) - mant;           /* exponent of one unit in the last place */
    const int shift = qexp - (e - 52);
    const uint64_t q = rne_shift_right(sig, shift);          /* value ~= q * 2^qexp */
    if (e < -126) return (uint32_t)q;                        /* subnormal (q == 2^mant is the min normal) */
    int be = e + 127;
    uint64_t qq = q;
    if (qq == (1ull << (mant + 1))) { qq >>= 1; be += 1; }  /* carry into the exponent */
    if (be >= 255) return 0xFFu << mant;                     /* overflow -> Inf */
    return ((uint32_t)be << mant) | (uint32_t)(qq - (1ull << mant));
}

uint32_t oracle_round_f32_bits(double v)
{
    uint64_t b;
    memcpy(&b, &v, sizeof b);
    const uint32_t sign = (uint32_t)(b >> 63) << 31;
    const uint64_t M = b & ((1ull << 52) - 1ull);
    if (((b >> 52) & 0x7FF) == 0x7FF)
        return M ? (sign | 0x7FC00000u | (uint32_t)(M >> 29)) : (sign | 0x7F800000u);
    return sign | round_to_single_range(b, 23);
}

uint16_t oracle_round_bf16_bits(double v)
{
    uint64_t b;
    memcpy(&b, &v, sizeof b);
    const uint16_t sign = (uint16_t)((b >> 63) << 15);
    const uint64_t M = b & ((1ull << 52) - 1ull);
    if (((b >> 52) & 0x7FF) == 0x7FF)
        return M ? (uint16_t)(sign | 0x7FC0u | (uint16_t)(M >> 45)) : (uint16_t)(sign | 0x7F80u);
    return (uint16_t)(sign | round_to_single_range(b, 7));
}

void oracle_round_f32_array(int64_t n, const double *in, uint32_t *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = oracle_round_f32_bits(in[i]);
}

void oracle_round_bf16_array(int64_t n, const double *in, uint16_t *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = oracle_round_bf16_bits(in[i]);
}
