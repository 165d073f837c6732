// Direct kernel sums: FP32 VALU path (any d) and the matrix-core Gram path (Gaussian, d % 16 == 0).
#pragma once
#include "internal.h"

namespace fs {

float direct_coef(int kind, double lambda);

// out_i = sum_j K(|x_i - y_j|) w_j.  out (float) and/or out64 (double) may be NULL.
void direct_valu(int kind, double lambda, const float *x, int64_t n, const float *y, int64_t m,
                 int d, const float *w, float *out, double *out64, hipStream_t s);

// out_i = log sum_j exp(-|x_i - y_j|^r / lambda + u_j) in FP64 (r = 2 Gauss, 1 Laplace), with a
// running per-row maximum, so it holds for rows far from every source (no underflow); u is given
// in log2 units (u_j log2 e).
void direct_lse(int kind, double lambda, const float *x, int64_t n, const float *y, int64_t m,
                int d, const float *u, double *out, hipStream_t s);

// Gaussian kernel sum with the exponent on the matrix cores: FP16 hi/lo splits of the centred,
// scaled coordinates (3 products) plus one BF16 K step carrying the squared-norm terms, FP32
// accumulate.
struct GramOperand {
    int64_t count = 0;
    int d = 0, parts = 0;
    DevBuf<uint16_t> packed;  // per tile of 32 points and per part: 64 lanes x 8 halves
};
bool mfma_supported(int kind, int d);
// Largest exponent scale of the Gram path, Q = (log2 e / lambda) (R_x + R_y)^2 with R the largest
// norm of a set after centring; the path meets 1e-5 where Q <= GRAM_Q_MAX.
constexpr double GRAM_Q_MAX = 64.0;
// Common centre of x and y (midpoint of the joint bounding box, device, d floats) and the Q of
// the pair; synchronises the stream twice.
double gram_frame(const float *x, int64_t n, const float *y, int64_t m, bool same, int d,
                  double lambda, DevBuf<float> &center, hipStream_t s);
// Packs the points for kernel width lambda (the scaling depends on it), centred on `center`.
void gram_prepare(const float *pts, int64_t count, int d, double lambda, const float *center,
                  GramOperand &op, hipStream_t s);
// ext_partial (nullable): caller-owned FP64 buffer of ext_count elements for the per-split
// partial row sums; the splits are then limited to ext_count / x.count and nothing is allocated.
void direct_mfma_gauss(const GramOperand &x, const GramOperand &y, const float *w, float *out,
                       double *out64, hipStream_t s, double *ext_partial = nullptr,
                       size_t ext_count = 0);

}  // namespace fs
