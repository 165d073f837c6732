// Direct kernel sums: FP32 VALU path (any d) and the MFMA BF16 hi/lo Gram path (Gaussian, d % 16 == 0).
#pragma once
#include "internal.h"

namespace fs {

float direct_coef(int kind, double lambda);

// out_i = sum_j K(|x_i - y_j|) w_j.  out (float) and/or out64 (double) may be NULL.
void direct_valu(int kind, double lambda, const float *x, int64_t n, const float *y, int64_t m,
                 int d, const float *w, float *out, double *out64, hipStream_t s);

// Gaussian kernel sum with the exponent on MFMA: BF16 hi/lo splits of the scaled coordinates
// (3 products) plus one K step carrying the squared-norm terms, FP32 accumulate.
struct GramOperand {
    int64_t count = 0;
    int d = 0, parts = 0;
    DevBuf<uint16_t> packed;  // per tile of 32 points and per part: 64 lanes x 8 bf16
};
bool mfma_supported(int kind, int d);
// Packs the points for kernel width lambda (the scaling depends on it).
void gram_prepare(const float *pts, int64_t count, int d, double lambda, GramOperand &op,
                  hipStream_t s);
void direct_mfma_gauss(const GramOperand &x, const GramOperand &y, const float *w, float *out,
                       double *out64, hipStream_t s);

}  // namespace fs
