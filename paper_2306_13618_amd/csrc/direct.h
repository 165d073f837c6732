// Direct kernel sums: FP32 VALU path (any d) and the MFMA BF16 hi/lo Gram path (Gaussian, d % 16 == 0).
#pragma once
#include "internal.h"

namespace fs {

float direct_coef(int kind, double lambda);

// out_i = sum_j K(|x_i - y_j|) w_j.  out (float) and/or out64 (double) may be NULL.
void direct_valu(int kind, double lambda, const float *x, int64_t n, const float *y, int64_t m,
                 int d, const float *w, float *out, double *out64, hipStream_t s);

// Gaussian kernel sum with x.y^T on MFMA from BF16 hi/lo splits (3 products, FP32 accumulate).
struct GramOperand {
    int64_t count = 0;
    int d = 0;
    DevBuf<uint16_t> hi, lo;  // bf16 bits, count x d
    DevBuf<float> sqnorm;     // |p|^2 in FP32
};
bool mfma_supported(int kind, int d);
void gram_prepare(const float *pts, int64_t count, int d, GramOperand &op, hipStream_t s);
void direct_mfma_gauss(double lambda, const GramOperand &x, const GramOperand &y, const float *w,
                       float *out, double *out64, hipStream_t s);

}  // namespace fs
