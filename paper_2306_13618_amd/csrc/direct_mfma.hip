// Gaussian kernel sum for high dimension (d a multiple of 16) with the Gram tiles x_i . y_j on
// the matrix cores.  Each coordinate is split into BF16 hi = bf16(v) and lo = bf16(v - hi); the
// dot product is hi.hi + hi.lo + lo.hi accumulated in FP32 (the dropped lo.lo term is ~2^-16 of
// the product).  Then  K_ij = exp(-(|x_i|^2 + |y_j|^2 - 2 x_i.y_j)/lambda)  with the squared norms
// in FP32, and the row sums sum_j K_ij w_j are accumulated per lane in FP32 over 8 column tiles
// and in FP64 beyond.
//
// Wave tile: 32 target rows x 32 source columns, v_mfma_f32_32x32x16_bf16 (gfx950).
// Operand layout of that instruction (per lane l of the wave):
//   A (32 x 16):  row l % 32, k = 8 (l / 32) .. 8 (l / 32) + 7
//   B (16 x 32):  column l % 32, same k range
//   D (32 x 32):  register r holds row 8 (r / 4) + 4 (l / 32) + (r % 4), column l % 32
#include "direct.h"

namespace fs {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint16_t f2bf_bits(float v) {
    // round to nearest even (inputs are finite)
    uint32_t u = __float_as_uint(v);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf_bits2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__global__ void k_split(const float *__restrict__ p, int64_t count, int d,
                        uint16_t *__restrict__ hi, uint16_t *__restrict__ lo,
                        float *__restrict__ sq) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= count) return;
    float s = 0.0f;
    for (int k = 0; k < d; ++k) {
        float v = p[i * d + k];
        uint16_t h = f2bf_bits(v);
        float r = v - bf_bits2f(h);
        hi[i * d + k] = h;
        lo[i * d + k] = f2bf_bits(r);
        s = fmaf(v, v, s);
    }
    sq[i] = s;
}

template <int D>
__global__ void __launch_bounds__(256) k_gram_gauss(
    const uint16_t *__restrict__ xhi, const uint16_t *__restrict__ xlo,
    const float *__restrict__ xsq, int64_t n, const uint16_t *__restrict__ yhi,
    const uint16_t *__restrict__ ylo, const float *__restrict__ ysq, int64_t m,
    const float *__restrict__ w, float c2 /* 2 log2(e)/lambda */, float c1 /* -log2(e)/lambda */,
    float *__restrict__ out, double *__restrict__ out64) {
    constexpr int KS = D / 16;  // K steps of 16
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave) * 32;
    const int half = lane >> 5;   // 0 or 1
    const int col = lane & 31;
    // A operands: row row0 + col, k = 16 s + 8 half .. +7
    bf16x8 ah[KS], al[KS];
    {
        int64_t r = row0 + col;
        bool ok = r < n;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            u16x8 vh = {}, vl = {};
            if (ok) {
                vh = *reinterpret_cast<const u16x8 *>(xhi + r * D + 16 * s + 8 * half);
                vl = *reinterpret_cast<const u16x8 *>(xlo + r * D + 16 * s + 8 * half);
            }
            ah[s] = __builtin_bit_cast(bf16x8, vh);
            al[s] = __builtin_bit_cast(bf16x8, vl);
        }
    }
    // per-register row norms term: rows 8 (r/4) + 4 half + (r%4)
    float rowterm[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        int64_t rr = row0 + 8 * (r / 4) + 4 * half + (r % 4);
        rowterm[r] = (rr < n) ? c1 * xsq[rr] : 0.0f;
    }
    float part[16];
    double acc[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) { part[r] = 0.0f; acc[r] = 0.0; }
    int tiles_in_part = 0;
    for (int64_t j0 = 0; j0 < m; j0 += 32) {
        const int64_t j = j0 + col;
        const bool okj = j < m;
        bf16x8 bh[KS], bl[KS];
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            u16x8 vh = {}, vl = {};
            if (okj) {
                vh = *reinterpret_cast<const u16x8 *>(yhi + j * D + 16 * s + 8 * half);
                vl = *reinterpret_cast<const u16x8 *>(ylo + j * D + 16 * s + 8 * half);
            }
            bh[s] = __builtin_bit_cast(bf16x8, vh);
            bl[s] = __builtin_bit_cast(bf16x8, vl);
        }
        const float colterm = okj ? c1 * ysq[j] : 0.0f;
        const float wj = okj ? w[j] : 0.0f;
        f32x16 g = {};
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            g = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[s], bh[s], g, 0, 0, 0);
            g = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[s], bl[s], g, 0, 0, 0);
            g = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[s], bh[s], g, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            // exponent in log2 units: (2 x.y - |x|^2 - |y|^2) log2(e) / lambda  (<= 0 up to rounding)
            float e = fminf(fmaf(g[r], c2, rowterm[r] + colterm), 0.0f);
            part[r] = fmaf(exp2f(e), wj, part[r]);
        }
        if (++tiles_in_part == 8) {
#pragma unroll
            for (int r = 0; r < 16; ++r) { acc[r] += (double)part[r]; part[r] = 0.0f; }
            tiles_in_part = 0;
        }
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] += (double)part[r];
    // reduce over the 32 lanes of each half-wave (they hold the same rows, different columns)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        double v = acc[r];
#pragma unroll
        for (int off = 16; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        acc[r] = v;
    }
    if (col == 0) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            int64_t rr = row0 + 8 * (r / 4) + 4 * half + (r % 4);
            if (rr < n) {
                if (out) out[rr] = (float)acc[r];
                if (out64) out64[rr] = acc[r];
            }
        }
    }
}

}  // namespace

bool mfma_supported(int kind, int d) { return kind == FS_GAUSS && (d == 16 || d == 32 || d == 64 || d == 128); }

void gram_prepare(const float *pts, int64_t count, int d, GramOperand &op, hipStream_t s) {
    op.count = count;
    op.d = d;
    op.hi.alloc((size_t)(count * d) + 8);
    op.lo.alloc((size_t)(count * d) + 8);
    op.sqnorm.alloc((size_t)count + 1);
    if (count == 0) return;
    hipLaunchKernelGGL(k_split, dim3(blocks_for(count, 256, int64_t(1) << 30)), dim3(256), 0, s,
                       pts, count, d, op.hi.p, op.lo.p, op.sqnorm.p);
    FS_LAUNCHED();
}

void direct_mfma_gauss(double lambda, const GramOperand &x, const GramOperand &y, const float *w,
                       float *out, double *out64, hipStream_t s) {
    FS_REQUIRE(x.d == y.d && mfma_supported(FS_GAUSS, x.d), FS_EINVAL,
               "MFMA path needs matching d in {16,32,64,128}");
    if (x.count == 0) return;
    const float c1 = (float)(-1.4426950408889634 / lambda);
    const float c2 = (float)(2.0 * 1.4426950408889634 / lambda);
    dim3 grid(blocks_for(x.count, 128, int64_t(1) << 30)), block(256);
#define FS_GRAM(DD)                                                                            \
    hipLaunchKernelGGL(k_gram_gauss<DD>, grid, block, 0, s, x.hi.p, x.lo.p, x.sqnorm.p,        \
                       x.count, y.hi.p, y.lo.p, y.sqnorm.p, y.count, w, c2, c1, out, out64)
    switch (x.d) {
        case 16: FS_GRAM(16); break;
        case 32: FS_GRAM(32); break;
        case 64: FS_GRAM(64); break;
        default: FS_GRAM(128); break;
    }
#undef FS_GRAM
    FS_LAUNCHED();
}

}  // namespace fs
