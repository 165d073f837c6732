// Direct O(n m) kernel sums (Algorithm 1's mat-vec evaluated pair by pair).
//
//   out_i = sum_j K(|x_i - y_j|) w_j
//
// FP32 VALU kernel: every thread owns R targets in registers, the workgroup stages a tile of
// sources (coordinates + weights) in LDS, each pair is evaluated in FP32, and the partial sum of
// each source tile is promoted to FP64 before it joins the running row sum (so the rounding error
// grows with the tile length, not with m).
#include <cfloat>

#include "direct.h"

namespace fs {

namespace {

constexpr int DT = 256;  // threads per block
constexpr int DR = 2;    // targets per thread
constexpr int DTILE = 256;

template <int KIND>
__device__ __forceinline__ float kval(float r2, float c) {
    // c: Gauss -log2(e)/lambda ; Laplace -log2(e)/lambda ; IMQ lambda^2
    if (KIND == FS_GAUSS) return exp2f(r2 * c);
    if (KIND == FS_LAPLACE) return exp2f(sqrtf(r2) * c);
    if (KIND == FS_IMQ) return rsqrtf(r2 + c);
    return -sqrtf(r2);
}

template <int D, int KIND>
__global__ void __launch_bounds__(DT) k_direct_small(const float *__restrict__ x, int64_t n,
                                                     const float *__restrict__ y, int64_t m,
                                                     const float *__restrict__ w, float c,
                                                     float *__restrict__ out,
                                                     double *__restrict__ out64) {
    __shared__ float sy[DTILE * D];
    __shared__ float sw[DTILE];
    const int64_t base = (int64_t)blockIdx.x * DT * DR;
    float xi[DR][D];
    double acc[DR];
#pragma unroll
    for (int r = 0; r < DR; ++r) {
        int64_t i = base + threadIdx.x + r * DT;
        acc[r] = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) xi[r][k] = (i < n) ? x[i * D + k] : 0.0f;
    }
    for (int64_t j0 = 0; j0 < m; j0 += DTILE) {
        const int cnt = (int)((m - j0) < DTILE ? (m - j0) : DTILE);
        __syncthreads();
        for (int t = threadIdx.x; t < DTILE; t += DT) {
            bool ok = t < cnt;
#pragma unroll
            for (int k = 0; k < D; ++k) sy[t * D + k] = ok ? y[(j0 + t) * D + k] : 0.0f;
            sw[t] = ok ? w[j0 + t] : 0.0f;
        }
        __syncthreads();
        float part[DR];
#pragma unroll
        for (int r = 0; r < DR; ++r) part[r] = 0.0f;
        for (int t = 0; t < cnt; ++t) {
            float yj[D];
#pragma unroll
            for (int k = 0; k < D; ++k) yj[k] = sy[t * D + k];
            const float wj = sw[t];
#pragma unroll
            for (int r = 0; r < DR; ++r) {
                float r2 = 0.0f;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    float dd = xi[r][k] - yj[k];
                    r2 = fmaf(dd, dd, r2);
                }
                part[r] = fmaf(kval<KIND>(r2, c), wj, part[r]);
            }
        }
#pragma unroll
        for (int r = 0; r < DR; ++r) acc[r] += (double)part[r];
    }
#pragma unroll
    for (int r = 0; r < DR; ++r) {
        int64_t i = base + threadIdx.x + r * DT;
        if (i < n) {
            if (out) out[i] = (float)acc[r];
            if (out64) out64[i] = acc[r];
        }
    }
}

// Any dimension d <= 128: coordinates of the source tile in LDS, targets read from global.
template <int KIND>
__global__ void __launch_bounds__(DT) k_direct_general(const float *__restrict__ x, int64_t n,
                                                       const float *__restrict__ y, int64_t m,
                                                       int d, const float *__restrict__ w,
                                                       float c, float *__restrict__ out,
                                                       double *__restrict__ out64) {
    constexpr int GT = 32;  // sources per tile
    __shared__ float sy[GT * 128];
    __shared__ float sw[GT];
    const int64_t i = (int64_t)blockIdx.x * DT + threadIdx.x;
    double acc = 0.0;
    const float *xi = x + (i < n ? i : 0) * d;
    for (int64_t j0 = 0; j0 < m; j0 += GT) {
        const int cnt = (int)((m - j0) < GT ? (m - j0) : GT);
        __syncthreads();
        for (int t = threadIdx.x; t < GT * d; t += DT) {
            int jj = t / d;
            sy[t] = (jj < cnt) ? y[(j0 + jj) * d + (t - jj * d)] : 0.0f;
        }
        for (int t = threadIdx.x; t < GT; t += DT) sw[t] = (t < cnt) ? w[j0 + t] : 0.0f;
        __syncthreads();
        float part = 0.0f;
        for (int t = 0; t < cnt; ++t) {
            float r2 = 0.0f;
            for (int k = 0; k < d; ++k) {
                float dd = xi[k] - sy[t * d + k];
                r2 = fmaf(dd, dd, r2);
            }
            part = fmaf(kval<KIND>(r2, c), sw[t], part);
        }
        acc += (double)part;
    }
    if (i < n) {
        if (out) out[i] = (float)acc;
        if (out64) out64[i] = acc;
    }
}

// Log-domain direct sum for the Sinkhorn half-step:
//   out_i = log sum_j exp(-r_ij^p / lambda + u_j)    (FP64 result; r^2 for Gauss, r for Laplace)
// with u_j the log source weights, given in log2 units (u_j log2 e).  Each row keeps a running
// maximum M of its exponents (log2 units) and the sum of 2^(e - M): a larger exponent rescales the
// sum once (rare after the first few terms), so the sum never underflows however far the row is
// from every source, and the result is (M + log2(sum)) ln 2.  DR targets per thread (coordinates
// in registers for d <= 3); sources staged in LDS tiles; per-tile FP32 partial sums joined in
// FP64.  D = 0: any d (coordinates read from global memory, one target per thread).
template <int D, int KIND>
__global__ void __launch_bounds__(DT) k_direct_lse(const float *__restrict__ x, int64_t n,
                                                   const float *__restrict__ y, int64_t m, int d,
                                                   const float *__restrict__ u2, float c2,
                                                   double *__restrict__ out) {
    constexpr int R = D > 0 ? DR : 1;
    constexpr int LT = D > 0 ? DTILE : 64;  // sources per tile
    __shared__ float sy[LT * (D > 0 ? D : 128)];
    __shared__ float su[LT];
    const int dd = D > 0 ? D : d;
    const int64_t base = (int64_t)blockIdx.x * DT * R;
    float xr[R][D > 0 ? D : 1];
    const float *xg = x + (base + threadIdx.x < n ? base + threadIdx.x : 0) * dd;
    if (D > 0) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t i = base + threadIdx.x + r * DT;
#pragma unroll
            for (int k = 0; k < (D > 0 ? D : 1); ++k) xr[r][k] = (i < n) ? x[i * dd + k] : 0.0f;
        }
    }
    float M[R];
    double S[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        M[r] = -FLT_MAX;
        S[r] = 0.0;
    }
    for (int64_t j0 = 0; j0 < m; j0 += LT) {
        const int cnt = (int)((m - j0) < LT ? (m - j0) : LT);
        __syncthreads();
        for (int t = threadIdx.x; t < LT * dd; t += DT) {
            const int jj = t / dd;
            sy[t] = (jj < cnt) ? y[(j0 + jj) * dd + (t - jj * dd)] : 0.0f;
        }
        for (int t = threadIdx.x; t < LT; t += DT) su[t] = (t < cnt) ? u2[j0 + t] : -INFINITY;
        __syncthreads();
        float P[R];
#pragma unroll
        for (int r = 0; r < R; ++r) P[r] = 0.0f;
        // chunks of CH sources: the running maximum is raised at most once per chunk (padded
        // tile entries have u = -inf and contribute nothing)
        constexpr int CH = 8;
        for (int t0 = 0; t0 < cnt; t0 += CH) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                float e[CH];
                float mx = -FLT_MAX;
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    const int t = t0 + c;  // t < LT: the tile is padded to LT entries
                    float r2 = 0.0f;
                    if (D > 0) {
#pragma unroll
                        for (int k = 0; k < (D > 0 ? D : 1); ++k) {
                            const float df = xr[r][k] - sy[t * dd + k];
                            r2 = fmaf(df, df, r2);
                        }
                    } else {
                        for (int k = 0; k < dd; ++k) {
                            const float df = xg[k] - sy[t * dd + k];
                            r2 = fmaf(df, df, r2);
                        }
                    }
                    e[c] = fmaf(KIND == FS_GAUSS ? r2 : __builtin_sqrtf(r2), c2, su[t]);
                    mx = fmaxf(mx, e[c]);
                }
                if (mx > M[r]) {
                    const float f = exp2f(M[r] - mx);
                    S[r] *= (double)f;
                    P[r] *= f;
                    M[r] = mx;
                }
#pragma unroll
                for (int c = 0; c < CH; ++c) P[r] += exp2f(e[c] - M[r]);
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) S[r] += (double)P[r];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = base + threadIdx.x + r * DT;
        if (i < n)
            out[i] = (S[r] > 0.0) ? ((double)M[r] + log2(S[r])) * 0.6931471805599453 : -INFINITY;
    }
}

template <int D>
void launch_small(int kind, const float *x, int64_t n, const float *y, int64_t m, const float *w,
                  float c, float *out, double *out64, hipStream_t s) {
    dim3 grid(blocks_for(n, DT * DR, int64_t(1) << 30)), block(DT);
    switch (kind) {
        case FS_GAUSS:
            hipLaunchKernelGGL((k_direct_small<D, FS_GAUSS>), grid, block, 0, s, x, n, y, m, w, c,
                               out, out64);
            break;
        case FS_LAPLACE:
            hipLaunchKernelGGL((k_direct_small<D, FS_LAPLACE>), grid, block, 0, s, x, n, y, m, w,
                               c, out, out64);
            break;
        case FS_IMQ:
            hipLaunchKernelGGL((k_direct_small<D, FS_IMQ>), grid, block, 0, s, x, n, y, m, w, c,
                               out, out64);
            break;
        default:
            hipLaunchKernelGGL((k_direct_small<D, FS_ENERGY>), grid, block, 0, s, x, n, y, m, w,
                               c, out, out64);
    }
    FS_LAUNCHED();
}

}  // namespace

float direct_coef(int kind, double lambda) {
    if (kind == FS_ENERGY) return 0.0f;
    if (kind == FS_IMQ) return (float)(lambda * lambda);
    return (float)(-1.4426950408889634 / lambda);
}

void direct_valu(int kind, double lambda, const float *x, int64_t n, const float *y, int64_t m,
                 int d, const float *w, float *out, double *out64, hipStream_t s) {
    if (n <= 0) return;
    const float c = direct_coef(kind, lambda);
    if (d == 1) return launch_small<1>(kind, x, n, y, m, w, c, out, out64, s);
    if (d == 2) return launch_small<2>(kind, x, n, y, m, w, c, out, out64, s);
    if (d == 3) return launch_small<3>(kind, x, n, y, m, w, c, out, out64, s);
    FS_REQUIRE(d <= 128, FS_EINVAL, "direct summation supports d <= 128 (got %d)", d);
    dim3 grid(blocks_for(n, DT, int64_t(1) << 30)), block(DT);
    switch (kind) {
        case FS_GAUSS:
            hipLaunchKernelGGL(k_direct_general<FS_GAUSS>, grid, block, 0, s, x, n, y, m, d, w, c,
                               out, out64);
            break;
        case FS_LAPLACE:
            hipLaunchKernelGGL(k_direct_general<FS_LAPLACE>, grid, block, 0, s, x, n, y, m, d, w,
                               c, out, out64);
            break;
        case FS_IMQ:
            hipLaunchKernelGGL(k_direct_general<FS_IMQ>, grid, block, 0, s, x, n, y, m, d, w, c,
                               out, out64);
            break;
        default:
            hipLaunchKernelGGL(k_direct_general<FS_ENERGY>, grid, block, 0, s, x, n, y, m, d, w,
                               c, out, out64);
    }
    FS_LAUNCHED();
}

void direct_lse(int kind, double lambda, const float *x, int64_t n, const float *y, int64_t m,
                int d, const float *u, double *out, hipStream_t s) {
    if (n <= 0) return;
    FS_REQUIRE(kind == FS_GAUSS || kind == FS_LAPLACE, FS_EINVAL,
               "log-domain direct sums need the Gauss or Laplace kernel");
    FS_REQUIRE(d >= 1 && d <= 128, FS_EINVAL, "direct summation supports d <= 128 (got %d)", d);
    const float c2 = (float)(-1.4426950408889634 / lambda);
    const int per = d <= 3 ? DT * DR : DT;
    dim3 grid(blocks_for(n, per, int64_t(1) << 30)), block(DT);
#define FS_LSE(DD)                                                                             \
    if (kind == FS_GAUSS)                                                                      \
        hipLaunchKernelGGL((k_direct_lse<DD, FS_GAUSS>), grid, block, 0, s, x, n, y, m, d, u,  \
                           c2, out);                                                           \
    else                                                                                       \
        hipLaunchKernelGGL((k_direct_lse<DD, FS_LAPLACE>), grid, block, 0, s, x, n, y, m, d,   \
                           u, c2, out)
    switch (d) {
        case 1: FS_LSE(1); break;
        case 2: FS_LSE(2); break;
        case 3: FS_LSE(3); break;
        default: FS_LSE(0); break;
    }
#undef FS_LSE
    FS_LAUNCHED();
}

}  // namespace fs
