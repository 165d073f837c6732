// NFFT fast summation (Section "NFFT fast summation", eq. (1724)) on gfx950.
//
//   s(x_i) ~= sum_k b_k ( sum_j alpha_j e^{-2 pi i k . y_j} ) e^{2 pi i k . x_i},  k in I_N
//
// evaluated as: spread the weighted sources onto an oversampled grid of G = sigma N points per
// dimension with a Kaiser-Bessel window (adjoint NFFT), FFT, multiply by
//   M_k = b_k / (G^{2d} phihat(k)^2)        (kernel coefficients and both window deconvolutions)
// inside the band |k_i| <= N/2 (zero outside), inverse FFT, and interpolate at the targets with the
// same window (NFFT).  Nodes are scaled to the torus [-1/2, 1/2)^d by x / P (eq. (boundaries)).
//
// Hardware mapping:
//  * nodes are counting-sorted by grid tile (T^d points) once per plan; every spread/gather
//    workgroup owns one chunk of a tile's nodes and the tile's padded box (T + 2m - 1)^d in LDS;
//  * spreading accumulates into the LDS box with LDS float atomics (no global atomics); each lane
//    walks its node's window in a lane-rotated order so lanes whose nodes share a cell hit
//    different addresses; the boxes go to a scratch array and a fold pass sums, per grid point,
//    the boxes that cover it in a fixed order;
//  * FFTs are batched 1-D Stockham radix-2 transforms staged in LDS, one pass per axis, with the
//    real-to-complex step done two rows at a time and the spectrum pruned to the band after the
//    first forward pass of each axis; the multiply by M_k is fused between the forward and inverse
//    transform of the last axis.
#include <algorithm>
#include <array>
#include <atomic>
#include <cfloat>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>

#include "nfft.h"

namespace fs {

// =====================================================================================
//                                   host-side mathematics
// =====================================================================================
namespace {

// Derivatives K^{(j)}(s), j < cnt, of the radial kernel in data units.
void kernel_derivs(int kind, double lambda, double s, int cnt, double *out) {
    if (kind == FS_GAUSS) {
        // K(s) = exp(-u^2), u = s / sqrt(lambda):  d^j/ds^j = lambda^{-j/2} (-1)^j H_j(u) e^{-u^2}
        // (Rodrigues' formula; H_{j+1} = 2u H_j - 2j H_{j-1}, H_0 = 1, H_{-1} = 0)
        const double sl = std::sqrt(lambda), u = s / sl, e = std::exp(-u * u);
        double hprev = 0.0, h = 1.0;
        for (int j = 0; j < cnt; ++j) {
            out[j] = ((j & 1) ? -1.0 : 1.0) * h * e / std::pow(sl, j);
            const double hn = 2.0 * u * h - 2.0 * j * hprev;
            hprev = h;
            h = hn;
        }
    } else if (kind == FS_LAPLACE) {
        const double e = std::exp(-s / lambda);
        for (int j = 0; j < cnt; ++j) out[j] = std::pow(-1.0 / lambda, j) * e;
    } else if (kind == FS_IMQ) {
        // K(s) = (s^2 + c^2)^(-1/2): expanding K(s + h) in h gives the Legendre generating
        // function, K^{(j)}(s) = (-1)^j j! P_j(s / q) / q^(j+1) with q = sqrt(s^2 + c^2)
        // ((j+1) P_{j+1} = (2j+1) x P_j - j P_{j-1})
        const double q = std::sqrt(s * s + lambda * lambda), x = s / q;
        double pprev = 0.0, pc = 1.0, fact = 1.0, qp = q;
        for (int j = 0; j < cnt; ++j) {
            out[j] = ((j & 1) ? -1.0 : 1.0) * fact * pc / qp;
            const double pn = ((2.0 * j + 1.0) * x * pc - j * pprev) / (j + 1.0);
            pprev = pc;
            pc = pn;
            fact *= (j + 1.0);
            qp *= q;
        }
    } else {
        for (int j = 0; j < cnt; ++j) out[j] = (j == 0) ? -s : (j == 1 ? -1.0 : 0.0);
    }
}

// Solve A x = rhs (n <= 32) by Gaussian elimination with partial pivoting.
void solve_dense(int n, std::vector<double> A, std::vector<double> rhs, double *x) {
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
        FS_REQUIRE(std::fabs(A[piv * n + c]) > 0, FS_ENUMERIC, "singular regularisation system");
        if (piv != c) {
            for (int k = 0; k < n; ++k) std::swap(A[c * n + k], A[piv * n + k]);
            std::swap(rhs[c], rhs[piv]);
        }
        for (int r = c + 1; r < n; ++r) {
            double f = A[r * n + c] / A[c * n + c];
            for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
            rhs[r] -= f * rhs[c];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = rhs[r];
        for (int k = r + 1; k < n; ++k) s -= A[r * n + k] * x[k];
        x[r] = s / A[r * n + r];
    }
}

double falling(int e, int j) {  // e (e-1) ... (e-j+1)
    double v = 1.0;
    for (int t = 0; t < j; ++t) v *= (e - t);
    return v;
}

// Inner regularisation: even polynomial in rho = r / epsI (torus units),
//   q(r) = sum_{k<p} c_k rho^{2k},
// matching d^j/dr^j K(P r) at r = epsI for j < p, so that K_R is p-1 times differentiable there
// (and smooth at the origin as a function of the difference vector).  Written in the scaled
// variable rho so that the linear system has integer coefficients.
void inner_poly(int kind, double lambda, double P, double epsI, int p, double *c) {
    std::vector<double> der(p), A(p * p, 0.0), rhs(p);
    kernel_derivs(kind, lambda, P * epsI, p, der.data());
    for (int j = 0; j < p; ++j) {
        rhs[j] = der[j] * std::pow(P * epsI, j);
        for (int k = 0; k < p; ++k)
            if (2 * k >= j) A[j * p + k] = falling(2 * k, j);
    }
    solve_dense(p, A, rhs, c);
}

// Boundary regularisation: polynomial in zeta = (r - 1/2) / epsB,
//   q(r) = sum_{k <= 2p-2} c_k zeta^k,
// matching d^j/dr^j K(P r) at r_B = 1/2 - epsB (zeta = -1) for j < p, with q^{(j)} = 0 at r = 1/2
// for 1 <= j < p, so the kernel continues smoothly into the constant q(1/2) = c_0 beyond r = 1/2
// and its periodic continuation is smooth.
void boundary_poly(int kind, double lambda, double P, double epsB, int p, double *c) {
    const int nc = 2 * p - 1;
    const double rb = 0.5 - epsB;
    std::vector<double> der(p), A(nc * nc, 0.0), rhs(nc, 0.0);
    kernel_derivs(kind, lambda, P * rb, p, der.data());
    int row = 0;
    for (int j = 0; j < p; ++j, ++row) {
        for (int k = j; k < nc; ++k) A[row * nc + k] = falling(k, j) * (((k - j) & 1) ? -1.0 : 1.0);
        rhs[row] = der[j] * std::pow(P * epsB, j);
    }
    for (int j = 1; j < p; ++j, ++row) {
        A[row * nc + j] = falling(j, j);
        rhs[row] = 0.0;
    }
    solve_dense(nc, A, rhs, c);
}

// Modified Bessel function I_0 by its power series (all terms positive).
double bessel_i0(double x) {
    double s = 1.0, t = 1.0, h = 0.25 * x * x;
    for (int k = 1; k < 500; ++k) {
        t *= h / ((double)k * k);
        s += t;
        if (t < 1e-18 * s) break;
    }
    return s;
}

// Fourier transform of the normalised window (phi(0) = 1) at integer frequency k on a grid of G
// points:  phihat(k) = (1/G) I_0(m sqrt(b^2 - (2 pi k / G)^2)) / phi0,  phi0 = sinh(b m)/(pi m)
// (the transform pair of the Kaiser-Bessel window; the (1/pi) sinh form has transform I_0).
double kb_hat(double m, double b, int G, int k) {
    const double w = 2.0 * M_PI * k / G;
    const double arg = m * std::sqrt(std::max(b * b - w * w, 0.0));
    const double phi0 = std::sinh(b * m) / (M_PI * m);
    return bessel_i0(arg) / G / phi0;
}

// Kaiser-Bessel window (normalised, phi(0) = 1) and its derivative in FP64, grid units.
double kb_value(double m, double b, double s) {
    const double q2 = m * m - s * s;
    if (q2 <= 0.0) return (q2 == 0.0) ? b * m / (-std::expm1(-2.0 * b * m)) * 2.0 * std::exp(-b * m) : 0.0;
    const double q = std::sqrt(q2);
    return std::exp(b * (q - m)) * (-std::expm1(-2.0 * b * q)) / q * m / (-std::expm1(-2.0 * b * m));
}
double kb_deriv(double m, double b, double s) {
    const double h = 1e-6;
    // complex-step-free central difference in FP64 is accurate to ~1e-10 here (smooth segment)
    return (kb_value(m, b, s + h) - kb_value(m, b, s - h)) / (2.0 * h);
}

// Least-squares fit of f on [-1, 1] by sum_{k<K} c_k u^k at 4K Chebyshev points (normal equations
// in FP64; the Vandermonde basis is well conditioned at this degree on these points).
template <class F>
void fit_poly(F f, int K, double *c) {
    const int M = 4 * K;
    std::vector<double> A(K * K, 0.0), rhs(K, 0.0);
    for (int i = 0; i < M; ++i) {
        const double u = std::cos(M_PI * (i + 0.5) / M);
        const double fv = f(u);
        double pu[32];
        pu[0] = 1.0;
        for (int k = 1; k < K; ++k) pu[k] = pu[k - 1] * u;
        for (int r = 0; r < K; ++r) {
            rhs[r] += pu[r] * fv;
            for (int k = 0; k < K; ++k) A[r * K + k] += pu[r] * pu[k];
        }
    }
    solve_dense(K, A, rhs, c);
}

}  // namespace

// =====================================================================================
//                                    device helpers
// =====================================================================================
namespace {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Eight-point DFT in registers, V[k] = sum_m v[m] w^{mk}, w = e^{DIR 2 pi i / 8} (radix 2,
// decimation in frequency; the outputs are written back in natural order).
template <int DIR>
__device__ __forceinline__ void dft8(float2 *v) {
    constexpr float r = 0.70710678118654752f;
    // stage 1: pairs (m, m + 4)
    float2 t[8];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        t[m] = make_float2(v[m].x + v[m + 4].x, v[m].y + v[m + 4].y);
        t[m + 4] = make_float2(v[m].x - v[m + 4].x, v[m].y - v[m + 4].y);
    }
    // twiddles w^m on the difference half: m = 1: (1 -/+ i) r, m = 2: -/+ i, m = 3: (-1 -/+ i) r
    const float s = (DIR < 0) ? -1.0f : 1.0f;
    {
        const float2 a = t[5];
        t[5] = make_float2(r * (a.x - s * a.y), r * (a.y + s * a.x));
        const float2 b = t[6];
        t[6] = make_float2(-s * b.y, s * b.x);
        const float2 c = t[7];
        t[7] = make_float2(r * (-c.x - s * c.y), r * (-c.y + s * c.x));
    }
    // stage 2: within each half, pairs (m, m + 2); twiddle w^{2m} = -/+ i on m = 1 (odd index)
    float2 u[8];
#pragma unroll
    for (int h = 0; h < 8; h += 4) {
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            u[h + m] = make_float2(t[h + m].x + t[h + m + 2].x, t[h + m].y + t[h + m + 2].y);
            u[h + m + 2] = make_float2(t[h + m].x - t[h + m + 2].x, t[h + m].y - t[h + m + 2].y);
        }
        const float2 d = u[h + 3];
        u[h + 3] = make_float2(-s * d.y, s * d.x);
    }
    // stage 3: pairs (m, m + 1); the first half gives the even outputs, the second the odd ones
    const float2 y0 = make_float2(u[0].x + u[1].x, u[0].y + u[1].y);
    const float2 y4 = make_float2(u[0].x - u[1].x, u[0].y - u[1].y);
    const float2 y2 = make_float2(u[2].x + u[3].x, u[2].y + u[3].y);
    const float2 y6 = make_float2(u[2].x - u[3].x, u[2].y - u[3].y);
    const float2 y1 = make_float2(u[4].x + u[5].x, u[4].y + u[5].y);
    const float2 y5 = make_float2(u[4].x - u[5].x, u[4].y - u[5].y);
    const float2 y3 = make_float2(u[6].x + u[7].x, u[6].y + u[7].y);
    const float2 y7 = make_float2(u[6].x - u[7].x, u[6].y - u[7].y);
    v[0] = y0; v[1] = y1; v[2] = y2; v[3] = y3; v[4] = y4; v[5] = y5; v[6] = y6; v[7] = y7;
}

// Batched 64-point FFTs as 8 x 8 (same contract as lds_fft with logL = 6, transform t at
// a[t ST .. t ST + 64), ST = 64 unless padded against bank conflicts): thread (t, j) takes the
// 8-point DFT over m of a[t][j + 8 m], multiplies output k1 by w64^{j k1} and stores it at
// b[t][8 k1 + j]; then thread (t, k1) takes the 8-point DFT over j of b[t][8 k1 + j] and stores
// output k2 at a[t][k1 + 8 k2].  Two passes over LDS instead of six.
template <int DIR, int ST = 64>
__device__ float2 *lds_fft64(float2 *a, float2 *b, int NB, const float2 *__restrict__ tw) {
    for (int q = threadIdx.x; q < NB * 8; q += blockDim.x) {
        const int t = q >> 3, j = q & 7;
        float2 v[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) v[m] = a[t * ST + j + 8 * m];
        dft8<DIR>(v);
#pragma unroll
        for (int k1 = 0; k1 < 8; ++k1) {
            const int e = j * k1;  // < 64
            float2 w = tw[e & 31];
            if (e & 32) w = make_float2(-w.x, -w.y);
            if (DIR > 0) w.y = -w.y;
            b[t * ST + 8 * k1 + j] = cmul(v[k1], w);
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < NB * 8; q += blockDim.x) {
        const int t = q >> 3, k1 = q & 7;
        float2 v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = b[t * ST + 8 * k1 + j];
        dft8<DIR>(v);
#pragma unroll
        for (int k2 = 0; k2 < 8; ++k2) a[t * ST + k1 + 8 * k2] = v[k2];
    }
    __syncthreads();
    return a;
}

// lds_fft64 whose second pass hands every output to out(t, k, value) (k = frequency or sample
// index of transform t) instead of storing it in natural order; `a` may be overwritten by out.
template <int DIR, int ST, class Out>
__device__ void lds_fft64_out(float2 *a, float2 *b, int NB, const float2 *__restrict__ tw,
                              Out out) {
    for (int q = threadIdx.x; q < NB * 8; q += blockDim.x) {
        const int t = q >> 3, j = q & 7;
        float2 v[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) v[m] = a[t * ST + j + 8 * m];
        dft8<DIR>(v);
#pragma unroll
        for (int k1 = 0; k1 < 8; ++k1) {
            const int e = j * k1;  // < 64
            float2 w = tw[e & 31];
            if (e & 32) w = make_float2(-w.x, -w.y);
            if (DIR > 0) w.y = -w.y;
            b[t * ST + 8 * k1 + j] = cmul(v[k1], w);
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < NB * 8; q += blockDim.x) {
        const int t = q >> 3, k1 = q & 7;
        float2 v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = b[t * ST + 8 * k1 + j];
        dft8<DIR>(v);
#pragma unroll
        for (int k2 = 0; k2 < 8; ++k2) out(t, k1 + 8 * k2, v[k2]);
    }
    __syncthreads();
}

// Batched complex FFT of NB transforms of length L = 2^logL held in LDS (transform t at
// a[t L .. t L + L)), Stockham radix-2, natural order in and out.  DIR = -1 forward
// (e^{-2 pi i jk/L}), +1 inverse (unnormalised).  Returns the buffer holding the result.
// tw[q] = exp(-2 pi i q / L) for q < L/2.  All threads of the block must call it.
template <int DIR>
__device__ float2 *lds_fft(float2 *a, float2 *b, int logL, int NB, const float2 *__restrict__ tw) {
    if (logL == 6) return lds_fft64<DIR>(a, b, NB, tw);
    const int L = 1 << logL, H = L >> 1;
    for (int ls = 0; (1 << ls) < L; ++ls) {
        const int Ns = 1 << ls;
        const int stride = H >> ls;  // L / (2 Ns)
        for (int q = threadIdx.x; q < NB * H; q += blockDim.x) {
            const int t = q >> (logL - 1), j = q & (H - 1);
            const int k = j & (Ns - 1);
            float2 a0 = a[t * L + j], a1 = a[t * L + j + H];
            float2 w = tw[k * stride];
            if (DIR > 0) w.y = -w.y;
            a1 = cmul(a1, w);
            const int o = ((j - k) << 1) + k;
            b[t * L + o] = make_float2(a0.x + a1.x, a0.y + a1.y);
            b[t * L + o + Ns] = make_float2(a0.x - a1.x, a0.y - a1.y);
        }
        __syncthreads();
        float2 *tmp = a;
        a = b;
        b = tmp;
    }
    return a;
}

// Horner evaluation of one window segment polynomial at u = 2t - 1.
__device__ __forceinline__ float wpoly_eval(const float *__restrict__ c, float u) {
    float v = c[WPOLY - 1];
#pragma unroll
    for (int k = WPOLY - 2; k >= 0; --k) v = fmaf(v, u, c[k]);
    return v;
}

// Largest v over the workgroup (wave shuffles, then one value per wave through red, which holds
// blockDim.x / 64 values); every thread gets the result.
__device__ __forceinline__ double block_max_f64(double v, double *red) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    __syncthreads();  // red may still be read by a previous call
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double m = red[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) m = fmax(m, red[i]);
    return m;
}

constexpr int FFT_THREADS = 256;
constexpr int FFT_BATCH = 4;  // loads per thread in flight in the FFT passes' load loops
constexpr int FFT_ELEMS = 4096;  // complex elements per LDS buffer (two buffers: 64 KB)

// ------------------------------------------------------------------ scaling and binning
// Per-workgroup coordinate ranges of n points (n x d floats): the array is read flat with a grid
// stride that is a multiple of d, so every thread sees one coordinate k; four loads per thread in
// flight.  part[6 b + k] / part[6 b + 3 + k]: workgroup b's minimum and maximum of coordinate k.
__global__ void __launch_bounds__(256) k_bbox(const float *__restrict__ p, int64_t n, int d,
                                              float *__restrict__ part, int *__restrict__ nonfinite) {
    __shared__ float smin[256 * 3], smax[256 * 3];
    const int64_t total = n * d;
    const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
    const int64_t stride = nthreads / d * d;
    const int64_t j0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int kc = (int)(j0 % d);
    float l = INFINITY, h = -INFINITY;
    bool bad = false;
    if (j0 < stride) {
        int64_t j = j0;
        for (; j + 3 * stride < total; j += 4 * stride) {
            const float v0 = p[j], v1 = p[j + stride], v2 = p[j + 2 * stride], v3 = p[j + 3 * stride];
            bad |= !(isfinite(v0) && isfinite(v1) && isfinite(v2) && isfinite(v3));
            l = fminf(l, fminf(fminf(v0, v1), fminf(v2, v3)));
            h = fmaxf(h, fmaxf(fmaxf(v0, v1), fmaxf(v2, v3)));
        }
        for (; j < total; j += stride) {
            const float v = p[j];
            bad |= !isfinite(v);
            l = fminf(l, v);
            h = fmaxf(h, v);
        }
    }
    if (bad) atomicAdd(nonfinite, 1);
    for (int k = 0; k < 3; ++k) {
        smin[threadIdx.x * 3 + k] = (k == kc) ? l : INFINITY;
        smax[threadIdx.x * 3 + k] = (k == kc) ? h : -INFINITY;
    }
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < 3; ++k) {
                smin[threadIdx.x * 3 + k] = fminf(smin[threadIdx.x * 3 + k], smin[(threadIdx.x + s) * 3 + k]);
                smax[threadIdx.x * 3 + k] = fmaxf(smax[threadIdx.x * 3 + k], smax[(threadIdx.x + s) * 3 + k]);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) {
            part[blockIdx.x * 6 + k] = smin[k];
            part[blockIdx.x * 6 + 3 + k] = smax[k];
        }
}

struct ScaleArgs {
    double c[3];
    double inv_P;
    int G, T, ntd, d;
    int S;  // box side T + W - 1
};

// Sort key of a node: its tile, and (when the key space is small enough) its cell inside the
// tile, so that nodes are ordered by tile and, within a tile, by grid cell.
// The node's rank among the nodes of its key (the counter's old value) is kept, so that the
// scatter needs no second round of atomics.
__global__ void k_keys(const float *__restrict__ p, int64_t n, ScaleArgs sa, int cell_keys,
                       int *__restrict__ key, int *__restrict__ rank, float4 *__restrict__ tmp,
                       int *__restrict__ hist) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int cell[3] = {0, 0, 0};
    float fr[3] = {0, 0, 0};
    for (int k = 0; k < sa.d; ++k) {
        double u = ((double)p[i * sa.d + k] - sa.c[k]) * sa.inv_P * sa.G + 0.5 * sa.G;
        double fl = floor(u);
        int c = (int)fl;
        double f = u - fl;
        if (c < 0) { c = 0; f = 0.0; }
        if (c > sa.G - 1) { c = sa.G - 1; f = 0.99999994; }
        cell[k] = c;
        fr[k] = (float)f;
        if (fr[k] >= 1.0f) fr[k] = 0.99999994f;
    }
    int tk = 0, loc = 0;
    for (int k = sa.d - 1; k >= 0; --k) {
        tk = tk * sa.ntd + cell[k] / sa.T;
        loc = loc * sa.T + cell[k] % sa.T;
    }
    // the cell as a linear offset inside its tile's box: (oz S + oy) S + ox, o = cell - tile T
    int packed = 0;
    for (int k = sa.d - 1; k >= 0; --k) packed = packed * sa.S + cell[k] % sa.T;
    int cells_per_tile = 1;
    for (int k = 0; k < sa.d; ++k) cells_per_tile *= sa.T;
    const int kk = cell_keys ? tk * cells_per_tile + loc : tk;
    key[i] = kk;
    tmp[i] = make_float4(fr[0], fr[1], fr[2], __int_as_float(packed));
    rank[i] = atomicAdd(&hist[kk], 1);
}

// Multi-block exclusive scan of an int array (up to 2^31 elements): block sums, a scan of the
// block sums (k_scan_tiles with chunk = 1 as a plain scan), then each block rescans its part.
constexpr int SCAN_PER_BLOCK = 4096;
__global__ void __launch_bounds__(256) k_block_sums(const int *__restrict__ in, int64_t n,
                                                    int *__restrict__ bsum) {
    __shared__ int sm[256];
    const int64_t base = (int64_t)blockIdx.x * SCAN_PER_BLOCK;
    int s = 0;
    for (int q = threadIdx.x; q < SCAN_PER_BLOCK; q += 256) {
        const int64_t i = base + q;
        if (i < n) s += in[i];
    }
    sm[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = sm[0];
}

__global__ void __launch_bounds__(256) k_block_scan(const int *__restrict__ in, int64_t n,
                                                    const int *__restrict__ boff,
                                                    int *__restrict__ out) {
    __shared__ int sm[256];
    const int64_t base = (int64_t)blockIdx.x * SCAN_PER_BLOCK;
    constexpr int PER = SCAN_PER_BLOCK / 256;  // 16 consecutive elements per thread
    int v[PER];
    int s = 0;
    for (int q = 0; q < PER; ++q) {
        const int64_t i = base + threadIdx.x * PER + q;
        v[q] = (i < n) ? in[i] : 0;
        s += v[q];
    }
    sm[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        int t = ((int)threadIdx.x >= o) ? sm[threadIdx.x - o] : 0;
        __syncthreads();
        sm[threadIdx.x] += t;
        __syncthreads();
    }
    int run = boff[blockIdx.x] + sm[threadIdx.x] - s;
    for (int q = 0; q < PER; ++q) {
        const int64_t i = base + threadIdx.x * PER + q;
        if (i < n) out[i] = run;
        run += v[q];
    }
}

// Node count of every tile from the cell-level offsets.
__global__ void k_tile_counts(const int *__restrict__ key_start, int ntiles, int cells_per_tile,
                              int total, int *__restrict__ tile_count) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    const int64_t k0 = (int64_t)t * cells_per_tile, k1 = k0 + cells_per_tile;
    const int s0 = key_start[k0];
    const int s1 = (t + 1 < ntiles) ? key_start[k1] : total;
    tile_count[t] = s1 - s0;
}

// Exclusive scans of node counts and chunk counts per tile (single workgroup).
__global__ void __launch_bounds__(1024) k_scan_tiles(const int *__restrict__ hist, int ntiles,
                                                     int chunk, int *__restrict__ tile_start,
                                                     int *__restrict__ tile_chunk,
                                                     int *__restrict__ totals) {
    __shared__ int sa[1024], sb[1024];
    const int per = (ntiles + 1023) / 1024;
    const int lo = threadIdx.x * per, hi = min(lo + per, ntiles);
    int s1 = 0, s2 = 0;
    for (int t = lo; t < hi; ++t) {
        s1 += hist[t];
        s2 += (hist[t] + chunk - 1) / chunk;
    }
    sa[threadIdx.x] = s1;
    sb[threadIdx.x] = s2;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int va = (threadIdx.x >= (unsigned)off) ? sa[threadIdx.x - off] : 0;
        int vb = (threadIdx.x >= (unsigned)off) ? sb[threadIdx.x - off] : 0;
        __syncthreads();
        sa[threadIdx.x] += va;
        sb[threadIdx.x] += vb;
        __syncthreads();
    }
    int r1 = sa[threadIdx.x] - s1, r2 = sb[threadIdx.x] - s2;
    for (int t = lo; t < hi; ++t) {
        int c = hist[t], nc = (c + chunk - 1) / chunk;
        tile_start[t] = r1;
        tile_chunk[2 * t] = r2;
        tile_chunk[2 * t + 1] = nc;
        r1 += c;
        r2 += nc;
    }
    if (threadIdx.x == 1023) {
        totals[0] = sa[1023];
        totals[1] = sb[1023];
    }
}

__global__ void k_scatter_nodes(const float *__restrict__ p, int64_t n, int d,
                                const int *__restrict__ key, const int *__restrict__ rank,
                                const float4 *__restrict__ tmp,
                                const int *__restrict__ tile_start, float4 *__restrict__ rec,
                                int *__restrict__ perm, float *__restrict__ xs) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int pos = tile_start[key[i]] + rank[i];
    rec[pos] = tmp[i];
    perm[pos] = (int)i;
    for (int k = 0; k < d; ++k) xs[(int64_t)pos * d + k] = p[i * d + k];
}

__global__ void k_fill_chunks(int ntiles, const int *__restrict__ tile_start,
                              const int *__restrict__ hist, const int *__restrict__ tile_chunk,
                              int chunk, int4 *__restrict__ chunks) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    const int c0 = tile_chunk[2 * t], nc = tile_chunk[2 * t + 1];
    const int s = tile_start[t], cnt = hist[t];
    for (int c = 0; c < nc; ++c) chunks[c0 + c] = make_int4(t, s + c * chunk, min(chunk, cnt - c * chunk), 0);
}

// First node and node count of every block of groups (read by the spread without the
// dependent load of the group records).
__global__ void k_block_nodes(const int4 *__restrict__ mblocks, const int4 *__restrict__ mgroups,
                              int nblocks, int2 *__restrict__ out) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nblocks) return;
    const int4 mb = mblocks[b];
    const int4 g0 = mgroups[mb.y], gl = mgroups[mb.y + mb.z - 1];
    out[b] = make_int2(g0.x, gl.x + gl.y - g0.x);
}

// Largest |base_k| over the nodes of every block of groups, one workgroup per block.
__global__ void __launch_bounds__(256) k_block_absmax(const float *__restrict__ base,
                                                      const int2 *__restrict__ mbnodes,
                                                      float *__restrict__ out) {
    __shared__ float red[4];
    const int2 kn = mbnodes[blockIdx.x];
    float mx = 0.0f;
    for (int k = kn.x + threadIdx.x; k < kn.x + kn.y; k += blockDim.x) mx = fmaxf(mx, fabsf(base[k]));
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

// Matrix-core groups (d = 3, nodes ordered by tile and cell, x fastest): a brick is BRICK_X
// consecutive cell keys (cells along x with the same y and z), so its nodes are contiguous; each
// brick is cut into groups of up to 16 nodes.
__global__ void k_brick_groups(const int *__restrict__ key_start, int64_t nbricks, int total,
                               int *__restrict__ gcount) {
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= nbricks) return;
    const int s0 = key_start[b * BRICK_X];
    const int s1 = (b + 1 < nbricks) ? key_start[(b + 1) * BRICK_X] : total;
    gcount[b] = (s1 - s0 + 15) / 16;
}

// Sum of `per` consecutive entries per tile: one workgroup of 256 threads per tile.
__global__ void __launch_bounds__(256) k_tile_sum(const int *__restrict__ in, int ntiles, int per,
                                                  int *__restrict__ out) {
    __shared__ int red[4];
    const int t = blockIdx.x;
    int acc = 0;
    for (int i = threadIdx.x; i < per; i += blockDim.x) acc += in[(int64_t)t * per + i];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[t] = red[0] + red[1] + red[2] + red[3];
}

// groups[gstart[b] + j] = (first node, node count, brick offset inside the tile's box, 0)
// (d = 2 or 3; the brick's cells are consecutive along x)
__global__ void k_fill_groups(const int *__restrict__ key_start, const int *__restrict__ gstart,
                              int64_t nbricks, int total, int d, int T, int S,
                              int4 *__restrict__ groups) {
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= nbricks) return;
    const int s0 = key_start[b * BRICK_X];
    const int s1 = (b + 1 < nbricks) ? key_start[(b + 1) * BRICK_X] : total;
    const int cnt = s1 - s0, g0 = gstart[b];
    const int bpr = T / BRICK_X;  // bricks per tile row
    int off;
    if (d == 3) {
        const int lb = (int)(b % ((int64_t)bpr * T * T));
        const int bx = lb % bpr, by = (lb / bpr) % T, bz = lb / (bpr * T);
        off = (bz * S + by) * S + bx * BRICK_X;
    } else {
        const int lb = (int)(b % ((int64_t)bpr * T));
        const int bx = lb % bpr, by = lb / bpr;
        off = by * S + bx * BRICK_X;
    }
    for (int j = 0; 16 * j < cnt; ++j)
        groups[g0 + j] = make_int4(s0 + 16 * j, min(16, cnt - 16 * j), off, 0);
}

// ------------------------------------------------------------------ kernel coefficients b_k
struct RegArgs {
    int kind, regime, p;
    double lambda, P, epsI, epsB;
    double ci[16], cb[32];
};

// The kernel kind is a template parameter: a runtime chain of kind tests in this FP64 kernel
// gave wrong values for the last kind on this compiler.
template <int KIND>
__device__ double kr_eval(const RegArgs &ra, double r) {
    // regularised kernel K_R at torus distance r (data-unit kernel value K(P r))
    if (ra.epsI > 0.0 && r < ra.epsI) {
        double rho2 = (r / ra.epsI) * (r / ra.epsI), v = 0.0;
        for (int k = ra.p - 1; k >= 0; --k) v = v * rho2 + ra.ci[k];
        return v;
    }
    if (ra.regime == REGIME_BALL && r > 0.5 - ra.epsB) {
        double z = (fmin(r, 0.5) - 0.5) / ra.epsB, v = 0.0;
        for (int k = 2 * ra.p - 2; k >= 0; --k) v = v * z + ra.cb[k];
        return v;
    }
    const double s = ra.P * r;
    if constexpr (KIND == FS_GAUSS) return exp(-s * s / ra.lambda);
    if constexpr (KIND == FS_LAPLACE) return exp(-s / ra.lambda);
    if constexpr (KIND == FS_IMQ) return 1.0 / sqrt(s * s + ra.lambda * ra.lambda);
    if constexpr (KIND == FS_ENERGY) return -s;
}

template <int KIND>
__global__ void k_sample_kr(RegArgs ra, int N, int d, double *__restrict__ out) {
    int64_t total = 1;
    for (int k = 0; k < d; ++k) total *= N;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        int64_t rem = q;
        double r2 = 0.0;
        for (int k = 0; k < d; ++k) {
            int j = (int)(rem % N);
            rem /= N;
            double t = (double)(j - N / 2) / N;
            r2 += t * t;
        }
        out[q] = kr_eval<KIND>(ra, sqrt(r2));
    }
}

// Cosine DFT along one axis: out[a][kk][b] = sum_j in[a][j][b] cos(2 pi (j - N/2) kk / N),
// kk <= N/2 (the samples are even, so the transform is real and even in kk).
__global__ void k_cos_dft(const double *__restrict__ in, int64_t A, int N, int64_t B,
                          const double *__restrict__ costab, double *__restrict__ out) {
    const int H = N / 2 + 1;
    const int64_t total = A * H * B;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = q % B;
        const int kk = (int)((q / B) % H);
        const int64_t a = q / (B * H);
        double s = 0.0;
        for (int j = 0; j < N; ++j) {
            int ph = (int)(((int64_t)(j - N / 2) * kk) % N);
            if (ph < 0) ph += N;
            s += in[(a * N + j) * B + b] * costab[ph];
        }
        out[(a * H + kk) * B + b] = s;
    }
}

__global__ void k_build_mult(const double *__restrict__ bk, int N, int d,
                             const double *__restrict__ dconv, double scale,
                             float *__restrict__ M) {
    const int H = N / 2 + 1;
    int64_t total = 1;
    for (int k = 0; k < d; ++k) total *= H;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        int64_t rem = q;
        double v = bk[q] * scale;
        for (int k = 0; k < d; ++k) {
            int kk = (int)(rem % H);
            rem /= H;
            v *= dconv[kk];
            if (kk == N / 2) v *= 0.5;  // the band edge +-N/2 is split symmetrically
        }
        M[q] = (float)v;
    }
}

// ------------------------------------------------------------------ spread (adjoint NFFT)
struct SpreadArgs {
    KB kb;
    int G, T, ntd, m;
    const float *wp;  // window polynomials: value (W x WPOLY) then derivative (W x WPOLY)
    // 3-D moment form: the transform from the WPOLY^2 Chebyshev moments of the (y, z) window
    // factor to the W x W window products, CC[(y, z)][q] x 2^MOM_CC_SHIFT, as matrix-core A
    // operands (FP16 hi and lo parts in separate operands, two K steps per operand)
    const uint4 *cc;
};
// CC is stored times 2^15: with the moments scaled to at most 2^15 in magnitude (fixed-point
// scale 2^30 / count, weights at most 1) both operands stay in FP16 range while |CC| < 2
constexpr int MOM_CC_SHIFT = 15;

template <int D>
__device__ __forceinline__ void tile_coords(int tile, int ntd, int *t) {
    t[0] = tile % ntd;
    if (D > 1) t[1] = (tile / ntd) % ntd;
    if (D > 2) t[2] = tile / (ntd * ntd);
}

// Fixed-point scale for one chunk: every partial sum of the box is bounded by
// sum_j |alpha_j| * max(phi)^d <= count * max|alpha| (phi <= 1), so with
// scale = 2^30 / (count * max|alpha|) all int32 partial sums stay below 2^30 in magnitude.
// LDS integer atomics are the fast path on gfx950 (LDS float atomics are far slower), and integer
// addition is associative, so the box additions themselves do not depend on the order in which
// the lanes' atomics land (the values added still depend on the node order within a cell).
template <class WF>
__device__ float chunk_scale_fn(WF wf, int k0, int cnt, float *red, float *wmax = nullptr) {
    float mx = 0.0f;
    for (int k = k0 + threadIdx.x; k < k0 + cnt; k += blockDim.x) mx = fmaxf(mx, fabsf(wf(k)));
    for (int off = 32; off >= 1; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    float m = 0.0f;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) m = fmaxf(m, red[i]);
    if (wmax) *wmax = m;
    return (m > 0.0f && cnt > 0) ? 1073741824.0f / ((float)cnt * m) : 1.0f;
}
__device__ float chunk_scale(const float *__restrict__ w, int k0, int cnt, float *red,
                            float *wmax = nullptr) {
    return chunk_scale_fn([&](int k) { return w[k]; }, k0, cnt, red, wmax);
}

template <int D, int W, int T>
__global__ void __launch_bounds__(256) k_spread(const float4 *__restrict__ rec,
                                                const float *__restrict__ w,
                                                const int4 *__restrict__ chunks, SpreadArgs sa,
                                                float *__restrict__ scratch) {
    constexpr int S = T + W - 1;
    constexpr int BOX = (D == 1) ? S : (D == 2 ? S * S : S * S * S);
    __shared__ int box[BOX];
    __shared__ float red[4];
    const int4 ch = chunks[blockIdx.x];
    for (int q = threadIdx.x; q < BOX; q += blockDim.x) box[q] = 0;
    const float scale = chunk_scale(w, ch.y, ch.z, red);
    const int lane = threadIdx.x & 63;
    const int ra = lane % W;
    for (int k = ch.y + threadIdx.x; k < ch.y + ch.z; k += blockDim.x) {
        const float4 r = rec[k];
        const int lb = __float_as_int(r.w);  // cell offset inside the tile's box
        const float alpha = w[k] * scale;
#pragma unroll
        for (int i = 0; i < W; ++i) {
            int a = i + ra;
            a = (a >= W) ? a - W : a;
            const float v = alpha * wpoly_eval(sa.wp + a * WPOLY, 2.0f * r.x - 1.0f);
            atomicAdd(&box[lb + a], __float2int_rn(v));
        }
    }
    __syncthreads();
    const float inv = 1.0f / scale;
    float *dst = scratch + (int64_t)blockIdx.x * BOX;
    for (int q = threadIdx.x; q < BOX; q += blockDim.x) dst[q] = (float)box[q] * inv;
}

// Wave-cooperative spreading (d = 2, 3).  Nodes are sorted by grid cell inside each tile; every
// wave takes a contiguous run of its chunk's nodes, one node at a time: lane l < d W evaluates the
// window value of dimension l / W at offset l % W and stores it in the wave's LDS slot; the lanes
// own the W^2 (y, x) pairs of the window (ceil(W^2 / 64) passes, the last one split over z where
// that fills it), read their x and y values and the z values back, and accumulate
// alpha phi_x phi_y phi_z in registers while consecutive nodes share a cell.  When the cell changes the registers are added
// to the chunk's LDS box with integer atomics (fixed point, see chunk_scale); the 64 addresses of
// every such atomic instruction are distinct and contiguous.
template <int D, int W, int T>
__global__ void __launch_bounds__(256) k_spread_wave(const float4 *__restrict__ rec,
                                                     const float *__restrict__ w,
                                                     const int4 *__restrict__ chunks,
                                                     SpreadArgs sa, float *__restrict__ scratch) {
    constexpr int S = T + W - 1;
    constexpr int BOX = (D == 2) ? S * S : S * S * S;
    constexpr int NZ = (D == 3) ? W : 1;
    // (y, x) pairs: NF full passes of 64 lanes and R pairs left over.  In 3-D the leftover pass
    // splits the W z offsets over 64 / R lane groups when that divides evenly (W = 8, 12, 16), so
    // every lane does W^3 / 64 multiply-adds per node; otherwise the leftover pass masks lanes.
    constexpr int NF = (W * W) / 64;
    constexpr int R = W * W - 64 * NF;
    constexpr bool SPLITZ = (D == 3) && R > 0 && (64 % R == 0) && (W % (64 / R) == 0);
    constexpr int ZL = SPLITZ ? W / (64 / R) : NZ;  // z offsets per lane in the leftover pass
    constexpr int NP = NF + (R > 0 ? 1 : 0);        // passes
    __shared__ int box[BOX];
    __shared__ float red[16];
    __shared__ __align__(16) float wslot[4][3 * 16 + 4];  // per wave: window values of one node
    const int4 ch = chunks[blockIdx.x];
    for (int q = threadIdx.x; q < BOX; q += blockDim.x) box[q] = 0;
    const float scale = chunk_scale(w, ch.y, ch.z, red);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    int poff[NP];
    int pa[NP], pb[NP];
    bool pv[NP];
#pragma unroll
    for (int P = 0; P < NP; ++P) {
        const int q = (SPLITZ && P == NF) ? NF * 64 + lane % R : P * 64 + lane;
        pv[P] = q < W * W;
        pb[P] = pv[P] ? q / W : 0;
        pa[P] = pv[P] ? q % W : 0;
        poff[P] = pb[P] * S + pa[P];
    }
    const int zoff = SPLITZ ? (lane / R) * ZL : 0;  // first z offset of this lane's leftover pass
    const int wdim = (lane < D * W) ? lane / W : 0;
    const int woff = lane % W;
    float wc[WPOLY];
#pragma unroll
    for (int k = 0; k < WPOLY; ++k) wc[k] = sa.wp[woff * WPOLY + k];
    // contiguous node range of this wave
    const int per = (ch.z + nwaves - 1) / nwaves;
    const int k0 = ch.y + wave * per, k1 = min(ch.y + ch.z, k0 + per);
    float acc[NP][NZ];
#pragma unroll
    for (int P = 0; P < NP; ++P)
#pragma unroll
        for (int l = 0; l < NZ; ++l) acc[P][l] = 0.0f;
    // the record's .w is the cell's linear offset inside the tile's box
    int cur = -1;
    auto flush = [&](int lb) {
#pragma unroll
        for (int P = 0; P < NP; ++P) {
            const bool part = SPLITZ && P == NF;
            const int b0 = lb + poff[P] + (part ? zoff * S * S : 0);
#pragma unroll
            for (int l = 0; l < (part ? ZL : NZ); ++l)
                if (pv[P]) atomicAdd(&box[b0 + (D == 3 ? l * S * S : 0)], __float2int_rn(acc[P][l]));
        }
    };
    // the next node's record and weight are requested while this node is processed
    float4 rn = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    float wn = 0.0f;
    if (k0 < k1) {
        rn = rec[k0];
        wn = w[k0];
    }
    for (int k = k0; k < k1; ++k) {
        const float4 r = rn;
        const float wk = wn;
        if (k + 1 < k1) {
            rn = rec[k + 1];
            wn = w[k + 1];
        }
        const int packed = __float_as_int(r.w);
        // a new cell: the registers go to the box and restart from this node's products
        const bool first = packed != cur;
        if (first) {
            if (cur >= 0) flush(cur);
            cur = packed;
        }
        const float alpha = wk * scale;
        const float fr = (wdim == 0) ? r.x : (wdim == 1 ? r.y : r.z);
        float *slot = wslot[wave];
        if (lane < D * W) slot[lane] = wpoly_eval(wc, 2.0f * fr - 1.0f);
        // the wave's LDS accesses complete in order; the fence keeps the compiler from reordering
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        float wxy[NP];
#pragma unroll
        for (int P = 0; P < NP; ++P) wxy[P] = pv[P] ? alpha * slot[pa[P]] * slot[W + pb[P]] : 0.0f;
        if (D == 2) {
            if (first) {
#pragma unroll
                for (int P = 0; P < NP; ++P) acc[P][0] = wxy[P];
            } else {
#pragma unroll
                for (int P = 0; P < NP; ++P) acc[P][0] += wxy[P];
            }
        } else {
            float wz[NZ];
#pragma unroll
            for (int l = 0; l < NZ; ++l) wz[l] = slot[2 * W + l];
            float wzp[ZL];
#pragma unroll
            for (int l = 0; l < ZL; ++l) wzp[l] = SPLITZ ? slot[2 * W + zoff + l] : wz[l];
            if (first) {
#pragma unroll
                for (int P = 0; P < NF; ++P)
#pragma unroll
                    for (int l = 0; l < NZ; ++l) acc[P][l] = wz[l] * wxy[P];
                if constexpr (NP > NF) {
#pragma unroll
                    for (int l = 0; l < ZL; ++l) acc[NF][l] = wzp[l] * wxy[NF];
                }
            } else {
#pragma unroll
                for (int P = 0; P < NF; ++P)
#pragma unroll
                    for (int l = 0; l < NZ; ++l) acc[P][l] = fmaf(wz[l], wxy[P], acc[P][l]);
                if constexpr (NP > NF) {
#pragma unroll
                    for (int l = 0; l < ZL; ++l) acc[NF][l] = fmaf(wzp[l], wxy[NF], acc[NF][l]);
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (cur >= 0) flush(cur);
    __syncthreads();
    const float inv = 1.0f / scale;
    float *dst = scratch + (int64_t)blockIdx.x * BOX;
    for (int q = threadIdx.x; q < BOX; q += blockDim.x) dst[q] = (float)box[q] * inv;
}

// Sum the boxes of all chunks of a tile into the tile's first chunk box (fixed chunk order), one
// thread per box element; `tiles` lists the ntiles tiles that hold more than one chunk.
__global__ void k_reduce_chunks(float *__restrict__ scratch, const int *__restrict__ tile_chunk,
                                const int *__restrict__ tiles, int ntiles, int box) {
    for (int ti = blockIdx.y; ti < ntiles; ti += gridDim.y) {
        const int t = tiles[ti];
        const int c0 = tile_chunk[2 * t], nc = tile_chunk[2 * t + 1];
        for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < box; e += gridDim.x * blockDim.x) {
            // eight loads in flight per step (fixed order)
            const float *base = scratch + (int64_t)c0 * box + e;
            float acc = base[0];
            int c = 1;
            for (; c + 8 <= nc; c += 8) {
                float v[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) v[i] = base[(int64_t)(c + i) * box];
                acc += ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
            }
            for (; c < nc; ++c) acc += base[(int64_t)c * box];
            scratch[(int64_t)c0 * box + e] = acc;
        }
    }
}

// The same sum when few tiles hold many chunks (clustered or low-dimensional sets): a block of 256
// threads takes 64 consecutive box elements of one tile; its 4 waves split the tile's chunks
// (wave w sums chunks w, w + 4, ..., four loads in flight) and the wave sums are added in order.
__global__ void __launch_bounds__(256) k_reduce_chunks_split(float *__restrict__ scratch,
                                                             const int *__restrict__ tile_chunk,
                                                             const int *__restrict__ tiles,
                                                             int ntiles, int box) {
    __shared__ float part[4][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int ti = blockIdx.y; ti < ntiles; ti += gridDim.y) {
        const int t = tiles[ti];
        const int c0 = tile_chunk[2 * t], nc = tile_chunk[2 * t + 1];
        for (int e0 = blockIdx.x * 64; e0 < box; e0 += gridDim.x * 64) {
            const int e = e0 + lane;
            float acc = 0.0f;
            if (e < box) {
                const float *base = scratch + (int64_t)c0 * box + e;
                int c = wv;
                for (; c + 12 < nc; c += 16) {
                    const float v0 = base[(int64_t)c * box], v1 = base[(int64_t)(c + 4) * box];
                    const float v2 = base[(int64_t)(c + 8) * box];
                    const float v3 = base[(int64_t)(c + 12) * box];
                    acc += (v0 + v1) + (v2 + v3);
                }
                for (; c < nc; c += 4) acc += base[(int64_t)c * box];
            }
            part[wv][lane] = acc;
            __syncthreads();
            if (wv == 0 && e < box)
                scratch[(int64_t)c0 * box + e] = ((part[0][lane] + part[1][lane]) + part[2][lane]) +
                                                 part[3][lane];
            __syncthreads();
        }
    }
}

// Fold for the common case (at least 3 tiles per dimension, boxes narrower than the grid,
// m <= T), after k_reduce_chunks: blockIdx.x picks a tile of the list (or tile blockIdx.x when
// there is no list), blockIdx.y a group of its points; the reduced box offsets of the 3^d
// neighbouring tiles sit in LDS and every grid point of the tile sums the boxes that cover it, in
// a fixed neighbour order.
template <int D>
__global__ void __launch_bounds__(256) k_fold_tiles(const float *__restrict__ scratch,
                                                    const int *__restrict__ tile_chunk,
                                                    const int *__restrict__ tiles, int G,
                                                    int T, int ntd, int m, int S,
                                                    float *__restrict__ grid) {
    constexpr int NN = (D == 1) ? 3 : (D == 2 ? 9 : 27);
    __shared__ int nc0[NN], nnc[NN];
    const int t = tiles ? tiles[blockIdx.x] : (int)blockIdx.x;
    int tc[3] = {0, 0, 0};
    tile_coords<D>(t, ntd, tc);
    if ((int)threadIdx.x < NN) {
        int rem = threadIdx.x, tid = 0, mul = 1;
        for (int k = 0; k < D; ++k) {
            const int dk = rem % 3 - 1;
            rem /= 3;
            const int tk = (tc[k] + dk + ntd) % ntd;
            tid += tk * mul;
            mul *= ntd;
        }
        nnc[threadIdx.x] = tile_chunk[2 * tid + 1];
        int box = S;
        if (D > 1) box *= S;
        if (D > 2) box *= S;
        nc0[threadIdx.x] = tile_chunk[2 * tid] * box;  // offset of the neighbour's reduced box
    }
    __syncthreads();
    int npts = T;
    if (D > 1) npts *= T;
    if (D > 2) npts *= T;
    for (int q = blockIdx.y * blockDim.x + threadIdx.x; q < npts; q += gridDim.y * blockDim.x) {
        int p[3] = {0, 0, 0};
        // the point's offset inside the box of the neighbour d (d = -1, 0, 1) along each axis:
        // i + m - 1 - d T (independent of the periodic wrap), inside when in [0, S)
        int loc[3][3] = {};
        bool in[3][3] = {};
        {
            int rem = q;
            for (int k = 0; k < D; ++k) {
                const int i = rem % T;
                rem /= T;
                p[k] = tc[k] * T + i;
#pragma unroll
                for (int e = 0; e < 3; ++e) {
                    loc[k][e] = i + m - 1 - (e - 1) * T;
                    in[k][e] = loc[k][e] >= 0 && loc[k][e] < S;
                }
            }
        }
        // the covering boxes are read together (all loads in flight), then summed in order
        float v[NN];
#pragma unroll
        for (int j = 0; j < NN; ++j) {
            const int e0 = j % 3, e1 = (j / 3) % 3, e2 = j / 9;
            int l = loc[0][e0];
            bool inside = nnc[j] > 0 && in[0][e0];
            if (D > 1) {
                l += S * loc[1][e1];
                inside = inside && in[1][e1];
            }
            if (D > 2) {
                l += S * S * loc[2][e2];
                inside = inside && in[2][e2];
            }
            v[j] = inside ? scratch[nc0[j] + l] : 0.0f;
        }
        float acc = 0.0f;
#pragma unroll
        for (int j = 0; j < NN; ++j) acc += v[j];
        int64_t gi = p[0];
        if (D > 1) gi += (int64_t)G * p[1];
        if (D > 2) gi += (int64_t)G * G * p[2];
        grid[gi] = acc;
    }
}

// Sum the tile boxes covering every grid point (fixed order), after k_reduce_chunks has summed
// each tile's chunk boxes into its first chunk box.
template <int D>
__global__ void k_fold(const float *__restrict__ scratch, const int *__restrict__ tile_chunk,
                       int G, int T, int ntd, int m, int S, float *__restrict__ grid) {
    const int BOX = (D == 1) ? S : (D == 2 ? S * S : S * S * S);
    int64_t total = 1;
    for (int k = 0; k < D; ++k) total *= G;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        int pc[3] = {0, 0, 0};
        {
            int64_t rem = q;
            for (int k = 0; k < D; ++k) { pc[k] = (int)(rem % G); rem /= G; }
        }
        // per dimension: covering (tile, local index) pairs
        int nt[3] = {1, 1, 1}, tl[3][6], lc[3][6];
        for (int k = 0; k < D; ++k) {
            nt[k] = 0;
            const int t0 = pc[k] / T;
            int seen[3];
            int ns = 0;
            for (int dt = -1; dt <= 1; ++dt) {
                int t = ((t0 + dt) % ntd + ntd) % ntd;
                bool dup = false;
                for (int u = 0; u < ns; ++u) dup |= (seen[u] == t);
                if (dup) continue;
                seen[ns++] = t;
                const int origin = t * T - (m - 1);
                int loc = ((pc[k] - origin) % G + G) % G;
                for (; loc < S && nt[k] < 6; loc += G) {
                    tl[k][nt[k]] = t;
                    lc[k][nt[k]] = loc;
                    ++nt[k];
                }
            }
        }
        float acc = 0.0f;
        for (int a2 = 0; a2 < (D > 2 ? nt[2] : 1); ++a2)
            for (int a1 = 0; a1 < (D > 1 ? nt[1] : 1); ++a1)
                for (int a0 = 0; a0 < nt[0]; ++a0) {
                    int tile = tl[0][a0], loc = lc[0][a0];
                    if (D > 1) { tile += ntd * tl[1][a1]; loc += S * lc[1][a1]; }
                    if (D > 2) { tile += ntd * ntd * tl[2][a2]; loc += S * S * lc[2][a2]; }
                    const int c0 = tile_chunk[2 * tile], nc = tile_chunk[2 * tile + 1];
                    if (nc > 0) acc += scratch[(int64_t)c0 * BOX + loc];
                }
        grid[q] = acc;
    }
}

// ------------------------------------------------------------------ FFT passes
struct FftArgs {
    int G, logG, N, KX;
    int nb;   // row pairs per block in the first-axis passes
    int nbx;  // columns per block in the strided passes
};

// First axis, forward: two real rows as one complex row (spectrum specA[row][kx]).
__global__ void __launch_bounds__(FFT_THREADS) k_fft_x_r2c(const float *__restrict__ grid,
                                                            int rows, FftArgs fa,
                                                            const float2 *__restrict__ tw,
                                                            float2 *__restrict__ specA) {
    extern __shared__ float2 fft_lds[];
    const int G = fa.G, NB = fa.nb;
    float2 *bufa = fft_lds, *bufb = fft_lds + NB * G;
    const int pairs = rows / 2;
    const int p0 = blockIdx.x * NB;
    const int nb = min(NB, pairs - p0);
    // FFT_BATCH loads per thread in flight before their stores to LDS
    for (int q0 = threadIdx.x; q0 < NB * G; q0 += FFT_BATCH * blockDim.x) {
        float2 v[FFT_BATCH];
#pragma unroll
        for (int u = 0; u < FFT_BATCH; ++u) {
            const int q = q0 + u * blockDim.x, t = q / G, i = q - t * G;
            v[u] = make_float2(0.f, 0.f);
            if (q < NB * G && t < nb) {
                const int64_t r0 = (int64_t)(p0 + t) * 2;
                v[u] = make_float2(grid[r0 * G + i], grid[(r0 + 1) * G + i]);
            }
        }
#pragma unroll
        for (int u = 0; u < FFT_BATCH; ++u) {
            const int q = q0 + u * blockDim.x;
            if (q < NB * G) bufa[q] = v[u];
        }
    }
    __syncthreads();
    float2 *res = lds_fft<-1>(bufa, bufb, fa.logG, NB, tw);
    for (int q = threadIdx.x; q < NB * fa.KX; q += blockDim.x) {
        const int t = q / fa.KX, k = q - t * fa.KX;
        if (t >= nb) continue;
        const float2 z = res[t * G + k], zm = res[t * G + ((G - k) & (G - 1))];
        const float2 A = make_float2(0.5f * (z.x + zm.x), 0.5f * (z.y - zm.y));
        const float2 B = make_float2(0.5f * (z.y + zm.y), 0.5f * (zm.x - z.x));
        const int64_t r0 = (int64_t)(p0 + t) * 2;
        specA[r0 * fa.KX + k] = A;
        specA[(r0 + 1) * fa.KX + k] = B;
    }
}

// First axis, inverse.
__global__ void __launch_bounds__(FFT_THREADS) k_fft_x_c2r(const float2 *__restrict__ specA,
                                                            int rows, FftArgs fa,
                                                            const float2 *__restrict__ tw,
                                                            float *__restrict__ grid) {
    extern __shared__ float2 fft_lds[];
    const int G = fa.G, NB = fa.nb, h = fa.N / 2;
    float2 *bufa = fft_lds, *bufb = fft_lds + NB * G;
    const int pairs = rows / 2;
    const int p0 = blockIdx.x * NB;
    const int nb = min(NB, pairs - p0);
    // FFT_BATCH loads per thread in flight before their stores to LDS
    for (int q0 = threadIdx.x; q0 < NB * G; q0 += FFT_BATCH * blockDim.x) {
        float2 v[FFT_BATCH];
#pragma unroll
        for (int u = 0; u < FFT_BATCH; ++u) {
            const int q = q0 + u * blockDim.x, t = q / G, k = q - t * G;
            float2 z = make_float2(0.f, 0.f);
            if (q < NB * G && t < nb) {
                const int64_t r0 = (int64_t)(p0 + t) * 2;
                if (k <= h) {
                    const float2 A = specA[r0 * fa.KX + k], B = specA[(r0 + 1) * fa.KX + k];
                    z = make_float2(A.x - B.y, A.y + B.x);
                } else if (k >= G - h) {
                    const int kk = G - k;
                    const float2 A = specA[r0 * fa.KX + kk], B = specA[(r0 + 1) * fa.KX + kk];
                    z = make_float2(A.x + B.y, -A.y + B.x);
                }
            }
            v[u] = z;
        }
#pragma unroll
        for (int u = 0; u < FFT_BATCH; ++u) {
            const int q = q0 + u * blockDim.x;
            if (q < NB * G) bufa[q] = v[u];
        }
    }
    __syncthreads();
    float2 *res = lds_fft<1>(bufa, bufb, fa.logG, NB, tw);
    for (int q = threadIdx.x; q < NB * G; q += blockDim.x) {
        const int t = q / G, i = q - t * G;
        if (t >= nb) continue;
        const int64_t r0 = (int64_t)(p0 + t) * 2;
        grid[r0 * G + i] = res[q].x;
        grid[(r0 + 1) * G + i] = res[q].y;
    }
}

// 1-D: whole convolution in one workgroup.
__global__ void __launch_bounds__(FFT_THREADS) k_fft_1d_conv(float *__restrict__ grid, FftArgs fa,
                                                              const float2 *__restrict__ tw,
                                                              const float *__restrict__ M) {
    extern __shared__ float2 fft_lds[];
    const int G = fa.G, h = fa.N / 2;
    float2 *bufa = fft_lds, *bufb = fft_lds + G;
    for (int q = threadIdx.x; q < G; q += blockDim.x) bufa[q] = make_float2(grid[q], 0.f);
    __syncthreads();
    float2 *res = lds_fft<-1>(bufa, bufb, fa.logG, 1, tw);
    float2 *other = (res == bufa) ? bufb : bufa;
    for (int q = threadIdx.x; q < G; q += blockDim.x) {
        int k = (q < G / 2) ? q : q - G;
        int ak = k < 0 ? -k : k;
        float mk = (ak <= h) ? M[ak] : 0.0f;
        res[q] = make_float2(res[q].x * mk, res[q].y * mk);
    }
    __syncthreads();
    res = lds_fft<1>(res, other, fa.logG, 1, tw);
    for (int q = threadIdx.x; q < G; q += blockDim.x) grid[q] = res[q].x;
}

// Strided pass along y of layout [z][y][kx] (KX columns).  MODE 0: 3-D forward, store the band
// ky in [-N/2, N/2] to specB[z][ky + N/2][kx].  MODE 1: 2-D forward, multiply, inverse, in place.
// MODE 2: 3-D inverse from the band in specB back to specA.
template <int MODE>
__global__ void __launch_bounds__(FFT_THREADS) k_fft_y(float2 *__restrict__ specA,
                                                        float2 *__restrict__ specB, FftArgs fa,
                                                        const float2 *__restrict__ tw,
                                                        const float *__restrict__ M) {
    extern __shared__ float2 fft_lds[];
    const int G = fa.G, KX = fa.KX, NBX = fa.nbx, h = fa.N / 2, NB1 = fa.N + 1;
    float2 *bufa = fft_lds, *bufb = fft_lds + NBX * G;
    const int nkb = (KX + NBX - 1) / NBX;
    const int z = blockIdx.x / nkb, kb = blockIdx.x - z * nkb;
    const int kx0 = kb * NBX, nbx = min(NBX, KX - kx0);
    // FFT_BATCH loads per thread in flight before their stores to LDS
    for (int q0 = threadIdx.x; q0 < NBX * G; q0 += FFT_BATCH * blockDim.x) {
        float2 v[FFT_BATCH];
#pragma unroll
        for (int u = 0; u < FFT_BATCH; ++u) {
            const int q = q0 + u * blockDim.x, y = q / NBX, c = q - y * NBX;
            v[u] = make_float2(0.f, 0.f);
            if (q < NBX * G && c < nbx) {
                if (MODE == 2) {
                    const int ky = (y <= G / 2) ? y : y - G;
                    if (ky >= -h && ky <= h)
                        v[u] = specB[((int64_t)z * NB1 + ky + h) * KX + kx0 + c];
                } else {
                    v[u] = specA[((int64_t)z * G + y) * KX + kx0 + c];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < FFT_BATCH; ++u) {
            const int q = q0 + u * blockDim.x, y = q / NBX, c = q - y * NBX;
            if (q < NBX * G) bufa[c * G + y] = v[u];
        }
    }
    __syncthreads();
    float2 *res;
    if (MODE == 2) {
        res = lds_fft<1>(bufa, bufb, fa.logG, NBX, tw);
    } else {
        res = lds_fft<-1>(bufa, bufb, fa.logG, NBX, tw);
    }
    if (MODE == 1) {
        float2 *other = (res == bufa) ? bufb : bufa;
        for (int q0 = threadIdx.x; q0 < NBX * G; q0 += FFT_BATCH * blockDim.x) {
            float mk[FFT_BATCH];
#pragma unroll
            for (int u = 0; u < FFT_BATCH; ++u) {
                const int q = q0 + u * blockDim.x, c = q / G, yi = q - c * G;
                const int ky = (yi <= G / 2) ? yi : yi - G;
                const int aky = ky < 0 ? -ky : ky;
                mk[u] = (q < NBX * G && aky <= h && c < nbx) ? M[aky * (h + 1) + kx0 + c] : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < FFT_BATCH; ++u) {
                const int q = q0 + u * blockDim.x;
                if (q < NBX * G) res[q] = make_float2(res[q].x * mk[u], res[q].y * mk[u]);
            }
        }
        __syncthreads();
        res = lds_fft<1>(res, other, fa.logG, NBX, tw);
    }
    if (MODE == 0) {
        for (int q = threadIdx.x; q < NBX * NB1; q += blockDim.x) {
            const int kyb = q / NBX, c = q - kyb * NBX;
            if (c >= nbx) continue;
            const int yi = (kyb - h) & (G - 1);
            specB[((int64_t)z * NB1 + kyb) * KX + kx0 + c] = res[c * G + yi];
        }
    } else {
        for (int q = threadIdx.x; q < NBX * G; q += blockDim.x) {
            const int y = q / NBX, c = q - y * NBX;
            if (c >= nbx) continue;
            specA[((int64_t)z * G + y) * KX + kx0 + c] = res[c * G + y];
        }
    }
}

// 3-D: along z for every (ky in band, kx): forward, multiply by M, inverse, in place in specB.
__global__ void __launch_bounds__(FFT_THREADS) k_fft_z_conv(float2 *__restrict__ specB,
                                                             FftArgs fa,
                                                             const float2 *__restrict__ tw,
                                                             const float *__restrict__ M) {
    extern __shared__ float2 fft_lds[];
    const int G = fa.G, KX = fa.KX, NBX = fa.nbx, h = fa.N / 2, NB1 = fa.N + 1, H = h + 1;
    float2 *bufa = fft_lds, *bufb = fft_lds + NBX * G;
    const int nkb = (KX + NBX - 1) / NBX;
    const int kyb = blockIdx.x / nkb, kb = blockIdx.x - kyb * nkb;
    const int kx0 = kb * NBX, nbx = min(NBX, KX - kx0);
    const int ky = kyb - h, aky = ky < 0 ? -ky : ky;
    // FFT_BATCH loads per thread in flight before their stores to LDS
    for (int q0 = threadIdx.x; q0 < NBX * G; q0 += FFT_BATCH * blockDim.x) {
        float2 v[FFT_BATCH];
#pragma unroll
        for (int u = 0; u < FFT_BATCH; ++u) {
            const int q = q0 + u * blockDim.x, zz = q / NBX, c = q - zz * NBX;
            v[u] = (q < NBX * G && c < nbx) ? specB[((int64_t)zz * NB1 + kyb) * KX + kx0 + c]
                                            : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < FFT_BATCH; ++u) {
            const int q = q0 + u * blockDim.x, zz = q / NBX, c = q - zz * NBX;
            if (q < NBX * G) bufa[c * G + zz] = v[u];
        }
    }
    __syncthreads();
    float2 *res = lds_fft<-1>(bufa, bufb, fa.logG, NBX, tw);
    float2 *other = (res == bufa) ? bufb : bufa;
    for (int q0 = threadIdx.x; q0 < NBX * G; q0 += FFT_BATCH * blockDim.x) {
        float mk[FFT_BATCH];
#pragma unroll
        for (int u = 0; u < FFT_BATCH; ++u) {
            const int q = q0 + u * blockDim.x, c = q / G, zi = q - c * G;
            const int kz = (zi <= G / 2) ? zi : zi - G;
            const int akz = kz < 0 ? -kz : kz;
            mk[u] = (q < NBX * G && akz <= h && c < nbx)
                        ? M[((int64_t)akz * H + aky) * H + kx0 + c]
                        : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < FFT_BATCH; ++u) {
            const int q = q0 + u * blockDim.x;
            if (q < NBX * G) res[q] = make_float2(res[q].x * mk[u], res[q].y * mk[u]);
        }
    }
    __syncthreads();
    res = lds_fft<1>(res, other, fa.logG, NBX, tw);
    for (int q = threadIdx.x; q < NBX * G; q += blockDim.x) {
        const int zz = q / NBX, c = q - zz * NBX;
        if (c >= nbx) continue;
        specB[((int64_t)zz * NB1 + kyb) * KX + kx0 + c] = res[c * G + zz];
    }
}

// 3-D, G = 64, in z slabs, so that every pass runs on 64 or more workgroups (the x passes, the y
// passes and the z convolution of the general path, k_fft_x_r2c, k_fft_y, k_fft_z_conv and
// k_fft_x_c2r, in three launches).  The band spectrum is kept as S[z][ky + h][kx] (|ky| <= h =
// N / 2, 0 <= kx <= h; N + 1 rows of N / 2 + 1; N < G, so that h + 1 <= 32 columns fit the LDS
// tables).
//   k_fft_xy_fwd64: one z slab per workgroup, forward along x (row pairs as complex rows) and
//                   then along y, the band stored to S;
//   k_fft_z_conv64: FFT_ZCOLS (ky, kx) columns per workgroup, forward along z, times M_k (zero
//                   outside |kz| <= h), inverse along z, in place in S;
//   k_fft_xy_inv64: one z slab per workgroup, inverse along y (zeros outside the band), then the
//                   real rows along x back to the grid.
// Every load of a workgroup is issued before its first store to LDS: the passes are short enough
// that one memory round trip per step would dominate them.
constexpr int FFT_ZCOLS = 8;
constexpr int FFT_ST = 64 + 7;  // padded LDS rows (few bank conflicts in the radix-8 passes)

__global__ void __launch_bounds__(256) k_fft_xy_fwd64(const float *__restrict__ grid, FftArgs fa,
                                                      const float2 *__restrict__ tw,
                                                      float2 *__restrict__ S) {
    constexpr int G = 64, ST = FFT_ST;
    __shared__ float2 a[(G / 2) * ST], b[(G / 2) * ST], twl[G / 2];
    const int h = fa.N / 2, KX = fa.KX, NB1 = fa.N + 1;
    const int z = blockIdx.x;
    const float *slab = grid + (int64_t)z * G * G;  // [y][x]
    // rows 2t and 2t + 1 as the real and imaginary parts of complex row t (all loads in flight
    // before the first store to LDS)
    constexpr int NT = 256, PT = (G / 2) * G / NT;
    float2 v[PT];
#pragma unroll
    for (int i = 0; i < PT; ++i) {
        const int q = threadIdx.x + i * NT, t = q / G, x = q % G;
        v[i] = make_float2(slab[(2 * t) * G + x], slab[(2 * t + 1) * G + x]);
    }
    const float2 tv = tw[threadIdx.x & (G / 2 - 1)];
#pragma unroll
    for (int i = 0; i < PT; ++i) {
        const int q = threadIdx.x + i * NT;
        a[(q / G) * ST + q % G] = v[i];
    }
    if (threadIdx.x < G / 2) twl[threadIdx.x] = tv;
    __syncthreads();
    lds_fft64<-1, ST>(a, b, G / 2, twl);
    // the two real rows' spectra at kx <= h, transposed to b[kx][y]
    for (int q = threadIdx.x; q < (G / 2) * KX; q += blockDim.x) {
        const int t = q / KX, k = q % KX;
        const float2 zz = a[t * ST + k], zm = a[t * ST + ((G - k) & (G - 1))];
        b[k * ST + 2 * t] = make_float2(0.5f * (zz.x + zm.x), 0.5f * (zz.y - zm.y));
        b[k * ST + 2 * t + 1] = make_float2(0.5f * (zz.y + zm.y), 0.5f * (zm.x - zz.x));
    }
    __syncthreads();
    // along y for every kx; the band |ky| <= h goes to S
    float2 *out = S + (int64_t)z * NB1 * KX;
    lds_fft64_out<-1, ST>(b, a, KX, twl, [&](int kx, int yi, float2 v) {
        const int ky = (yi <= G / 2) ? yi : yi - G;
        if (ky >= -h && ky <= h) out[(ky + h) * KX + kx] = v;
    });
}

__global__ void __launch_bounds__(64) k_fft_z_conv64(float2 *__restrict__ S, FftArgs fa,
                                                     const float2 *__restrict__ tw,
                                                     const float *__restrict__ M) {
    constexpr int G = 64, ST = FFT_ST, C = FFT_ZCOLS;
    __shared__ float2 a[C * ST], b[C * ST], twl[G / 2];
    __shared__ float ml[C][G / 2];  // the columns' multipliers by |kz| (h + 1 <= G / 2)
    const int h = fa.N / 2, KX = fa.KX, H = h + 1;
    const int ncol = (fa.N + 1) * KX, rowlen = ncol;
    const int c0 = blockIdx.x * C;
    const int nc = min(C, ncol - c0);
    // column data, twiddles and the columns' multipliers, all loads in flight before the first
    // store to LDS
    constexpr int NT = 64, PT = C * G / NT, MT = C * (G / 2) / NT;
    float2 v[PT];
    float mv[MT];
#pragma unroll
    for (int i = 0; i < PT; ++i) {
        const int q = threadIdx.x + i * NT, zi = q / C, c = q % C;
        v[i] = (c < nc) ? S[(int64_t)zi * rowlen + c0 + c] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int i = 0; i < MT; ++i) {
        const int q = threadIdx.x + i * NT, c = q / (G / 2), akz = q % (G / 2);
        const int col = min(c0 + c, ncol - 1);
        const int kyb = col / KX, kx = col % KX;
        const int aky = kyb >= h ? kyb - h : h - kyb;
        mv[i] = (akz < H) ? M[((int64_t)akz * H + aky) * H + kx] : 0.0f;
    }
    const float2 tv = tw[threadIdx.x & (G / 2 - 1)];
#pragma unroll
    for (int i = 0; i < PT; ++i) {
        const int q = threadIdx.x + i * NT;
        a[(q % C) * ST + q / C] = v[i];
    }
#pragma unroll
    for (int i = 0; i < MT; ++i) {
        const int q = threadIdx.x + i * NT;
        ml[q / (G / 2)][q % (G / 2)] = mv[i];
    }
    if (threadIdx.x < G / 2) twl[threadIdx.x] = tv;
    __syncthreads();
    lds_fft64_out<-1, ST>(a, b, C, twl, [&](int c, int zi, float2 v) {
        const int kz = (zi <= G / 2) ? zi : zi - G;
        const int akz = kz < 0 ? -kz : kz;
        const float mk = (akz <= h) ? ml[c][akz] : 0.0f;
        a[c * ST + zi] = make_float2(v.x * mk, v.y * mk);
    });
    lds_fft64_out<1, ST>(a, b, C, twl, [&](int c, int zo, float2 v) {
        if (c < nc) S[(int64_t)zo * rowlen + c0 + c] = v;
    });
}

__global__ void __launch_bounds__(256) k_fft_xy_inv64(const float2 *__restrict__ S, FftArgs fa,
                                                      const float2 *__restrict__ tw,
                                                      float *__restrict__ grid) {
    constexpr int G = 64, ST = FFT_ST;
    __shared__ float2 a[(G / 2) * ST], b[(G / 2) * ST], twl[G / 2];
    const int h = fa.N / 2, KX = fa.KX, NB1 = fa.N + 1;
    const int z = blockIdx.x;
    const float2 *in = S + (int64_t)z * NB1 * KX;
    // a[kx][y frequency]: the band, zeros elsewhere (kx < G / 2; all loads in flight before the
    // first store to LDS)
    constexpr int NT = 256, PT = (G / 2) * G / NT;
    float2 v[PT];
#pragma unroll
    for (int i = 0; i < PT; ++i) {
        const int q = threadIdx.x + i * NT, kx = q / G, yi = q % G;
        const int ky = (yi <= G / 2) ? yi : yi - G;
        v[i] = (kx < KX && ky >= -h && ky <= h) ? in[(ky + h) * KX + kx] : make_float2(0.f, 0.f);
    }
    const float2 tv = tw[threadIdx.x & (G / 2 - 1)];
#pragma unroll
    for (int i = 0; i < PT; ++i) {
        const int q = threadIdx.x + i * NT;
        if (q / G < KX) a[(q / G) * ST + q % G] = v[i];
    }
    if (threadIdx.x < G / 2) twl[threadIdx.x] = tv;
    __syncthreads();
    lds_fft64<1, ST>(a, b, KX, twl);
    // rows 2t, 2t + 1 as one complex row: A + i B at kx <= h, their conjugates at G - kx
    for (int q = threadIdx.x; q < (G / 2) * G; q += blockDim.x) {
        const int t = q / G, k = q % G;
        float2 zz = make_float2(0.f, 0.f);
        if (k <= h) {
            const float2 A = a[k * ST + 2 * t], B = a[k * ST + 2 * t + 1];
            zz = make_float2(A.x - B.y, A.y + B.x);
        } else if (k >= G - h) {
            const int kk = G - k;
            const float2 A = a[kk * ST + 2 * t], B = a[kk * ST + 2 * t + 1];
            zz = make_float2(A.x + B.y, -A.y + B.x);
        }
        b[t * ST + k] = zz;
    }
    __syncthreads();
    float *slab = grid + (int64_t)z * G * G;
    lds_fft64_out<1, ST>(b, a, G / 2, twl, [&](int t, int i, float2 v) {
        slab[(2 * t) * G + i] = v.x;
        slab[(2 * t + 1) * G + i] = v.y;
    });
}

// ------------------------------------------------------------------ gather (NFFT)
template <int D, int W, int T, bool GRAD>
__global__ void __launch_bounds__(256) k_gather(const float4 *__restrict__ rec,
                                                const int4 *__restrict__ chunks, SpreadArgs sa,
                                                const float *__restrict__ grid,
                                                float *__restrict__ out, float *__restrict__ gout,
                                                float gscale) {
    constexpr int S = T + W - 1;
    constexpr int BOX = (D == 1) ? S : (D == 2 ? S * S : S * S * S);
    __shared__ float box[BOX];
    const int4 ch = chunks[blockIdx.x];
    int tc[3] = {0, 0, 0};
    tile_coords<D>(ch.x, sa.ntd, tc);
    const int G = sa.G;
    for (int q = threadIdx.x; q < BOX; q += blockDim.x) {
        int l0 = q % S, l1 = (q / S) % S, l2 = q / (S * S);
        int g0 = (tc[0] * T - (sa.m - 1) + l0 + G) & (G - 1);
        int64_t gi = g0;
        if (D > 1) gi += (int64_t)G * ((tc[1] * T - (sa.m - 1) + l1 + G) & (G - 1));
        if (D > 2) gi += (int64_t)G * G * ((tc[2] * T - (sa.m - 1) + l2 + G) & (G - 1));
        box[q] = grid[gi];
    }
    __syncthreads();
    // this workgroup's share of the chunk (gridDim.y workgroups per chunk)
    const int per = (ch.z + (int)gridDim.y - 1) / (int)gridDim.y;
    const int kb = ch.y + (int)blockIdx.y * per, ke = min(ch.y + ch.z, kb + per);
    for (int k = kb + threadIdx.x; k < ke; k += blockDim.x) {
        const float4 r = rec[k];
        const int lb = __float_as_int(r.w);  // cell offset inside the tile's box
        const float fr[3] = {r.x, r.y, r.z};
        float wx[W], dwx[W];
        const float ux = 2.0f * fr[0] - 1.0f;
#pragma unroll
        for (int a = 0; a < W; ++a) {
            wx[a] = wpoly_eval(sa.wp + a * WPOLY, ux);
            if (GRAD) dwx[a] = wpoly_eval(sa.wp + (W + a) * WPOLY, ux);
        }
        float val = 0.0f, g0 = 0.0f, g1 = 0.0f, g2 = 0.0f;
        if (D == 1) {
#pragma unroll
            for (int a = 0; a < W; ++a) {
                val = fmaf(wx[a], box[lb + a], val);
                if (GRAD) g0 = fmaf(dwx[a], box[lb + a], g0);
            }
        } else {
            float wy[W], dwy[W];
            const float uy = 2.0f * fr[1] - 1.0f;
#pragma unroll
            for (int b = 0; b < W; ++b) {
                wy[b] = wpoly_eval(sa.wp + b * WPOLY, uy);
                if (GRAD) dwy[b] = wpoly_eval(sa.wp + (W + b) * WPOLY, uy);
            }
            const int nz = (D == 3) ? W : 1;
            for (int l = 0; l < nz; ++l) {
                float wz = 1.0f, dwz = 0.0f;
                int zb = 0;
                if (D == 3) {
                    const float uz = 2.0f * fr[2] - 1.0f;
                    wz = wpoly_eval(sa.wp + l * WPOLY, uz);
                    if (GRAD) dwz = wpoly_eval(sa.wp + (W + l) * WPOLY, uz);
                    zb = l * S * S;
                }
                float pv = 0.0f, pgx = 0.0f, pgy = 0.0f;
#pragma unroll
                for (int b = 0; b < W; ++b) {
                    const float *row = box + lb + zb + b * S;
                    float rv = 0.0f, rg = 0.0f;
#pragma unroll
                    for (int a = 0; a < W; ++a) {
                        const float hv = row[a];
                        rv = fmaf(wx[a], hv, rv);
                        if (GRAD) rg = fmaf(dwx[a], hv, rg);
                    }
                    pv = fmaf(wy[b], rv, pv);
                    if (GRAD) {
                        pgx = fmaf(wy[b], rg, pgx);
                        pgy = fmaf(dwy[b], rv, pgy);
                    }
                }
                val = fmaf(wz, pv, val);
                if (GRAD) {
                    g0 = fmaf(wz, pgx, g0);
                    g1 = fmaf(wz, pgy, g1);
                    if (D == 3) g2 = fmaf(dwz, pv, g2);
                }
            }
        }
        out[k] = val;
        if (GRAD) {
            gout[(int64_t)k * D] = g0 * gscale;
            if (D > 1) gout[(int64_t)k * D + 1] = g1 * gscale;
            if (D > 2) gout[(int64_t)k * D + 2] = g2 * gscale;
        }
    }
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

// Two FP32 values as FP16 pairs v = hi + lo: hi = v rounded to FP16, lo = the remainder rounded
// to FP16 (about 22 significant bits together for values in FP16's normal range).
__device__ __forceinline__ void split_f16(float a, float b, f16x2 &hi, f16x2 &lo) {
    hi = __builtin_convertvector(f32x2{a, b}, f16x2);
    const f32x2 back = __builtin_convertvector(hi, f32x2);
    lo = __builtin_convertvector(f32x2{a - back.x, b - back.y}, f16x2);
}

// 3-D spreading on the matrix cores in moment form.  Each window segment is a degree-(WPOLY-1)
// polynomial in u = 2t - 1 (t the node's offset inside its cell); in the Chebyshev basis,
// phi_n[y] = sum_k C[y][k] T_k(u_n), so the (y, z) factor of a node's window is C (x) C applied to
// the WPOLY^2 products Ty_n[k] Tz_n[l].  The nodes of one brick (BRICK_X cells along x with the
// same y and z cell) share that transform, so the kernel accumulates their moments
//   M[(k, l)][x] += sum_n Ty_n[k] Tz_n[l] (alpha_n px_n[x - ox_n])      (per group: 64 x 16)
// (alpha the weights divided by the block's largest |weight|, px the x window, ox the node's
// cell inside the brick) and, when the brick changes, adds
//   H[(y, z)][x] = sum_(k,l) C[y][k] C[z][l] M[(k, l)][x]
// to the block's LDS box as int32 fixed point (scale 2^30 / (count max|w|)).  Both products run on
// v_mfma_f32_16x16x32_f16 with every FP32 factor carried as a pair of FP16 numbers, v = hi + lo
// (hi = v rounded to FP16, lo = the remainder rounded to FP16, about 22 significant bits together):
// per group, lane l holds nodes 4 (l / 16) .. + 3 as K elements, (hi, lo) of the moment products
// for row q = 16 j + l % 16 against (hi, hi) and then (lo, lo) of alpha px at column x = l % 16
// (two products per block j of 16 moment rows).  The accumulator layout of M (row
// 16 j + 4 (l / 16) + r, column l % 16) is the B-operand layout of the second product, so the
// moments never leave the registers; its constant operand (sa.cc, copied to LDS) holds hi and lo
// of C[y][k] C[z][l] for two K steps each, and three products per pair of steps sum hi hi, lo hi
// and hi lo.  A group thus costs 64 instead of W^2 window products and splits on the VALU, and only
// the x window is evaluated per node.
template <int W, bool POT>
__global__ void __launch_bounds__(64 * MW) __attribute__((amdgpu_waves_per_eu(4, 4)))
k_spread_mom16(const float4 *__restrict__ rec, const float *__restrict__ w,
               const int4 *__restrict__ mblocks, const int4 *__restrict__ mgroups,
               const int2 *__restrict__ mbnodes, SpreadArgs sa, float *__restrict__ scratch,
               PotWeights pw) {
    constexpr int T = 8, S = T + W - 1, BOX = S * S * S;
    constexpr int NZ = (W + 3) / 4;      // (y, z) offsets in blocks of 4
    constexpr int NB = NZ * NZ;          // 4 x 4 blocks of (y, z)
    constexpr int XR = W + BRICK_X - 1;  // box columns a brick reaches
    constexpr int PX = W + 1;            // row stride of the x table (odd: no bank conflicts)
    constexpr int PD = WPOLY;            // Chebyshev terms per axis
    constexpr int NJ = PD * PD / 16;     // moment row blocks
    constexpr int NP = NJ / 2;           // K-step pairs of the transform
    constexpr int NCC = NB * NP * 2 * 64;                 // transform operands
    constexpr int CPT = (NCC + 64 * MW - 1) / (64 * MW);  // of them per thread
    static_assert(XR <= 16, "brick and window exceed the 16 matrix rows");
    static_assert(PD == 8, "moment layout assumes 8 Chebyshev terms");
    __shared__ int box[BOX];
    __shared__ uint4 cct[NCC];               // copy of sa.cc
    __shared__ float phx[MW][16 * PX];       // per wave: alpha px, node-major
    __shared__ float4 tyz[MW][2][16][2];     // per wave, axis, node: T_0,2,4,6 then T_1,3,5,7
    __shared__ int4 oxs[MW][4];              // per wave: x cell offsets of the 16 nodes
    __shared__ double red2[2][MW];
    const int4 mb = mblocks[blockIdx.x];
    const int2 kn = mbnodes[blockIdx.x];
    const int k0 = kn.x, cnt = kn.y;
    uint4 ccv[CPT];
#pragma unroll
    for (int i = 0; i < CPT; ++i) ccv[i] = sa.cc[min((int)threadIdx.x + i * 64 * MW, NCC - 1)];
    for (int q = threadIdx.x; q < BOX; q += blockDim.x) box[q] = 0;
    // the block's largest |weight| in one pass: with potentials, w_k = base_k
    // exp((pot_k - pmax) / eps), so max_k |w_k| = exp(max_k (log |base_k| + pot_k / eps) -
    // pmax / eps), and the largest potential pmax is reduced alongside
    double m0 = -INFINITY, m1 = -INFINITY;
    // (node data read in batches of 8 per thread, all in flight before the first use)
    constexpr int PB = 8;
    if (POT)
        for (int b = threadIdx.x; b < pw.nparts; b += blockDim.x) m0 = fmax(m0, pw.parts[b]);
    // with per-block maxima of the potential and of |base|, their sum bounds the block's largest
    // log-weight and the block's nodes need not be read here
    const bool bounded = POT && pw.bbase != nullptr;
    if (bounded && threadIdx.x == 0)
        m1 = pw.parts[blockIdx.x] * pw.inv_eps + (double)logf(pw.bbase[blockIdx.x]);
    for (int q0 = k0 + threadIdx.x; !bounded && q0 < k0 + cnt; q0 += PB * 64 * MW) {
        double pv[PB];
        float bv[PB];
#pragma unroll
        for (int i = 0; i < PB; ++i) {
            const int q = q0 + i * 64 * MW;
            const bool in = q < k0 + cnt;
            if (POT) {
                pv[i] = in ? pw.pot[q] : -INFINITY;
                bv[i] = in ? pw.base[q] : 1.0f;
            } else {
                bv[i] = in ? w[q] : 0.0f;
            }
        }
#pragma unroll
        for (int i = 0; i < PB; ++i)
            m1 = POT ? fmax(m1, pv[i] * pw.inv_eps + (double)logf(fabsf(bv[i])))
                     : fmax(m1, (double)fabsf(bv[i]));
    }
    for (int o = 32; o > 0; o >>= 1) {
        m0 = fmax(m0, __shfl_xor(m0, o, 64));
        m1 = fmax(m1, __shfl_xor(m1, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        red2[0][threadIdx.x >> 6] = m0;
        red2[1][threadIdx.x >> 6] = m1;
    }
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
        const int q = threadIdx.x + i * 64 * MW;
        if (q < NCC) cct[q] = ccv[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MW; ++i) {
        m0 = fmax(m0, red2[0][i]);
        m1 = fmax(m1, red2[1][i]);
    }
    const double pmax = (m0 == -INFINITY) ? 0.0 : m0;
    float wm = 0.0f;
    if (POT) wm = (m1 == -INFINITY) ? 0.0f : weight_exp(1.0f, m1 - pmax * pw.inv_eps);
    else wm = (m1 > 0.0) ? (float)m1 : 0.0f;
    const float scale = (wm > 0.0f && cnt > 0) ? 1073741824.0f / ((float)cnt * wm) : 1.0f;
    const float wmax = (wm > 0.0f) ? wm : 1.0f;
    const float inv_wmax = 1.0f / wmax;
    const float mscale = scale * wmax * (1.0f / (float)(1 << MOM_CC_SHIFT));
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int col = lane & 15, slot = lane >> 4;
    float wc[NZ][WPOLY];
#pragma unroll
    for (int e = 0; e < NZ; ++e) {
        const int a = slot + 4 * e;
#pragma unroll
        for (int k = 0; k < WPOLY; ++k) wc[e][k] = (a < W) ? sa.wp[a * WPOLY + k] : 0.0f;
    }
    float *px = phx[wave];
    float4(*tt)[16][2] = tyz[wave];
    int *ox = reinterpret_cast<int *>(oxs[wave]);
    const int per = (mb.z + MW - 1) / MW;
    const int gb = mb.y + wave * per, ge = min(mb.y + mb.z, gb + per);
    f32x4 acc[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    int cur = -1;
    auto flush = [&]() {
        // moments times fscale 2^-MOM_CC_SHIFT, at most 2^15 in magnitude, as B operands: K
        // elements of steps 2 sp and 2 sp + 1 side by side, hi and lo parts apart (the lo x lo
        // product is dropped: it is below the split's own rounding)
        f16x8 Bh[NP], Bl[NP];
#pragma unroll
        for (int sp = 0; sp < NP; ++sp) {
            f16x2 h0, l0, h1, l1, h2, l2, h3, l3;
            split_f16(acc[2 * sp][0] * mscale, acc[2 * sp][1] * mscale, h0, l0);
            split_f16(acc[2 * sp][2] * mscale, acc[2 * sp][3] * mscale, h1, l1);
            split_f16(acc[2 * sp + 1][0] * mscale, acc[2 * sp + 1][1] * mscale, h2, l2);
            split_f16(acc[2 * sp + 1][2] * mscale, acc[2 * sp + 1][3] * mscale, h3, l3);
            Bh[sp] = f16x8{h0[0], h0[1], h1[0], h1[1], h2[0], h2[1], h3[0], h3[1]};
            Bl[sp] = f16x8{l0[0], l0[1], l1[0], l1[1], l2[0], l2[1], l3[0], l3[1]};
        }
#pragma unroll
        for (int j = 0; j < NJ; ++j) acc[j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        const int x = col;
#pragma unroll
        for (int jb = 0; jb < NB; ++jb) {
            f32x4 h = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int sp = 0; sp < NP; ++sp) {
                const f16x8 Ah = __builtin_bit_cast(f16x8, cct[((jb * NP + sp) * 2 + 0) * 64 + lane]);
                const f16x8 Al = __builtin_bit_cast(f16x8, cct[((jb * NP + sp) * 2 + 1) * 64 + lane]);
                h = __builtin_amdgcn_mfma_f32_16x16x32_f16(Ah, Bh[sp], h, 0, 0, 0);
                h = __builtin_amdgcn_mfma_f32_16x16x32_f16(Al, Bh[sp], h, 0, 0, 0);
                h = __builtin_amdgcn_mfma_f32_16x16x32_f16(Ah, Bl[sp], h, 0, 0, 0);
            }
            // h[r] = H[(y, z)][x] with y = 4 (jb / NZ) + slot, z = 4 (jb % NZ) + r
            const int y = 4 * (jb / NZ) + slot;
            if (x < XR && (W % 4 == 0 || y < W)) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int z = 4 * (jb % NZ) + r;
                    if (W % 4 == 0 || z < W)
                        atomicAdd(&box[cur + y * S + z * S * S + x], __float2int_rn(h[r]));
                }
            }
        }
    };
    // software pipeline: while group g is processed, the node data of g + 1 and the group
    // record of g + 2 are in flight (the chain group record -> node record -> weight inputs
    // would otherwise stall every group)
    const int4 gnone = int4{0, 1, -1, 0};
    int4 g1 = (gb < ge) ? mgroups[gb] : gnone;
    int4 g2 = (gb + 1 < ge) ? mgroups[gb + 1] : gnone;
    float4 r1 = float4{0.0f, 0.0f, 0.0f, 0.0f};
    if (gb < ge) r1 = rec[g1.x + min(col, g1.y - 1)];
    // weights four groups at a time: lane slot s evaluates the weight of node `col` of group
    // gq + s (the exponential once per node instead of once per lane), and a group takes its
    // weights from the lanes of its slot by a shuffle; the node data of the next four groups is
    // loaded a batch ahead
    float bq = 0.0f;
    double pq = 0.0;
    auto fetchw = [&](int g0) {
        const int gg = g0 + slot;
        bq = 0.0f;
        pq = 0.0;
        if (gg < ge) {
            const int4 q = mgroups[gg];
            const int kk = q.x + min(col, q.y - 1);
            if (POT) {
                bq = pw.base[kk];
                pq = pw.pot[kk];
            } else {
                bq = w[kk];
            }
        }
    };
    auto weight = [&]() -> float {
        return POT ? weight_exp(bq, (pq - pmax) * pw.inv_eps) : bq;
    };
    int gq = gb;
    fetchw(gb);
    float wq = weight();
    fetchw(gb + 4);
    for (int g = gb;; ++g) {
        // one flush site: the pass after the last group flushes the last brick
        const int gz = (g < ge) ? g1.z : -1;
        if (gz != cur) {
            if (cur >= 0) flush();
            cur = gz;
        }
        if (g >= ge) break;
        const int4 gr = g1;
        const float4 r = r1;
        if (g - gq == 4) {
            gq = g;
            wq = weight();
            fetchw(g + 4);
        }
        const float wv = __shfl(wq, (g - gq) * 16 + col, 64);
        g1 = g2;
        if (g + 1 < ge) r1 = rec[g1.x + min(col, g1.y - 1)];
        g2 = (g + 2 < ge) ? mgroups[g + 2] : gnone;
        const float alpha = (col < gr.y) ? wv * inv_wmax : 0.0f;
        // x window values of node `col` at offsets slot + 4 e
#pragma unroll
        for (int e = 0; e < NZ; ++e) {
            const int a = slot + 4 * e;
            if (W % 4 == 0 || a < W) px[col * PX + a] = alpha * wpoly_eval(wc[e], 2.0f * r.x - 1.0f);
        }
        // Chebyshev values T_k(u) of the offsets: slots 0, 1 take y and slots 2, 3 take z; the
        // slot's parity picks the even or the odd degrees
        {
            const int axis = slot >> 1;
            const float u = 2.0f * (axis ? r.z : r.y) - 1.0f;
            float t[PD];
            t[0] = 1.0f;
            t[1] = u;
#pragma unroll
            for (int q = 2; q < PD; ++q) t[q] = fmaf(2.0f * u, t[q - 1], -t[q - 2]);
            tt[axis][col][slot & 1] = (slot & 1) ? float4{t[1], t[3], t[5], t[7]}
                                                 : float4{t[0], t[2], t[4], t[6]};
        }
        if (slot == 0) ox[col] = __float_as_int(r.w) % S - gr.z % S;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // operand B: alpha px of nodes 4 slot .. + 3 at box column `col`, (hi, lo) repeated
        const int4 o4 = oxs[wave][slot];
        const int oxn[4] = {o4.x, o4.y, o4.z, o4.w};
        float av[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int n = 4 * slot + e;
            const int a = col - oxn[e];
            av[e] = (a >= 0 && a < W) ? px[n * PX + (a < 0 ? 0 : (a >= W ? W - 1 : a))] : 0.0f;
        }
        f16x2 ah0, al0, ah1, al1;
        split_f16(av[0], av[1], ah0, al0);
        split_f16(av[2], av[3], ah1, al1);
        const f16x8 P1 = {ah0[0], ah0[1], ah1[0], ah1[1], ah0[0], ah0[1], ah1[0], ah1[1]};
        const f16x8 P2 = {al0[0], al0[1], al1[0], al1[1], al0[0], al0[1], al1[0], al1[1]};
        // operand A per moment block j: Ty[k] Tz[l] of nodes 4 slot .. + 3 for moment row
        // q = 16 j + col (k = q / 8 = 2 j + col / 8, l = col % 8), (hi, lo)
        const int kc = col >> 3, l = col & 7;
        f32x4 tyv[4];
        float tzv[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float4 yv = tt[0][4 * slot + e][kc];
            tyv[e] = f32x4{yv.x, yv.y, yv.z, yv.w};
            tzv[e] = reinterpret_cast<const float *>(tt[1][4 * slot + e])[(l & 1) * 4 + (l >> 1)];
        }
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            f16x2 bh0, bl0, bh1, bl1;
            split_f16(tyv[0][j] * tzv[0], tyv[1][j] * tzv[1], bh0, bl0);
            split_f16(tyv[2][j] * tzv[2], tyv[3][j] * tzv[3], bh1, bl1);
            const f16x8 A = {bh0[0], bh0[1], bh1[0], bh1[1], bl0[0], bl0[1], bl1[0], bl1[1]};
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A, P1, acc[j], 0, 0, 0);
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A, P2, acc[j], 0, 0, 0);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    __syncthreads();
    const float inv = 1.0f / scale;
    float *dst = scratch + (int64_t)blockIdx.x * BOX;
    for (int q = threadIdx.x; q < BOX; q += blockDim.x) dst[q] = (float)box[q] * inv;
}

// 3-D gather on the FP16 matrix cores with split operands.  For the nodes n of one brick
// (BRICK_X cells along x with the same y and z cell), px, py, pz their window values and ox their
// cell's x offset inside the brick,
//   t_n = sum_{y,z} py_n[y] pz_n[z] E_y[z][n],   E_y[z][n] = sum_x H[x][y][z] px_n[x - ox_n],
// x over 16 box columns from the brick's first cell.  Every factor of E is carried as a pair of
// FP16 numbers, v = hi + lo (hi = v rounded to FP16, lo = the remainder rounded to FP16, about 22
// significant bits together), and the four products hi hi, lo hi, hi lo, lo lo are summed in FP32
// by two v_mfma_f32_16x16x32_f16 per y.  Lane l covers the columns x = 4 (l / 16) .. + 3: its
// eight K elements are (hi, lo) of H at those columns against (hi, hi) of px in the first product
// and (lo, lo) in the second.  The box is kept in LDS in the same order (per row of x: groups of
// four columns, high parts then low parts, 16 bytes), scaled by a power of two so that its largest
// value is about 2^14 (no FP16 overflow; the lost low bits are below 2^-39 of the largest value).
// Lane l then holds E_y[4 (l / 16) + r][l % 16] and forms the y, z sums for node l % 16 over its
// four rows.  With UPD the sums are not stored; the potential update (PotUpdate) is applied to
// them and each workgroup writes its maxima.
template <int W, bool UPD>
__global__ void __launch_bounds__(64 * MW) k_gather_mfma16(const float4 *__restrict__ rec,
                                                       const int4 *__restrict__ mblocks,
                                                       const int4 *__restrict__ mgroups,
                                                       SpreadArgs sa,
                                                       const float *__restrict__ grid,
                                                       float *__restrict__ out, PotUpdate pu) {
    constexpr int T = 8, S = T + W - 1, BOX = S * S * S;
    constexpr int NC = 5;  // groups of 4 columns per row: x < 20 covers 4 + 16 columns
    constexpr int NZ = (W + 3) / 4;
    constexpr int NT = 64 * MW;
    constexpr int PER = (BOX + NT - 1) / NT;
    static_assert(W + BRICK_X - 1 <= 16 && S <= 4 * NC, "brick and window exceed the 16 columns");
    __shared__ __align__(16) _Float16 bx[S * S][NC][8];
    __shared__ float phi[MW][3][W][16];
    __shared__ float red[MW];
    __shared__ double dred[MW];
    const int4 mb = mblocks[blockIdx.x];
    int tc[3];
    tile_coords<3>(mb.x, sa.ntd, tc);
    const int G = sa.G;
    // the largest of the shift maxima (read together with the box)
    double sv = -INFINITY;
    if (UPD)
        for (int b = threadIdx.x; b < pu.nshift; b += blockDim.x) sv = fmax(sv, pu.shift_parts[b]);
    // the tile's box: values and their largest magnitude
    float v[PER];
    float mx = 0.0f;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int q = threadIdx.x + NT * i;
        v[i] = 0.0f;
        if (q < BOX) {
            const int l0 = q % S, l1 = (q / S) % S, l2 = q / (S * S);
            const int g0 = (tc[0] * T - (sa.m - 1) + l0 + G) & (G - 1);
            const int g1 = (tc[1] * T - (sa.m - 1) + l1 + G) & (G - 1);
            const int g2 = (tc[2] * T - (sa.m - 1) + l2 + G) & (G - 1);
            v[i] = grid[((int64_t)g2 * G + g1) * G + g0];
            mx = fmaxf(mx, fabsf(v[i]));
        }
    }
    for (int off = 32; off >= 1; off >>= 1) {
        mx = fmaxf(mx, __shfl_xor(mx, off, 64));
        if (UPD) sv = fmax(sv, __shfl_xor(sv, off, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6] = mx;
        dred[threadIdx.x >> 6] = sv;
    }
    // columns x >= S of every row are zero
    for (int q = threadIdx.x; q < S * S * (4 * NC - S); q += NT) {
        const int row = q / (4 * NC - S), x = S + q % (4 * NC - S);
        bx[row][x >> 2][x & 3] = (_Float16)0.0f;
        bx[row][x >> 2][4 + (x & 3)] = (_Float16)0.0f;
    }
    __syncthreads();
    mx = red[0];
    for (int i = 1; i < MW; ++i) mx = fmaxf(mx, red[i]);
    double shift = 0.0;
    if (UPD) {
        for (int i = 0; i < MW; ++i) sv = fmax(sv, dred[i]);
        shift = (sv == -INFINITY) ? 0.0 : sv;
    }
    // power-of-two scale: largest |value| in [2^13, 2^14)
    int ex = 0;
    frexpf(mx, &ex);
    const float scale = (mx > 0.0f) ? ldexpf(1.0f, 14 - ex) : 1.0f;
    const float unscale = (mx > 0.0f) ? ldexpf(1.0f, ex - 14) : 1.0f;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int q = threadIdx.x + NT * i;
        if (q < BOX) {
            const float u = v[i] * scale;
            const _Float16 h = (_Float16)u;
            const int row = q / S, x = q % S;
            bx[row][x >> 2][x & 3] = h;
            bx[row][x >> 2][4 + (x & 3)] = (_Float16)(u - (float)h);
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int node = lane & 15, slot = lane >> 4;
    double pmx = -INFINITY, dmx = 0.0;
    int bad = 0;
    float wc[NZ][WPOLY];
#pragma unroll
    for (int e = 0; e < NZ; ++e) {
        const int a = slot + 4 * e;
#pragma unroll
        for (int k = 0; k < WPOLY; ++k) wc[e][k] = (a < W) ? sa.wp[a * WPOLY + k] : 0.0f;
    }
    float(*ph)[W][16] = phi[wave];
    const int per = (mb.z + MW - 1) / MW;
    const int gb = mb.y + wave * per, ge = min(mb.y + mb.z, gb + per);
    // the sums of four consecutive groups wait in registers, one group per lane slot, and are
    // stored (with the update) by all 64 lanes at once
    float tq = 0.0f;
    int kq = -1, nq = 0;
    auto commit = [&]() {
        if (kq >= 0) {
            float t = tq;
            if (!UPD) {
                out[kq] = t;
            } else {
                if (!(t > 0.0f)) {
                    ++bad;
                    t = FLT_MIN;
                }
                const double f = -pu.kappa * (shift + pu.eps * sum_log(t));
                if (pu.delta_parts) dmx = fmax(dmx, fabs(f - pu.pot[kq]));
                pu.pot[kq] = f;
                pmx = fmax(pmx, f);
            }
        }
        kq = -1;
    };
    int4 grn = make_int4(0, 1, 0, 0);
    float4 rn = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (gb < ge) {
        grn = mgroups[gb];
        rn = rec[grn.x + min(node, grn.y - 1)];
    }
    for (int g = gb; g < ge; ++g) {
        const int4 gr = grn;
        const float4 r = rn;
        if (g + 1 < ge) {
            grn = mgroups[g + 1];
            rn = rec[grn.x + min(node, grn.y - 1)];
        }
        const float fr[3] = {r.x, r.y, r.z};
#pragma unroll
        for (int dim = 0; dim < 3; ++dim) {
            const float u = 2.0f * fr[dim] - 1.0f;
#pragma unroll
            for (int e = 0; e < NZ; ++e) {
                const int a = slot + 4 * e;
                if (W % 4 == 0 || a < W) ph[dim][a][node] = wpoly_eval(wc[e], u);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int cur = gr.z;
        const int cx0 = cur % S, cy = (cur / S) % S, cz = cur / (S * S);
        const int ox = __float_as_int(r.w) % S - cx0;  // the node's x cell inside the brick
        // operand B: px of node `node` at x = 4 slot .. + 3 as (hi, hi) and (lo, lo)
        f16x8 B1, B2;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int a = 4 * slot + e - ox;
            const float pv = (a >= 0 && a < W) ? ph[0][a < 0 ? 0 : (a >= W ? W - 1 : a)][node] : 0.0f;
            const _Float16 h = (_Float16)pv;
            const _Float16 l = (_Float16)(pv - (float)h);
            B1[e] = h;
            B1[4 + e] = h;
            B2[e] = l;
            B2[4 + e] = l;
        }
        float pz[4], py[W];
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int z = 4 * slot + rr;
            pz[rr] = (z < W) ? ph[2][z < W ? z : W - 1][node] : 0.0f;
        }
#pragma unroll
        for (int y = 0; y < W; ++y) py[y] = ph[1][y][node];
        // operand A: row z = lane % 16 (rows at or beyond W read row W - 1; their pz is zero)
        const int zr = node < W ? node : W - 1;
        const uint4 *arow = reinterpret_cast<const uint4 *>(&bx[(cz + zr) * S + cy][(cx0 >> 2) + slot][0]);
        f32x4 ty = {0.0f, 0.0f, 0.0f, 0.0f};  // sum over y of py E_y, per row
#pragma unroll
        for (int y = 0; y < W; ++y) {
            const f16x8 A = __builtin_bit_cast(f16x8, arow[y * NC]);
            f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(A, B1, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(A, B2, acc, 0, 0, 0);
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) ty[rr] = fmaf(py[y], acc[rr], ty[rr]);
        }
        float part = 0.0f;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) part = fmaf(pz[rr], ty[rr], part);
        part += __shfl_xor(part, 16, 64);
        part += __shfl_xor(part, 32, 64);
        // every lane of column `node` now holds the node's sum; slot nq keeps it
        if (slot == nq) {
            tq = part * unscale;
            kq = (node < gr.y) ? gr.x + node : -1;
        }
        if (++nq == 4) {
            commit();
            nq = 0;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    commit();
    if (UPD) {
        if (bad) atomicAdd(pu.nbad, bad);
        pmx = block_max_f64(pmx, dred);
        if (threadIdx.x == 0) pu.out_parts[blockIdx.x] = pmx;
        if (pu.delta_parts) {
            dmx = block_max_f64(dmx, dred);
            if (threadIdx.x == 0) pu.delta_parts[blockIdx.x] = dmx;
        }
    }
}

// 2-D spreading on the FP16 matrix cores.  For the nodes of one brick (BRICK_X cells along x with
// the same y cell), with alpha the weights divided by the block's largest |weight|,
//   H[x][y] += sum_n (alpha_n px_n[x - ox_n]) py_n[y],
// x over 16 box columns from the brick's first cell, y over the W rows from its cell: a plain
// rank-16 product of the two window factors, two v_mfma_f32_16x16x32_f16 per group with both
// factors split into FP16 hi + lo (as in the 3-D spread, whose y-z products are replaced here by
// py itself).  Lane l holds H[4 (l / 16) + r][l % 16]; the sums stay in registers while the brick
// stays the same and then go to the block's int32 LDS box (fixed point, see chunk_scale).  With
// POT the weights are formed from the potentials (weight_exp), as in the 3-D spread.
template <int W, int T, bool POT>
__global__ void __launch_bounds__(64 * MW) k_spread_mfma2d(const float4 *__restrict__ rec,
                                                       const float *__restrict__ w,
                                                       const int4 *__restrict__ mblocks,
                                                       const int4 *__restrict__ mgroups,
                                                       const int2 *__restrict__ mbnodes,
                                                       SpreadArgs sa, float *__restrict__ scratch,
                                                       PotWeights pw) {
    constexpr int S = T + W - 1, BOX = S * S;
    constexpr int NZ = (W + 3) / 4;      // window offsets per lane: slot + 4 e
    constexpr int XR = W + BRICK_X - 1;  // box columns a brick reaches
    constexpr int PX = W + 1;            // row stride of the x table (odd: no bank conflicts)
    static_assert(XR <= 16, "brick and window exceed the 16 matrix rows");
    __shared__ int box[BOX];
    __shared__ float phx[MW][16 * PX];  // per wave: alpha px, node-major
    __shared__ float phy[MW][W][16];    // per wave: py, offset-major
    __shared__ int oxs[MW][16];
    __shared__ float red[16];
    __shared__ double pmx[MW];
    const int4 mb = mblocks[blockIdx.x];
    for (int q = threadIdx.x; q < BOX; q += blockDim.x) box[q] = 0;
    const int2 kn = mbnodes[blockIdx.x];
    const int k0 = kn.x, cnt = kn.y;
    double pmax = 0.0;
    if (POT) {
        double mx = -INFINITY;
        for (int b = threadIdx.x; b < pw.nparts; b += blockDim.x) mx = fmax(mx, pw.parts[b]);
        mx = block_max_f64(mx, pmx);
        pmax = (mx == -INFINITY) ? 0.0 : mx;
    }
    auto weight = [&](int k) -> float {
        if (POT) return weight_exp(pw.base[k], (pw.pot[k] - pmax) * pw.inv_eps);
        return w[k];
    };
    float wm = 0.0f;
    float scale = 1.0f;
    if (POT && pw.bbase) {
        // per-block maxima of the potential and of |base| bound the block's largest weight
        const double lb = pw.parts[blockIdx.x] * pw.inv_eps + (double)logf(pw.bbase[blockIdx.x]);
        wm = (lb == -INFINITY) ? 0.0f : weight_exp(1.0f, lb - pmax * pw.inv_eps);
        scale = (wm > 0.0f && cnt > 0) ? 1073741824.0f / ((float)cnt * wm) : 1.0f;
    } else {
        scale = chunk_scale_fn(weight, k0, cnt, red, &wm);
    }
    const float wmax = (wm > 0.0f) ? wm : 1.0f;
    const float inv_wmax = 1.0f / wmax, fscale = scale * wmax;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int col = lane & 15, slot = lane >> 4;
    float wc[NZ][WPOLY];
#pragma unroll
    for (int e = 0; e < NZ; ++e) {
        const int a = slot + 4 * e;
#pragma unroll
        for (int k = 0; k < WPOLY; ++k) wc[e][k] = (a < W) ? sa.wp[a * WPOLY + k] : 0.0f;
    }
    float *px = phx[wave];
    float(*py)[16] = phy[wave];
    int *ox = oxs[wave];
    const int per = (mb.z + MW - 1) / MW;
    const int gb = mb.y + wave * per, ge = min(mb.y + mb.z, gb + per);
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    int cur = -1;
    auto flush = [&]() {
        if (col < W) {  // rows y = col >= W hold no window
            const int b0 = cur + col * S;  // row y = col of the brick's box rows
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int x = 4 * slot + r;
                if (x < XR) atomicAdd(&box[b0 + x], __float2int_rn(acc[r] * fscale));
            }
        }
        acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    };
    for (int g = gb; g < ge; ++g) {
        const int4 gr = mgroups[g];
        const int nn = min(col, gr.y - 1);
        const float4 r = rec[gr.x + nn];
        const float alpha = (col < gr.y) ? weight(gr.x + nn) * inv_wmax : 0.0f;
        // window values of node `col` at offsets slot + 4 e
#pragma unroll
        for (int e = 0; e < NZ; ++e) {
            const int a = slot + 4 * e;
            if (W % 4 == 0 || a < W) {
                px[col * PX + a] = alpha * wpoly_eval(wc[e], 2.0f * r.x - 1.0f);
                py[a][col] = wpoly_eval(wc[e], 2.0f * r.y - 1.0f);
            }
        }
        if (slot == 0) ox[col] = __float_as_int(r.w) % S - gr.z % S;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (gr.z != cur) {
            if (cur >= 0) flush();
            cur = gr.z;
        }
        // operand A: alpha px of nodes 4 slot .. + 3 at box column `col`, (hi, lo)
        float av[4], bv[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int n = 4 * slot + e;
            const int a = col - ox[n];
            av[e] = (a >= 0 && a < W) ? px[n * PX + (a < 0 ? 0 : (a >= W ? W - 1 : a))] : 0.0f;
            // operand B: py of the same nodes at box row `col`
            bv[e] = (col < W) ? py[col < W ? col : W - 1][n] : 0.0f;
        }
        f16x2 ah0, al0, ah1, al1, bh0, bl0, bh1, bl1;
        split_f16(av[0], av[1], ah0, al0);
        split_f16(av[2], av[3], ah1, al1);
        split_f16(bv[0], bv[1], bh0, bl0);
        split_f16(bv[2], bv[3], bh1, bl1);
        const f16x8 A1 = {ah0[0], ah0[1], ah1[0], ah1[1], ah0[0], ah0[1], ah1[0], ah1[1]};
        const f16x8 A2 = {al0[0], al0[1], al1[0], al1[1], al0[0], al0[1], al1[0], al1[1]};
        const f16x8 B = {bh0[0], bh0[1], bh1[0], bh1[1], bl0[0], bl0[1], bl1[0], bl1[1]};
        acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(A1, B, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(A2, B, acc, 0, 0, 0);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (cur >= 0) flush();
    __syncthreads();
    const float inv = 1.0f / scale;
    float *dst = scratch + (int64_t)blockIdx.x * BOX;
    for (int q = threadIdx.x; q < BOX; q += blockDim.x) dst[q] = (float)box[q] * inv;
}

// 2-D gather on the FP16 matrix cores, the transpose of k_spread_mfma2d: for the nodes n of one
// brick, t_n = sum_y py_n[y] E[y][n], E[y][n] = sum_x H[x][y] px_n[x - ox_n], x over 16 box
// columns from the brick's first cell.  E is two v_mfma_f32_16x16x32_f16 per group (rows y,
// columns the 16 nodes, K = 16 columns x the hi/lo cross products, the box kept in LDS as in the
// 3-D gather, scaled by a power of two); lane l then holds E[4 (l / 16) + r][l % 16] and forms
// its part of the y sum, the four parts of a node being added across lanes.  With UPD the
// potential update is applied to the sums instead of storing them, as in the 3-D gather.
template <int W, int T, bool UPD>
__global__ void __launch_bounds__(64 * MW) k_gather_mfma2d(const float4 *__restrict__ rec,
                                                       const int4 *__restrict__ mblocks,
                                                       const int4 *__restrict__ mgroups,
                                                       SpreadArgs sa,
                                                       const float *__restrict__ grid,
                                                       float *__restrict__ out, PotUpdate pu) {
    constexpr int S = T + W - 1, BOX = S * S;
    constexpr int NC = (T + 12) / 4;  // groups of 4 columns: the last brick reaches x < T - 4 + 16
    constexpr int NZ = (W + 3) / 4;
    constexpr int NT = 64 * MW;
    constexpr int PER = (BOX + NT - 1) / NT;
    static_assert(W + BRICK_X - 1 <= 16 && S <= 4 * NC, "brick and window exceed the 16 columns");
    __shared__ __align__(16) _Float16 bx[S][NC][8];
    __shared__ float phi[MW][2][W][16];
    __shared__ float red[MW];
    __shared__ double dred[MW];
    const int4 mb = mblocks[blockIdx.x];
    int tc[3];
    tile_coords<2>(mb.x, sa.ntd, tc);
    const int G = sa.G;
    // the largest of the shift maxima (read together with the box)
    double sv = -INFINITY;
    if (UPD)
        for (int b = threadIdx.x; b < pu.nshift; b += blockDim.x) sv = fmax(sv, pu.shift_parts[b]);
    // the tile's box: values and their largest magnitude
    float v[PER];
    float mx = 0.0f;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int q = threadIdx.x + NT * i;
        v[i] = 0.0f;
        if (q < BOX) {
            const int l0 = q % S, l1 = q / S;
            const int g0 = (tc[0] * T - (sa.m - 1) + l0 + G) & (G - 1);
            const int g1 = (tc[1] * T - (sa.m - 1) + l1 + G) & (G - 1);
            v[i] = grid[(int64_t)g1 * G + g0];
            mx = fmaxf(mx, fabsf(v[i]));
        }
    }
    for (int off = 32; off >= 1; off >>= 1) {
        mx = fmaxf(mx, __shfl_xor(mx, off, 64));
        if (UPD) sv = fmax(sv, __shfl_xor(sv, off, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6] = mx;
        dred[threadIdx.x >> 6] = sv;
    }
    // columns x >= S of every row are zero
    for (int q = threadIdx.x; q < S * (4 * NC - S); q += NT) {
        const int row = q / (4 * NC - S), x = S + q % (4 * NC - S);
        bx[row][x >> 2][x & 3] = (_Float16)0.0f;
        bx[row][x >> 2][4 + (x & 3)] = (_Float16)0.0f;
    }
    __syncthreads();
    mx = red[0];
    for (int i = 1; i < MW; ++i) mx = fmaxf(mx, red[i]);
    double shift = 0.0;
    if (UPD) {
        for (int i = 0; i < MW; ++i) sv = fmax(sv, dred[i]);
        shift = (sv == -INFINITY) ? 0.0 : sv;
    }
    // power-of-two scale: largest |value| in [2^13, 2^14)
    int ex = 0;
    frexpf(mx, &ex);
    const float scale = (mx > 0.0f) ? ldexpf(1.0f, 14 - ex) : 1.0f;
    const float unscale = (mx > 0.0f) ? ldexpf(1.0f, ex - 14) : 1.0f;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int q = threadIdx.x + NT * i;
        if (q < BOX) {
            const float u = v[i] * scale;
            const _Float16 h = (_Float16)u;
            const int row = q / S, x = q % S;
            bx[row][x >> 2][x & 3] = h;
            bx[row][x >> 2][4 + (x & 3)] = (_Float16)(u - (float)h);
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int node = lane & 15, slot = lane >> 4;
    double pmx = -INFINITY, dmx = 0.0;
    int bad = 0;
    float wc[NZ][WPOLY];
#pragma unroll
    for (int e = 0; e < NZ; ++e) {
        const int a = slot + 4 * e;
#pragma unroll
        for (int k = 0; k < WPOLY; ++k) wc[e][k] = (a < W) ? sa.wp[a * WPOLY + k] : 0.0f;
    }
    float(*ph)[W][16] = phi[wave];
    const int per = (mb.z + MW - 1) / MW;
    const int gb = mb.y + wave * per, ge = min(mb.y + mb.z, gb + per);
    int4 grn = make_int4(0, 1, 0, 0);
    float4 rn = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (gb < ge) {
        grn = mgroups[gb];
        rn = rec[grn.x + min(node, grn.y - 1)];
    }
    for (int g = gb; g < ge; ++g) {
        const int4 gr = grn;
        const float4 r = rn;
        if (g + 1 < ge) {
            grn = mgroups[g + 1];
            rn = rec[grn.x + min(node, grn.y - 1)];
        }
        const float fr[2] = {r.x, r.y};
#pragma unroll
        for (int dim = 0; dim < 2; ++dim) {
            const float u = 2.0f * fr[dim] - 1.0f;
#pragma unroll
            for (int e = 0; e < NZ; ++e) {
                const int a = slot + 4 * e;
                if (W % 4 == 0 || a < W) ph[dim][a][node] = wpoly_eval(wc[e], u);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int cur = gr.z;
        const int cx0 = cur % S, cy = cur / S;
        const int ox = __float_as_int(r.w) % S - cx0;  // the node's x cell inside the brick
        // operand B: px of node `node` at x = 4 slot .. + 3 as (hi, hi) and (lo, lo)
        f16x8 B1, B2;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int a = 4 * slot + e - ox;
            const float pv = (a >= 0 && a < W) ? ph[0][a < 0 ? 0 : (a >= W ? W - 1 : a)][node] : 0.0f;
            const _Float16 h = (_Float16)pv;
            const _Float16 l = (_Float16)(pv - (float)h);
            B1[e] = h;
            B1[4 + e] = h;
            B2[e] = l;
            B2[4 + e] = l;
        }
        // operand A: box row y = lane % 16 (rows at or beyond W read row W - 1; their py is zero)
        const int yr = node < W ? node : W - 1;
        const uint4 *arow = reinterpret_cast<const uint4 *>(&bx[cy + yr][(cx0 >> 2) + slot][0]);
        const f16x8 A = __builtin_bit_cast(f16x8, arow[0]);
        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
        acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(A, B1, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(A, B2, acc, 0, 0, 0);
        float part = 0.0f;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int y = 4 * slot + rr;
            const float pyv = (y < W) ? ph[1][y < W ? y : W - 1][node] : 0.0f;
            part = fmaf(pyv, acc[rr], part);
        }
        part += __shfl_xor(part, 16, 64);
        part += __shfl_xor(part, 32, 64);
        if (slot == 0 && node < gr.y) {
            const int k = gr.x + node;
            float t = part * unscale;
            if (!UPD) {
                out[k] = t;
            } else {
                if (!(t > 0.0f)) {
                    ++bad;
                    t = FLT_MIN;
                }
                const double f = -pu.kappa * (shift + pu.eps * sum_log(t));
                if (pu.delta_parts) dmx = fmax(dmx, fabs(f - pu.pot[k]));
                pu.pot[k] = f;
                pmx = fmax(pmx, f);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (UPD) {
        if (bad) atomicAdd(pu.nbad, bad);
        pmx = block_max_f64(pmx, dred);
        if (threadIdx.x == 0) pu.out_parts[blockIdx.x] = pmx;
        if (pu.delta_parts) {
            dmx = block_max_f64(dmx, dred);
            if (threadIdx.x == 0) pu.delta_parts[blockIdx.x] = dmx;
        }
    }
}

// ------------------------------------------------------------------ permutations
__global__ void k_gather_perm(const int *__restrict__ perm, int64_t n, const float *__restrict__ v,
                              float *__restrict__ vs) {
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k < n) vs[k] = v[perm[k]];
}
__global__ void k_scatter_perm(const int *__restrict__ perm, int64_t n,
                               const float *__restrict__ vs, float *__restrict__ v) {
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k < n) v[perm[k]] = vs[k];
}
__global__ void k_gather_perm64(const int *__restrict__ perm, int64_t n,
                                const double *__restrict__ v, double *__restrict__ vs) {
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k < n) vs[k] = v[perm[k]];
}
__global__ void k_scatter_perm64(const int *__restrict__ perm, int64_t n,
                                 const double *__restrict__ vs, double *__restrict__ v) {
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k < n) v[perm[k]] = vs[k];
}
__global__ void k_scatter_rows(const int *__restrict__ perm, int64_t n, int d,
                               const float *__restrict__ vs, float *__restrict__ v) {
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k < n)
        for (int c = 0; c < d; ++c) v[(int64_t)perm[k] * d + c] = vs[k * d + c];
}

// ------------------------------------------------------------------ near field
// For Laplace and energy kernels K_R differs from K inside the inner radius; the difference is
// summed directly over the source points of the neighbouring cells:
//   t_i += sum_{|x_i - y_j| < epsI P} (K(|x_i - y_j|) - q_I(|x_i - y_j| / P)) alpha_j
struct NearArgs {
    int kind, p, d;
    // Laplace: exp(-r / lambda) = exp2(r * lambda_inv) with lambda_inv = -log2(e) / lambda, and
    // K'(r) = lambda_lin K(r) with lambda_lin = -1 / lambda
    float lambda_inv, lambda_lin;
    float c2;           // IMQ: c^2
    float rinv, r2max;  // rinv = 1/(epsI P), r2max = (epsI P)^2
    float ci[16];   // inner polynomial in s = (r / (epsI P))^2, zero-padded
    float dci[16];  // its derivative in s: dci[k] = 2 (k + 1) ci[k + 1]
    float h_inv;
    float lo[3];
    int dims[3];
};

__global__ void k_nf_keys(const float *__restrict__ xs, int64_t n, NearArgs na,
                          int *__restrict__ key, int *__restrict__ hist) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int kk = 0;
    for (int c = na.d - 1; c >= 0; --c) {
        int v = (int)floorf((xs[i * na.d + c] - na.lo[c]) * na.h_inv);
        v = max(0, min(na.dims[c] - 1, v));
        kk = kk * na.dims[c] + v;
    }
    key[i] = kk;
    atomicAdd(&hist[kk], 1);
}

// rank (nullable): each point's position inside its cell (deterministic mode); else the cell's
// atomic cursor.
__global__ void k_nf_scatter(const float *__restrict__ xs, int64_t n, int d,
                             const int *__restrict__ key, const int *__restrict__ start,
                             int *__restrict__ cursor, const int *__restrict__ rank,
                             int *__restrict__ order, float *__restrict__ cxs) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int pos = start[key[i]] + (rank ? rank[i] : atomicAdd(&cursor[key[i]], 1));
    order[pos] = (int)i;
    for (int c = 0; c < d; ++c) cxs[(int64_t)pos * d + c] = xs[i * d + c];
}

// Target blocks: runs of at most 64 consecutive targets (cell order) inside one row of cells,
// {first target, end, first cell x | last cell x << 16, row}.
__global__ void k_nf_row_counts(const int *__restrict__ cell_start, int nrows, int dims0,
                                int *__restrict__ cnt) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r <= nrows) cnt[r] = (r < nrows) ? cell_start[(r + 1) * dims0] - cell_start[r * dims0] : 0;
}

__global__ void k_nf_fill_blocks(const int *__restrict__ cell_start, int nrows, int dims0,
                                 const int *__restrict__ row_blk, int4 *__restrict__ blocks) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    const int base = r * dims0, end = cell_start[base + dims0];
    int o = row_blk[2 * r], cx = 0;
    for (int t0 = cell_start[base]; t0 < end; t0 += 64, ++o) {
        const int t1 = min(t0 + 64, end);
        while (cell_start[base + cx + 1] <= t0) ++cx;
        int cx1 = cx;
        while (cell_start[base + cx1 + 1] < t1) ++cx1;
        blocks[o] = make_int4(t0, t1, cx | (cx1 << 16), r);
    }
}

// Sources in cell order as (x, y, z, weight) records for the current weights; four zero records
// follow the last one so that the kernel may read whole groups of four.
__global__ void k_nf_pack(const float *__restrict__ xs, const int *__restrict__ order,
                          const float *__restrict__ w, int64_t m, int d, float4 *__restrict__ rec) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k < m) {
        float c[3] = {0.0f, 0.0f, 0.0f};
        for (int i = 0; i < d; ++i) c[i] = xs[k * d + i];
        rec[k] = make_float4(c[0], c[1], c[2], w[order[k]]);
    } else if (k < m + 4) {
        rec[k] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
}

struct Rec4 {
    float4 r[4];
};

// One wave per target block (and source split): each lane holds one target; the sources of the stencil rows around
// the block (cell side h >= radius / R, rows and cells whose distance to the block's cells is at
// least the radius are skipped) are read as wave-uniform records, so they arrive through scalar
// loads and feed every lane without LDS traffic.  NP = number of inner polynomial coefficients
// (zero-padded), KIND = Laplace, energy or IMQ.
template <int D, int KIND, int NP, bool GRAD>
__global__ void __launch_bounds__(64) k_nearfield(const int4 *__restrict__ blocks,
                                                   const float *__restrict__ t_xs,
                                                   const int *__restrict__ t_order,
                                                   const int *__restrict__ s_start,
                                                   const float4 *__restrict__ src,
                                                   NearArgs na, int R, float rr,
                                                   float *__restrict__ out,
                                                   float *__restrict__ gout) {
    const int4 bk = blocks[blockIdx.x];
    const int t = bk.x + (int)threadIdx.x;
    const bool active = t < bk.y;
    float xi[3] = {0.0f, 0.0f, 0.0f};
    if (active)
        for (int c = 0; c < D; ++c) xi[c] = t_xs[(int64_t)t * D + c];
    const int cxl = bk.z & 0xffff, cxh = bk.z >> 16;
    const int cy = (D >= 2) ? bk.w % na.dims[1] : 0;
    const int cz = (D == 3) ? bk.w / na.dims[1] : 0;
    const int Ry = (D >= 2) ? R : 0, Rz = (D == 3) ? R : 0;
    const float rinv2 = na.rinv * na.rinv;
    float acc = 0.0f, g[3] = {0.0f, 0.0f, 0.0f};
    for (int dz = -Rz; dz <= Rz; ++dz) {
        const int z = cz + dz;
        if (z < 0 || z >= na.dims[2]) continue;
        const int ez = max(abs(dz) - 1, 0);
        for (int dy = -Ry; dy <= Ry; ++dy) {
            const int y = cy + dy;
            if (y < 0 || y >= na.dims[1]) continue;
            const int ey = max(abs(dy) - 1, 0);
            const float M = rr - (float)(ey * ey + ez * ez);
            if (M <= 0.0f) continue;
            const int A = min(R, 1 + (int)sqrtf(M));
            const int row = (z * na.dims[1] + y) * na.dims[0];
            const int s0 = s_start[row + max(cxl - A, 0)];
            const int s1 = s_start[row + min(cxh + A, na.dims[0] - 1) + 1];
            // groups of four records (one 64-byte scalar load); the next group is requested
            // as soon as the current one has arrived.  With a source split (gridDim.y > 1) this
            // wave takes every gridDim.y-th group.
            const int k0 = s0 + 4 * (int)blockIdx.y, kstep = 4 * (int)gridDim.y;
            Rec4 cur = *reinterpret_cast<const Rec4 *>(src + min(k0, s1));
            for (int k = k0; k < s1; k += kstep) {
                __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): cur has arrived
                const Rec4 nxt = *reinterpret_cast<const Rec4 *>(src + min(k + kstep, s1));
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const float4 sv = cur.r[u];
                    const float wj = (k + u < s1) ? sv.w : 0.0f;
                    float dv[3];
                    dv[0] = xi[0] - sv.x;
                    dv[1] = xi[1] - sv.y;
                    dv[2] = xi[2] - sv.z;
                    float r2 = dv[0] * dv[0];
                    if (D >= 2) r2 = fmaf(dv[1], dv[1], r2);
                    if (D == 3) r2 = fmaf(dv[2], dv[2], r2);
                    if (r2 < na.r2max) {
                        const float s = r2 * rinv2;
                        float q = na.ci[NP - 1];
#pragma unroll
                        for (int kk = NP - 2; kk >= 0; --kk) q = fmaf(q, s, na.ci[kk]);
                        if (!GRAD) {
                            float kv;
                            if (KIND == FS_IMQ) {
                                kv = __builtin_amdgcn_rsqf(r2 + na.c2);
                            } else {
                                const float r = __builtin_amdgcn_sqrtf(r2);
                                kv = (KIND == FS_LAPLACE) ? __builtin_amdgcn_exp2f(r * na.lambda_inv)
                                                          : -r;
                            }
                            acc = fmaf(kv - q, wj, acc);
                        } else {
                            const float r2c = fmaxf(r2, 1e-30f);
                            const float ri = __builtin_amdgcn_rsqf(r2c);
                            const float r = r2c * ri;
                            float dq = na.dci[NP - 2];
#pragma unroll
                            for (int kk = NP - 3; kk >= 0; --kk) dq = fmaf(dq, s, na.dci[kk]);
                            float kv, dkr;  // K(r) and K'(r) / r
                            if (KIND == FS_LAPLACE) {
                                kv = __builtin_amdgcn_exp2f(r * na.lambda_inv);
                                dkr = na.lambda_lin * kv * ri;
                            } else if (KIND == FS_IMQ) {
                                kv = __builtin_amdgcn_rsqf(r2 + na.c2);
                                dkr = -kv * kv * kv;
                            } else {
                                kv = -r;
                                dkr = -ri;
                            }
                            acc = fmaf(kv - q, wj, acc);
                            // d/dr (K - q) / r = K'(r)/r - rinv2 * sum_k 2k c_k s^(k-1)
                            const float coef = (dkr - rinv2 * dq) * wj;
                            for (int c = 0; c < D; ++c) g[c] = fmaf(coef, dv[c], g[c]);
                        }
                    }
                }
                cur = nxt;
            }
        }
    }
    if (active) {
        const int o = t_order[t];
        if (gridDim.y == 1) {
            out[o] += acc;
            if (GRAD)
                for (int c = 0; c < D; ++c) gout[(int64_t)o * D + c] += g[c];
        } else {
            atomicAdd(&out[o], acc);
            if (GRAD)
                for (int c = 0; c < D; ++c) atomicAdd(&gout[(int64_t)o * D + c], g[c]);
        }
    }
}

}  // namespace

// =====================================================================================
//                                        host side
// =====================================================================================

void gather_to_sorted(const Nodes &nd, const float *v, float *vs, hipStream_t s) {
    if (nd.n == 0) return;
    hipLaunchKernelGGL(k_gather_perm, dim3(blocks_for(nd.n, 256, int64_t(1) << 30)), dim3(256),
                       0, s, nd.perm.p, nd.n, v, vs);
    FS_LAUNCHED();
}
void scatter_from_sorted(const Nodes &nd, const float *vs, float *v, hipStream_t s) {
    if (nd.n == 0) return;
    hipLaunchKernelGGL(k_scatter_perm, dim3(blocks_for(nd.n, 256, int64_t(1) << 30)), dim3(256),
                       0, s, nd.perm.p, nd.n, vs, v);
    FS_LAUNCHED();
}
void gather_to_sorted64(const Nodes &nd, const double *v, double *vs, hipStream_t s) {
    if (nd.n == 0) return;
    hipLaunchKernelGGL(k_gather_perm64, dim3(blocks_for(nd.n, 256, int64_t(1) << 30)), dim3(256),
                       0, s, nd.perm.p, nd.n, v, vs);
    FS_LAUNCHED();
}
void scatter_from_sorted64(const Nodes &nd, const double *vs, double *v, hipStream_t s) {
    if (nd.n == 0) return;
    hipLaunchKernelGGL(k_scatter_perm64, dim3(blocks_for(nd.n, 256, int64_t(1) << 30)),
                       dim3(256), 0, s, nd.perm.p, nd.n, vs, v);
    FS_LAUNCHED();
}
void scatter_rows_from_sorted(const Nodes &nd, const float *vs, int d, float *v, hipStream_t s) {
    if (nd.n == 0) return;
    hipLaunchKernelGGL(k_scatter_rows, dim3(blocks_for(nd.n, 256, int64_t(1) << 30)), dim3(256),
                       0, s, nd.perm.p, nd.n, d, vs, v);
    FS_LAUNCHED();
}

namespace {

// Exclusive scan of n ints (device), result in out (stream-ordered).  The temporaries are moved
// into `keep` when given (the caller releases them after its own synchronisation), else the
// stream is synchronised before they are released.
void exclusive_scan(const int *in, int64_t n, int *out, hipStream_t s,
                    std::vector<DevBuf<int>> *keep = nullptr) {
    const int64_t nb = (n + SCAN_PER_BLOCK - 1) / SCAN_PER_BLOCK;
    FS_REQUIRE(nb <= 1024 * 1024, FS_EINVAL, "scan too large");
    DevBuf<int> bsum(nb + 1), boff(nb + 1), tmp1(2 * (nb + 1)), tot(2);
    hipLaunchKernelGGL(k_block_sums, dim3((unsigned)nb), dim3(256), 0, s, in, n, bsum.p);
    FS_LAUNCHED();
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, s, bsum.p, (int)nb, 1 << 30, boff.p,
                       tmp1.p, tot.p);
    FS_LAUNCHED();
    hipLaunchKernelGGL(k_block_scan, dim3((unsigned)nb), dim3(256), 0, s, in, n, boff.p, out);
    FS_LAUNCHED();
    if (keep) {
        keep->push_back(std::move(bsum));
        keep->push_back(std::move(boff));
        keep->push_back(std::move(tmp1));
        keep->push_back(std::move(tot));
    } else {
        FS_HIP(hipStreamSynchronize(s));  // temporaries are released after this
    }
}

// Workgroups of the matrix-core spread and gather that the current device holds at once (compute
// units x resident workgroups per unit, the smaller of the two kernels), cached per device and
// window.
template <int W>
int mfma_blocks_per_cu() {
    int a = 0, b = 0;
    FS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_gather_mfma16<W, true>, 64 * MW, 0));
    FS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_spread_mom16<W, true>, 64 * MW, 0));
    return std::max(1, std::min(a, b));
}
template <int W, int T>
int mfma_blocks_per_cu_2d() {
    int a = 0, b = 0;
    FS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_gather_mfma2d<W, T, true>, 64 * MW,
                                                        0));
    FS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_spread_mfma2d<W, T, true>, 64 * MW,
                                                        0));
    return std::max(1, std::min(a, b));
}

// Resident matrix-core workgroups on the chip for window width W (d = 3, or d = 2 with tile T).
int mfma_slots(int W, int d, int T) {
    // per device, kind and width (plans may be built from several host threads at once)
    static std::atomic<int> cache[16][2][17];
    int dev = 0;
    FS_HIP(hipGetDevice(&dev));
    const int v = (d == 3) ? 0 : 1;
    if (dev < 16 && W <= 16 && (d == 3 || T == 32)) {
        const int c = cache[dev][v][W].load(std::memory_order_relaxed);
        if (c > 0) return c;
    }
    int cus = 0, per = 1;
    FS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    if (d == 3) {
        switch (W) {
            case 4: per = mfma_blocks_per_cu<4>(); break;
            case 6: per = mfma_blocks_per_cu<6>(); break;
            case 8: per = mfma_blocks_per_cu<8>(); break;
            case 10: per = mfma_blocks_per_cu<10>(); break;
            case 12: per = mfma_blocks_per_cu<12>(); break;
            default: per = 1;
        }
    } else if (T == 32) {
        switch (W) {
            case 4: per = mfma_blocks_per_cu_2d<4, 32>(); break;
            case 6: per = mfma_blocks_per_cu_2d<6, 32>(); break;
            case 8: per = mfma_blocks_per_cu_2d<8, 32>(); break;
            case 10: per = mfma_blocks_per_cu_2d<10, 32>(); break;
            case 12: per = mfma_blocks_per_cu_2d<12, 32>(); break;
            default: per = 1;
        }
    } else {
        switch (W) {
            case 4: per = mfma_blocks_per_cu_2d<4, 16>(); break;
            case 6: per = mfma_blocks_per_cu_2d<6, 16>(); break;
            case 8: per = mfma_blocks_per_cu_2d<8, 16>(); break;
            case 10: per = mfma_blocks_per_cu_2d<10, 16>(); break;
            case 12: per = mfma_blocks_per_cu_2d<12, 16>(); break;
            default: per = 1;
        }
    }
    const int slots = std::max(1, cus * per);
    if (dev < 16 && W <= 16 && (d == 3 || T == 32))
        cache[dev][v][W].store(slots, std::memory_order_relaxed);
    return slots;
}

// Matrix-core groups and their blocks from the cell offsets of cell-sorted nodes (d = 3), in two
// stages around the binning's host synchronisation.  The groups of a tile are cut into blocks of
// equal size, the smallest size for which all blocks fit on the chip at once (`slots` resident
// workgroups): a second, partly filled round of workgroups would nearly double the pass.
struct MGroupBuild {
    int64_t nbricks = 0;
    DevBuf<int> gcount;
    int *tgroups = nullptr;   // groups per tile (device, in the binning's count table)
    const int *tg = nullptr;  // pinned host copy of tgroups, valid after the synchronisation
};

// Stage 1 (before the synchronisation): groups per brick and per tile (into tgroups).
void mgroups_count(MGroupBuild &mg, const int *kstart, int64_t n, int64_t ntiles,
                   int64_t cells_per_tile, int *tgroups, hipStream_t s) {
    mg.nbricks = ntiles * cells_per_tile / BRICK_X;
    mg.gcount.alloc(mg.nbricks + 1);
    mg.tgroups = tgroups;
    hipLaunchKernelGGL(k_brick_groups, dim3(blocks_for(mg.nbricks, 256)), dim3(256), 0, s, kstart,
                       mg.nbricks, (int)n, mg.gcount.p);
    FS_LAUNCHED();
    hipLaunchKernelGGL(k_tile_sum, dim3((unsigned)ntiles), dim3(256), 0, s, mg.gcount.p,
                       (int)ntiles, (int)(cells_per_tile / BRICK_X), mg.tgroups);
    FS_LAUNCHED();
}

// Stage 2 (after it), host part: block size from the per-tile counts, and per tile the first
// group, then [first block, block count], then the tiles with several blocks, appended to `tab`
// (at offset `off`, returned).  Returns the groups per block.
int mgroups_plan(Nodes &nd, const MGroupBuild &mg, int64_t n, int64_t ntiles,
                 const PlanParams &pp, int slots, std::vector<int> &tab, size_t &off) {
    const int *tg = mg.tg;
    int64_t total = 0;
    int tmax = 0;
    for (int64_t t = 0; t < ntiles; ++t) {
        total += tg[t];
        tmax = std::max(tmax, tg[t]);
    }
    auto blocks_at = [&](int g) {
        int64_t b = 0;
        for (int64_t t = 0; t < ntiles; ++t) b += (tg[t] + g - 1) / g;
        return b;
    };
    // 2-D groups are cheap (two matrix instructions each): blocks of at least four groups per wave
    // keep the per-block fixed work and the number of boxes to reduce down
    const int min_gpb = (pp.d == 2) ? 4 * MIN_GROUPS_PER_BLOCK : MIN_GROUPS_PER_BLOCK;
    int lo = (int)std::max<int64_t>(min_gpb, (total + slots - 1) / std::max(slots, 1));
    int hi = std::max(lo, tmax);
    while (lo < hi) {
        const int mid = lo + (hi - lo) / 2;
        if (blocks_at(mid) <= slots) hi = mid;
        else lo = mid + 1;
    }
    const int gpb = lo;
    // at most n / 16 full groups plus one partial group per non-empty brick
    const int64_t cap = n / 16 + std::min<int64_t>(n, mg.nbricks) + 1;
    FS_REQUIRE(total <= cap, FS_EINVAL, "group count %lld above its bound", (long long)total);
    off = tab.size();
    tab.resize(off + 3 * ntiles);
    int *tgstart = tab.data() + off, *tblock = tgstart + ntiles;
    int64_t g0 = 0, b0 = 0;
    int nmulti = 0;
    for (int64_t t = 0; t < ntiles; ++t) {
        const int nb = (tg[t] + gpb - 1) / gpb;
        tgstart[t] = (int)g0;
        tblock[2 * t] = (int)b0;
        tblock[2 * t + 1] = nb;
        nmulti += nb > 1;
        g0 += tg[t];
        b0 += nb;
    }
    for (int64_t t = 0; t < ntiles; ++t)
        if (tab[off + ntiles + 2 * t + 1] > 1) tab.push_back((int)t);
    nd.n_mgroups = (int)total;
    nd.n_mblocks = (int)b0;
    nd.n_mmulti = nmulti;
    return gpb;
}

// Stage 2, device part: the group and block tables, given the uploaded per-tile tables `dtab`
// (laid out as mgroups_plan writes them).  Temporaries go to `keep`.
void mgroups_fill(Nodes &nd, MGroupBuild &mg, const int *kstart, int64_t n, int64_t ntiles,
                  const PlanParams &pp, int gpb, const int *dtab, hipStream_t s,
                  std::vector<DevBuf<int>> &keep) {
    nd.mtile_block = dtab + ntiles;
    nd.mmulti_tiles = dtab + 3 * ntiles;
    DevBuf<int> gstart(mg.nbricks + 1);
    nd.mgroups.alloc(std::max<int64_t>(nd.n_mgroups, 1));
    nd.mblocks.alloc(nd.n_mblocks + 1);
    exclusive_scan(mg.gcount.p, mg.nbricks, gstart.p, s, &keep);
    hipLaunchKernelGGL(k_fill_groups, dim3(blocks_for(mg.nbricks, 256)), dim3(256), 0, s, kstart,
                       gstart.p, mg.nbricks, (int)n, pp.d, pp.T, pp.T + pp.W - 1, nd.mgroups.p);
    FS_LAUNCHED();
    if (nd.n_mblocks > 0) {
        hipLaunchKernelGGL(k_fill_chunks, dim3(blocks_for(ntiles, 256)), dim3(256), 0, s,
                           (int)ntiles, dtab, mg.tgroups, nd.mtile_block, gpb, nd.mblocks.p);
        FS_LAUNCHED();
        nd.mbnodes.alloc(nd.n_mblocks);
        hipLaunchKernelGGL(k_block_nodes, dim3(blocks_for(nd.n_mblocks, 256)), dim3(256), 0, s,
                           nd.mblocks.p, nd.mgroups.p, nd.n_mblocks, nd.mbnodes.p);
        FS_LAUNCHED();
    }
    keep.push_back(std::move(gstart));
    keep.push_back(std::move(mg.gcount));
}

// Tile/cell binning of one point set, in two stages around a host synchronisation that the
// caller makes (one for both point sets of a plan).  Temporaries go to the build's stage `hs`
// (freed after its final synchronisation).
struct BinBuild {
    int64_t n = 0, ntiles = 1, cells_per_tile = 1, nkeys = 0;
    bool cell_keys = false, mgroups = false;
    DevBuf<int> key, rank, hist, kstart, tcount, tstart;
    DevBuf<float4> tmp;
    const int *tile_hist = nullptr;
    const int *hcounts = nullptr;  // pinned copy of the plan's tile_chunk table (with the totals
                                   // and groups per tile), valid after the synchronisation
    MGroupBuild mg;
    std::vector<DevBuf<int>> keep;
};

void bin_nodes_count(Nodes &nd, BinBuild &bb, const float *pts, int64_t n, const PlanParams &pp,
                     hipStream_t s, HostStage &hs) {
    nd.n = n;
    bb.n = n;
    const int d = pp.d, G = pp.G, T = pp.T, ntd = G / T;
    int64_t ntiles = 1, cells_per_tile = 1;
    for (int k = 0; k < d; ++k) {
        ntiles *= ntd;
        cells_per_tile *= T;
    }
    bb.ntiles = ntiles;
    bb.cells_per_tile = cells_per_tile;
    // order nodes by (tile, cell) when the cell key space is at most 2^24 (64 MB of counters)
    const int64_t ncellkeys = ntiles * cells_per_tile;
    bb.cell_keys = ncellkeys <= (int64_t(1) << 24);
    bb.nkeys = bb.cell_keys ? ncellkeys : ntiles;
    nd.rec.alloc(n + 1);
    nd.perm.alloc(n + 1);
    nd.xs.alloc(n * d + 1);
    // [first chunk, chunk count] per tile, then the totals (2), then the groups per tile: one
    // download after the kernels
    nd.tile_chunk.alloc(3 * ntiles + 2);
    bb.key.alloc(n + 1);
    bb.rank.alloc(n + 1);
    bb.hist.alloc(bb.nkeys);
    bb.kstart.alloc(bb.nkeys);
    bb.tcount.alloc(ntiles);
    bb.tstart.alloc(ntiles);
    bb.tmp.alloc(n + 1);
    int *totals = nd.tile_chunk.p + 2 * ntiles, *tgroups = totals + 2;
    fill_i32(bb.hist.p, bb.nkeys, 0, s);
    ScaleArgs sa{};
    for (int k = 0; k < 3; ++k) sa.c[k] = pp.center[k];
    sa.inv_P = 1.0 / pp.P;
    sa.G = G;
    sa.T = T;
    sa.ntd = ntd;
    sa.d = d;
    sa.S = T + pp.W - 1;
    if (n > 0) {
        hipLaunchKernelGGL(k_keys, dim3(blocks_for(n, 256, int64_t(1) << 30)), dim3(256), 0, s,
                           pts, n, sa, (int)bb.cell_keys, bb.key.p, bb.rank.p, bb.tmp.p, bb.hist.p);
        FS_LAUNCHED();
    }
    exclusive_scan(bb.hist.p, bb.nkeys, bb.kstart.p, s, &bb.keep);
    // deterministic mode: ranks inside a key in input order instead of the atomic counter's
    if (pp.stable) stable_ranks(bb.key.p, n, bb.nkeys, bb.kstart.p, bb.rank.p, s);
    bb.tile_hist = bb.hist.p;
    if (bb.cell_keys) {
        hipLaunchKernelGGL(k_tile_counts, dim3(blocks_for(ntiles, 256)), dim3(256), 0, s,
                           bb.kstart.p, (int)ntiles, (int)cells_per_tile, (int)n, bb.tcount.p);
        FS_LAUNCHED();
        bb.tile_hist = bb.tcount.p;
    }
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, s, bb.tile_hist, (int)ntiles,
                       pp.chunk, bb.tstart.p, nd.tile_chunk.p, totals);
    FS_LAUNCHED();
    if (n > 0) {
        hipLaunchKernelGGL(k_scatter_nodes, dim3(blocks_for(n, 256, int64_t(1) << 30)), dim3(256),
                           0, s, pts, n, d, bb.key.p, bb.rank.p, bb.tmp.p, bb.kstart.p, nd.rec.p,
                           nd.perm.p, nd.xs.p);
        FS_LAUNCHED();
    }
    // matrix-core groups (d = 2, 3): per-brick and per-tile counts, read back with the chunk table
    bb.mgroups = (d == 3 || (d == 2 && (T == 32 || T == 16))) && bb.cell_keys &&
                 T % BRICK_X == 0 && pp.W + BRICK_X - 1 <= 16 && n > 0;
    if (bb.mgroups) mgroups_count(bb.mg, bb.kstart.p, n, ntiles, cells_per_tile, tgroups, s);
    bb.hcounts = hs.download(nd.tile_chunk.p, (size_t)(bb.mgroups ? 3 * ntiles + 2 : 2 * ntiles + 2));
}

void bin_nodes_finish(Nodes &nd, BinBuild &bb, const PlanParams &pp, hipStream_t s,
                      HostStage &hs) {
    const int d = pp.d, ntd = pp.G / pp.T;
    const int64_t ntiles = bb.ntiles, n = bb.n;
    const int *tch = bb.hcounts, *tot = bb.hcounts + 2 * ntiles;
    bb.mg.tg = tot + 2;
    nd.nchunks = tot[1];
    // host tile lists, one upload: tiles with several chunks, touched tiles, then the
    // matrix-core per-tile tables
    std::vector<int> tab;
    for (int64_t t = 0; t < ntiles; ++t)
        if (tch[2 * t + 1] > 1) tab.push_back((int)t);
    nd.n_multi = (int)tab.size();
    // tiles whose 3^d neighbourhood (periodic) holds a chunk: the only ones the fold must sum
    // (occupied tiles dilated by one tile along each axis in turn)
    std::vector<char> occ(ntiles), tmpo(ntiles);
    for (int64_t t = 0; t < ntiles; ++t) occ[t] = tch[2 * t + 1] > 0;
    int64_t stride = 1;
    for (int k = 0; k < d; ++k, stride *= ntd) {
        for (int64_t t = 0; t < ntiles; ++t) {
            const int c = (int)((t / stride) % ntd);
            const int64_t base = t - (int64_t)c * stride;
            tmpo[t] = occ[t] || occ[base + (int64_t)((c + 1) % ntd) * stride] ||
                      occ[base + (int64_t)((c + ntd - 1) % ntd) * stride];
        }
        occ.swap(tmpo);
    }
    const size_t touched_off = tab.size();
    for (int64_t t = 0; t < ntiles; ++t)
        if (occ[t]) tab.push_back((int)t);
    nd.n_touched = (int)(tab.size() - touched_off);
    nd.n_mgroups = nd.n_mblocks = nd.n_mmulti = 0;
    int gpb = 0;
    size_t mg_off = 0;
    if (bb.mgroups)
        gpb = mgroups_plan(nd, bb.mg, n, ntiles, pp, mfma_slots(pp.W, d, pp.T), tab, mg_off);
    nd.tile_lists.alloc(std::max<size_t>(tab.size(), 1));
    hs.upload(nd.tile_lists.p, tab.data(), tab.size() * sizeof(int));
    nd.multi_tiles = nd.tile_lists.p;
    nd.touched_tiles = nd.tile_lists.p + touched_off;
    nd.chunks.alloc(nd.nchunks + 1);
    if (nd.nchunks > 0) {
        hipLaunchKernelGGL(k_fill_chunks, dim3(blocks_for(ntiles, 256)), dim3(256), 0, s,
                           (int)ntiles, bb.tstart.p, bb.tile_hist, nd.tile_chunk.p, pp.chunk,
                           nd.chunks.p);
        FS_LAUNCHED();
    }
    if (bb.mgroups)
        mgroups_fill(nd, bb.mg, bb.kstart.p, n, ntiles, pp, gpb, nd.tile_lists.p + mg_off, s,
                     bb.keep);
    for (auto &b : bb.keep) hs.hold(b);
    hs.hold(bb.key);
    hs.hold(bb.rank);
    hs.hold(bb.hist);
    hs.hold(bb.kstart);
    hs.hold(bb.tcount);
    hs.hold(bb.tstart);
    hs.hold(bb.tmp);
}

void build_nearfield_cells(Nodes &nd, const PlanParams &pp, hipStream_t s) {
    const int d = pp.d;
    int64_t ncells = 1;
    for (int k = 0; k < d; ++k) ncells *= pp.nf_dims[k];
    nd.nf_cell_start.alloc(ncells + 1);
    nd.nf_order.alloc(nd.n + 1);
    nd.nf_xs.alloc(nd.n * d + 1);
    DevBuf<int> key(nd.n + 1), hist(ncells + 1), cursor(ncells + 1), chunkdummy(2 * (ncells + 1)),
        totals(2);
    fill_i32(hist.p, ncells + 1, 0, s);
    fill_i32(cursor.p, ncells + 1, 0, s);
    NearArgs na{};
    na.d = d;
    na.h_inv = (float)(1.0 / pp.nf_h);
    for (int k = 0; k < 3; ++k) {
        na.lo[k] = (float)pp.nf_lo[k];
        na.dims[k] = pp.nf_dims[k];
    }
    if (nd.n > 0) {
        hipLaunchKernelGGL(k_nf_keys, dim3(blocks_for(nd.n, 256, int64_t(1) << 30)), dim3(256), 0,
                           s, nd.xs.p, nd.n, na, key.p, hist.p);
        FS_LAUNCHED();
    }
    // exclusive scan over ncells + 1 entries (last entry 0) gives start offsets and the total
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, s, hist.p, (int)(ncells + 1), 1 << 30,
                       nd.nf_cell_start.p, chunkdummy.p, totals.p);
    FS_LAUNCHED();
    DevBuf<int> nrank(pp.stable ? nd.n + 1 : 0);
    if (pp.stable) stable_ranks(key.p, nd.n, ncells + 1, nd.nf_cell_start.p, nrank.p, s);
    if (nd.n > 0) {
        hipLaunchKernelGGL(k_nf_scatter, dim3(blocks_for(nd.n, 256, int64_t(1) << 30)), dim3(256),
                           0, s, nd.xs.p, nd.n, d, key.p, nd.nf_cell_start.p, cursor.p, nrank.p,
                           nd.nf_order.p, nd.nf_xs.p);
        FS_LAUNCHED();
    }
    // target blocks per row of cells
    const int dims0 = pp.nf_dims[0];
    const int nrows = (int)(ncells / dims0);
    DevBuf<int> rcnt(nrows + 1), rstart(nrows + 1), rblk(2 * (nrows + 1));
    hipLaunchKernelGGL(k_nf_row_counts, dim3(blocks_for(nrows + 1, 256)), dim3(256), 0, s,
                       nd.nf_cell_start.p, nrows, dims0, rcnt.p);
    FS_LAUNCHED();
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, s, rcnt.p, nrows, 64, rstart.p,
                       rblk.p, totals.p);
    FS_LAUNCHED();
    int tot[2] = {0, 0};
    FS_HIP(hipMemcpyAsync(tot, totals.p, sizeof(tot), hipMemcpyDeviceToHost, s));
    FS_HIP(hipStreamSynchronize(s));
    nd.nf_nblocks = tot[1];
    nd.nf_blocks.alloc(std::max(tot[1], 1));
    if (tot[1] > 0) {
        hipLaunchKernelGGL(k_nf_fill_blocks, dim3(blocks_for(nrows, 64)), dim3(64), 0, s,
                           nd.nf_cell_start.p, nrows, dims0, rblk.p, nd.nf_blocks.p);
        FS_LAUNCHED();
    }
    FS_HIP(hipStreamSynchronize(s));
}

}  // namespace

namespace {
// Multipliers M_k of recent plans, keyed by everything they depend on, so that a plan of the same
// kernel, grid and scaling (a repeated solve on the same clouds) copies them instead of sampling
// K_R and transforming it again.  At most MULT_CACHE entries, least recently used first; `ready`
// is recorded after an entry's last write, and readers wait for it on their own stream.  An
// entry is freed only after a device synchronisation, since copies from it may still be queued
// on other streams.
struct MultKey {
    int dev, d, N, G, m, kind, regime, p;
    double b, lambda, P, epsI, epsB, ci[16], cb[32];
};
struct MultEntry {
    MultKey key;
    DevBuf<float> mk;
    hipEvent_t ready = nullptr;
};
constexpr size_t MULT_CACHE = 4;
std::mutex g_mult_mu;
std::vector<std::unique_ptr<MultEntry>> g_mult;

}  // namespace

void plan_multiplier(const Plan &pl, float *mult_host, double *phihat_host, int64_t count,
                     double *period, int *bandwidth, hipStream_t s) {
    const PlanParams &pp = pl.pp;
    const int H = pp.N / 2 + 1;
    int64_t nh = 1;
    for (int k = 0; k < pp.d; ++k) nh *= H;
    FS_REQUIRE(count >= nh, FS_EINVAL, "the multiplier has %lld values (count %lld)",
               (long long)nh, (long long)count);
    if (mult_host) {
        FS_HIP(hipMemcpyAsync(mult_host, pl.Mk.p, nh * sizeof(float), hipMemcpyDeviceToHost, s));
        FS_HIP(hipStreamSynchronize(s));
    }
    const double b = M_PI * (2.0 - (double)pp.N / pp.G);
    if (phihat_host)
        for (int k = 0; k < H; ++k) phihat_host[k] = kb_hat(pp.m, b, pp.G, k);
    if (period) *period = pp.P;
    if (bandwidth) *bandwidth = pp.N;
}

void plan_release_mult_cache() {
    std::lock_guard<std::mutex> lk(g_mult_mu);
    if (g_mult.empty()) return;
    (void)hipDeviceSynchronize();  // no queued copy still reads an entry
    for (auto &e : g_mult) (void)hipEventDestroy(e->ready);
    g_mult.clear();
}

namespace {
MultKey mult_key(const PlanParams &pp, double b) {
    MultKey k;
    std::memset(&k, 0, sizeof(k));  // padding included: keys are compared bytewise
    FS_HIP(hipGetDevice(&k.dev));
    k.d = pp.d;
    k.N = pp.N;
    k.G = pp.G;
    k.m = pp.m;
    k.kind = pp.kind;
    k.regime = pp.regime;
    k.p = pp.p;
    k.b = b;
    k.lambda = pp.lambda;
    k.P = pp.P;
    k.epsI = pp.epsI;
    k.epsB = pp.epsB;
    std::memcpy(k.ci, pp.ci, sizeof(k.ci));
    std::memcpy(k.cb, pp.cb, sizeof(k.cb));
    return k;
}
}  // namespace

namespace {
// Host tables of the window (they depend on m, N and G only): the segment polynomials of value
// and derivative, and for d = 3 the moment-form spread's transform operands.  Kept for the
// process, so that repeated plans of one grid skip the fits and the FP16 split.
struct WindowTables {
    std::vector<float> hp;      // value (W x WPOLY) then derivative
    std::vector<uint16_t> cc;   // empty unless requested
};
std::mutex g_win_mu;
std::map<std::array<int, 4>, std::shared_ptr<const WindowTables>> g_win;
constexpr size_t WIN_CACHE = 16;

std::shared_ptr<const WindowTables> window_tables(int m, int N, int G, bool mom) {
    const std::array<int, 4> key{m, N, G, (int)mom};
    {
        std::lock_guard<std::mutex> lk(g_win_mu);
        auto it = g_win.find(key);
        if (it != g_win.end()) return it->second;
    }
    auto wt = std::make_shared<WindowTables>();
    const int W = 2 * m;
    const double b = M_PI * (2.0 - (double)N / G);
    // window value phi(t + m - 1 - a) and derivative d phi/ds on t in [0, 1), u = 2t - 1
    wt->hp.assign(2 * W * WPOLY, 0.0f);
    std::vector<double> cheb(W * WPOLY);
    double c[WPOLY];
    for (int a = 0; a < W; ++a) {
        const double off = m - 1 - a;
        fit_poly([&](double u) { return kb_value(m, b, 0.5 * (u + 1.0) + off); }, WPOLY, c);
        for (int k = 0; k < WPOLY; ++k) wt->hp[a * WPOLY + k] = (float)c[k];
        // the same polynomial in the Chebyshev basis (exact: interpolation at WPOLY nodes)
        for (int k = 0; k < WPOLY; ++k) {
            double acc = 0.0;
            for (int j = 0; j < WPOLY; ++j) {
                const double th = M_PI * (j + 0.5) / WPOLY, u = std::cos(th);
                double v = c[WPOLY - 1];
                for (int q = WPOLY - 2; q >= 0; --q) v = v * u + c[q];
                acc += v * std::cos(k * th);
            }
            cheb[a * WPOLY + k] = acc * (k == 0 ? 1.0 : 2.0) / WPOLY;
        }
        fit_poly([&](double u) { return kb_deriv(m, b, 0.5 * (u + 1.0) + off); }, WPOLY, c);
        for (int k = 0; k < WPOLY; ++k) wt->hp[(W + a) * WPOLY + k] = (float)c[k];
    }
    if (mom) {
        // transform of the moment-form spread, CC[(y, z)][q = 8 k + l] = C[y][k] C[z][l] x
        // 2^MOM_CC_SHIFT, as A operands: per (yz block jb, K-step pair sp, part hi / lo, lane),
        // row (y, z) from lane % 16, K elements q = 16 (2 sp) + 4 (lane / 16) + i then
        // q = 16 (2 sp + 1) + 4 (lane / 16) + i, i < 4
        const int NZ = (W + 3) / 4, NB = NZ * NZ, NP = WPOLY * WPOLY / 32;
        wt->cc.assign((size_t)NB * NP * 2 * 64 * 8, 0);
        const double up = std::ldexp(1.0, MOM_CC_SHIFT);
        double amax = 0.0;
        for (int jb = 0; jb < NB; ++jb)
            for (int sp = 0; sp < NP; ++sp)
                for (int ln = 0; ln < 64; ++ln) {
                    const int col = ln & 15, grp = ln >> 4;
                    const int y = 4 * (jb / NZ) + (col >> 2), z = 4 * (jb % NZ) + (col & 3);
                    uint16_t *hi = wt->cc.data() + ((size_t)((jb * NP + sp) * 2 + 0) * 64 + ln) * 8;
                    uint16_t *lo = wt->cc.data() + ((size_t)((jb * NP + sp) * 2 + 1) * 64 + ln) * 8;
                    for (int t = 0; t < 8; ++t) {
                        const int q = 16 * (2 * sp + t / 4) + 4 * grp + t % 4;
                        const int k = q / WPOLY, l = q % WPOLY;
                        const double v =
                            (y < W && z < W) ? cheb[y * WPOLY + k] * cheb[z * WPOLY + l] * up : 0.0;
                        amax = std::max(amax, std::fabs(v));
                        const _Float16 h = (_Float16)(float)v;
                        const _Float16 r = (_Float16)(float)(v - (double)(float)h);
                        hi[t] = __builtin_bit_cast(uint16_t, h);
                        lo[t] = __builtin_bit_cast(uint16_t, r);
                    }
                }
        FS_REQUIRE(amax < 65504.0, FS_EUNSUPPORTED,
                   "window transform %g outside the FP16 range (window %d)", amax, W);
    }
    std::lock_guard<std::mutex> lk(g_win_mu);
    if (g_win.size() >= WIN_CACHE) g_win.clear();
    g_win.emplace(key, wt);
    return wt;
}
}  // namespace

void plan_build(Plan &pl, const float *x, int64_t n, const float *y, int64_t m, int d,
                const fs_params &p, hipStream_t s) {
    PlanParams &pp = pl.pp;
    pl.flags = p.flags;
    pp.stable = (p.flags & FS_FLAG_DETERMINISTIC) != 0;
    pp.d = d;
    pp.kind = p.kernel;
    pp.lambda = p.lambda;
    pp.G = p.grid;
    pp.sigma = p.oversampling ? p.oversampling : 2;
    pp.m = p.window ? p.window : 6;
    pp.W = 2 * pp.m;
    pp.p = p.smoothness ? p.smoothness : 8;
    FS_REQUIRE(d >= 1 && d <= 3, FS_EDOMAIN, "NFFT fast summation supports d in 1..3 (got %d)", d);
    FS_REQUIRE(pp.G >= 16 && pp.G <= 512 && (pp.G & (pp.G - 1)) == 0, FS_EINVAL,
               "grid must be a power of two in 16..512 (got %d)", pp.G);
    if (p.bandwidth > 0) {
        pp.N = p.bandwidth;
        FS_REQUIRE(pp.N % 2 == 0 && pp.N >= 4 && pp.N + 2 <= pp.G, FS_EINVAL,
                   "bandwidth must be even, >= 4 and <= grid - 2 (got %d for grid %d)", pp.N, pp.G);
    } else {
        FS_REQUIRE(pp.sigma >= 2 && pp.G % pp.sigma == 0, FS_EINVAL,
                   "oversampling must be an integer >= 2 dividing the grid (got %d)", pp.sigma);
        pp.N = pp.G / pp.sigma;
        FS_REQUIRE(pp.N >= 4 && pp.N % 2 == 0, FS_EINVAL, "bandwidth grid/oversampling must be even >= 4");
    }
    FS_REQUIRE(pp.m >= 2 && pp.m <= 8, FS_EINVAL, "window cutoff must be in 2..8 (got %d)", pp.m);
    FS_REQUIRE(pp.W <= pp.G, FS_EINVAL, "window support 2m=%d exceeds the grid %d", pp.W, pp.G);
    FS_REQUIRE(pp.p >= 2 && pp.p <= 16, FS_EINVAL, "smoothness must be in 2..16 (got %d)", pp.p);
    FS_REQUIRE(pp.kind == FS_GAUSS || pp.kind == FS_LAPLACE || pp.kind == FS_ENERGY ||
                   pp.kind == FS_IMQ, FS_EINVAL, "unknown kernel %d", pp.kind);
    FS_REQUIRE(pp.kind == FS_ENERGY || (pp.lambda > 0 && std::isfinite(pp.lambda)), FS_EINVAL,
               "lambda must be positive");
    pp.T = (d == 3) ? 8 : 32;
    if (pp.T > pp.G) pp.T = pp.G;
    const int64_t nmax = std::max(n, m);
    // chunk size: about 1000 chunks over the point set (four per CU), 64..2048 nodes
    int ch = 64;
    while (ch < 2048 && ch * 1024 < nmax) ch *= 2;
    pp.chunk = ch;

    // small host <-> device copies of the build (pinned staging, released at the end)
    HostStage hs(s);
    // window shape for the effective oversampling ratio G / N
    const double b = M_PI * (2.0 - (double)pp.N / pp.G);
    pp.kb.m = (float)pp.m;
    pp.kb.b = (float)b;
    pp.kb.inv_one_minus = (float)(1.0 / (-std::expm1(-2.0 * b * pp.m)));
    // ---- bounding box of both point sets (A1)
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    {
        const int nb = 512;
        // per-block partials of both sets, then the count of non-finite coordinates
        DevBuf<float> part(nb * 6 * 2 + 1);
        int *bad = reinterpret_cast<int *>(part.p + nb * 6 * 2);
        fill_f32(part.p, nb * 6 * 2 + 1, 0.0f, s);
        if (n > 0) {
            hipLaunchKernelGGL(k_bbox, dim3(nb), dim3(256), 0, s, x, n, d, part.p, bad);
            FS_LAUNCHED();
        }
        if (m > 0 && y != x) {
            hipLaunchKernelGGL(k_bbox, dim3(nb), dim3(256), 0, s, y, m, d, part.p + nb * 6, bad);
            FS_LAUNCHED();
        }
        const float *h = hs.download(part.p, (size_t)(nb * 12 + 1));
        const int *hb = reinterpret_cast<const int *>(h + nb * 12);
        // ---- window (independent of the data: prepared while the bounding box is reduced)
        const bool mom = d == 3 && pp.W + BRICK_X - 1 <= 16;
        const std::shared_ptr<const WindowTables> wt = window_tables(pp.m, pp.N, pp.G, mom);
        pl.wpoly.alloc(wt->hp.size());
        hs.upload(pl.wpoly.p, wt->hp.data(), wt->hp.size() * sizeof(float));
        if (mom) {
            pl.mom_cc.alloc(wt->cc.size() / 8);
            hs.upload(pl.mom_cc.p, wt->cc.data(), wt->cc.size() * sizeof(uint16_t));
        }
        FS_HIP(hipStreamSynchronize(s));
        FS_REQUIRE(*hb == 0, FS_EDOMAIN, "non-finite point coordinates");
        for (int set = 0; set < 2; ++set) {
            if ((set == 0 && n == 0) || (set == 1 && (m == 0 || y == x))) continue;
            for (int b = 0; b < nb; ++b)
                for (int k = 0; k < d; ++k) {
                    lo[k] = std::min(lo[k], (double)h[set * nb * 6 + b * 6 + k]);
                    hi[k] = std::max(hi[k], (double)h[set * nb * 6 + b * 6 + 3 + k]);
                }
        }
    }
    double ext = 0.0, diag2 = 0.0;
    for (int k = 0; k < d; ++k) {
        if (!(lo[k] <= hi[k])) { lo[k] = hi[k] = 0.0; }
        pp.center[k] = 0.5 * (lo[k] + hi[k]);
        double e = hi[k] - lo[k];
        ext = std::max(ext, e);
        diag2 += e * e;
    }
    const double diag = std::sqrt(diag2);

    // ---- period and regularisation (Section "approximation aspects": K is replaced by a smooth
    //      periodic K_R; "heuristic stabilisation": the data are rescaled into the torus)
    const double tolK = 1e-10, ltol = std::log(1.0 / tolK);
    double Pcube = INFINITY;
    if (pp.kind == FS_GAUSS) {
        const double rk = std::sqrt(pp.lambda * ltol);
        Pcube = std::max(ext + rk, 2.0 * rk);
    } else if (pp.kind == FS_LAPLACE) {
        const double rk = pp.lambda * ltol;
        Pcube = std::max(ext + rk, 2.0 * rk);
    }
    // the boundary-regularised (ball) torus needs a boundary zone epsB = p/N narrower than the
    // half period; the cube periodisation needs a kernel that decays within the padding
    const double epsB_default = (double)pp.p / pp.N;
    const bool ball_ok = epsB_default < 0.4;
    const double Pball = ball_ok ? std::max(diag, 1e-6) / (0.5 - epsB_default) * (1.0 + 1e-6)
                                 : INFINITY;
    if (std::isfinite(Pcube) && Pcube <= Pball) {
        pp.regime = REGIME_CUBE;
        pp.P = Pcube;
        pp.epsB = 0.0;
    } else {
        FS_REQUIRE(ball_ok, FS_EINVAL,
                   "smoothness %d too large for bandwidth %d: the boundary regularisation needs "
                   "p/N < 0.4 (raise grid or lower smoothness)", pp.p, pp.N);
        pp.regime = REGIME_BALL;
        pp.P = Pball;
        pp.epsB = epsB_default;
    }
    pp.nearfield = (pp.kind != FS_GAUSS);
    if (pp.kind != FS_GAUSS) {
        pp.epsI = (p.nearfield_radius > 0) ? p.nearfield_radius / pp.P : (double)pp.p / pp.N;
        FS_REQUIRE(pp.epsI < 0.5 - pp.epsB - 1e-9 && pp.epsI > 0, FS_EINVAL,
                   "near-field radius %g (torus %g) incompatible with the torus size",
                   p.nearfield_radius, pp.epsI);
        inner_poly(pp.kind, pp.lambda, pp.P, pp.epsI, pp.p, pp.ci);
    } else {
        pp.epsI = 0.0;
    }
    if (pp.regime == REGIME_BALL) boundary_poly(pp.kind, pp.lambda, pp.P, pp.epsB, pp.p, pp.cb);

    // ---- bin the point sets (A2)
    pl.same = (y == x && m == n);
    {
        BinBuild bx, by;
        bin_nodes_count(pl.X, bx, x, n, pp, s, hs);
        if (!pl.same) bin_nodes_count(pl.Y, by, y, m, pp, s, hs);
        FS_HIP(hipStreamSynchronize(s));
        bin_nodes_finish(pl.X, bx, pp, s, hs);
        if (!pl.same) bin_nodes_finish(pl.Y, by, pp, s, hs);
    }

    if (pp.nearfield) {
        // cells of side about radius / R, R chosen so that a cell holds about 32 points: blocks of
        // 64 targets then span a few cells of a row, and the distance pruning of the stencil
        // keeps about 2.4 times the ball's volume in 3-D.  The side is raised where needed to
        // keep the cell grid within 4000 per dimension and 2^24 cells; the stencil half-width is
        // then ceil(radius / side), so the stencil always covers the radius.
        {
            double vol = 1.0, ext = 0.0;
            for (int k = 0; k < d; ++k) {
                vol *= std::max(hi[k] - lo[k], 1e-12);
                ext = std::max(ext, hi[k] - lo[k]);
            }
            const double dens = (double)std::max<int64_t>(std::max(n, m), 1) / vol;
            const double ht = std::pow(32.0 / dens, 1.0 / d);
            const double r = pp.epsI * pp.P;
            const int R0 = (int)std::max(1.0, std::min(6.0, std::round(r / ht)));
            double h = r * (1.0 + 1e-6) / R0;
            h = std::max(h, ext / 4000.0);
            h = std::max(h, std::pow(vol / double(1 << 24), 1.0 / d));
            pp.nf_h = h;
            pp.nf_R = std::max(1, (int)std::ceil(r / h));
        }
        for (int k = 0; k < 3; ++k) {
            pp.nf_lo[k] = (k < d) ? lo[k] : 0.0;
            pp.nf_dims[k] = 1;
        }
        int64_t ncells = 1;
        for (int k = 0; k < d; ++k) {
            int64_t dk = (int64_t)std::floor((hi[k] - lo[k]) / pp.nf_h) + 1;
            FS_REQUIRE(dk <= 8192, FS_EINVAL, "near-field cell grid too large");
            pp.nf_dims[k] = (int)dk;
            ncells *= dk;
        }
        FS_REQUIRE(ncells < (int64_t(1) << 26), FS_EINVAL, "near-field cell grid too large");
        build_nearfield_cells(pl.X, pp, s);
        if (!pl.same) build_nearfield_cells(pl.Y, pp, s);
        pl.nf_src.alloc(std::max(pl.X.n, pl.same ? 0 : pl.Y.n) + 4);
    }

    // ---- Fourier coefficients b_k of K_R and the multiplier M_k (A3)
    const MultKey mkey = mult_key(pp, b);
    bool mult_cached = false;
    {
        const int N = pp.N, H = N / 2 + 1;
        int64_t nh = 1;
        for (int k = 0; k < d; ++k) nh *= H;
        std::lock_guard<std::mutex> lk(g_mult_mu);
        for (size_t i = 0; i < g_mult.size(); ++i)
            if (std::memcmp(&g_mult[i]->key, &mkey, sizeof(mkey)) == 0) {
                const MultEntry &e = *g_mult[i];
                pl.Mk.alloc(nh);
                FS_HIP(hipStreamWaitEvent(s, e.ready, 0));
                FS_HIP(hipMemcpyAsync(pl.Mk.p, e.mk.p, nh * sizeof(float),
                                      hipMemcpyDeviceToDevice, s));
                std::rotate(g_mult.begin() + i, g_mult.begin() + i + 1, g_mult.end());
                mult_cached = true;
                break;
            }
    }
    if (!mult_cached) {
        const int N = pp.N, H = N / 2 + 1;
        int64_t nsamp = 1, nh = 1;
        for (int k = 0; k < d; ++k) { nsamp *= N; nh *= H; }
        DevBuf<double> samp(nsamp), t1(nsamp), t2(nsamp), costab(N), dconv(H);
        std::vector<double> hc(N), hd(H);
        for (int q = 0; q < N; ++q) hc[q] = std::cos(2.0 * M_PI * q / N);
        for (int k = 0; k < H; ++k) {
            const double ph = kb_hat(pp.m, b, pp.G, k);
            hd[k] = 1.0 / ((double)pp.G * pp.G * ph * ph);
        }
        hs.upload(costab.p, hc.data(), N * sizeof(double));
        hs.upload(dconv.p, hd.data(), H * sizeof(double));
        RegArgs ra{};
        ra.kind = pp.kind;
        ra.regime = pp.regime;
        ra.p = pp.p;
        ra.lambda = pp.lambda;
        ra.P = pp.P;
        ra.epsI = pp.epsI;
        ra.epsB = pp.epsB;
        std::memcpy(ra.ci, pp.ci, sizeof(ra.ci));
        std::memcpy(ra.cb, pp.cb, sizeof(ra.cb));
        {
            const dim3 g(blocks_for(nsamp, 256, 65536)), b(256);
            switch (pp.kind) {
                case FS_GAUSS: hipLaunchKernelGGL(k_sample_kr<FS_GAUSS>, g, b, 0, s, ra, N, d, samp.p); break;
                case FS_LAPLACE: hipLaunchKernelGGL(k_sample_kr<FS_LAPLACE>, g, b, 0, s, ra, N, d, samp.p); break;
                case FS_IMQ: hipLaunchKernelGGL(k_sample_kr<FS_IMQ>, g, b, 0, s, ra, N, d, samp.p); break;
                default: hipLaunchKernelGGL(k_sample_kr<FS_ENERGY>, g, b, 0, s, ra, N, d, samp.p); break;
            }
        }
        FS_LAUNCHED();
        // axis 0 (fastest): A = N^{d-1}, B = 1 ; axis 1: A = N^{d-2}, B = H ; axis 2: A = 1, B = H^2
        const double *in = samp.p;
        double *outs[3] = {t1.p, t2.p, t1.p};
        int64_t B = 1, A = nsamp / N;
        for (int ax = 0; ax < d; ++ax) {
            const int64_t work = A * H * B;
            hipLaunchKernelGGL(k_cos_dft, dim3(blocks_for(work, 256, 65536)), dim3(256), 0, s, in, A,
                               N, B, costab.p, outs[ax]);
            FS_LAUNCHED();
            in = outs[ax];
            B *= H;
            A /= N;
        }
        pl.Mk.alloc(nh);
        const double scale = std::pow((double)N, -(double)d);
        hipLaunchKernelGGL(k_build_mult, dim3(blocks_for(nh, 256, 65536)), dim3(256), 0, s, in, N,
                           d, dconv.p, scale, pl.Mk.p);
        FS_LAUNCHED();
        hs.hold(samp);
        hs.hold(t1);
        hs.hold(t2);
        hs.hold(costab);
        hs.hold(dconv);
        std::lock_guard<std::mutex> lk(g_mult_mu);
        if (g_mult.size() >= MULT_CACHE) {
            FS_HIP(hipDeviceSynchronize());  // no queued copy still reads the oldest entry
            FS_HIP(hipEventDestroy(g_mult.front()->ready));
            g_mult.erase(g_mult.begin());
        }
        {
            auto e = std::make_unique<MultEntry>();
            e->key = mkey;
            e->mk.alloc(nh);
            FS_HIP(hipMemcpyAsync(e->mk.p, pl.Mk.p, nh * sizeof(float), hipMemcpyDeviceToDevice,
                                  s));
            FS_HIP(hipEventCreateWithFlags(&e->ready, hipEventDisableTiming));
            FS_HIP(hipEventRecord(e->ready, s));
            g_mult.push_back(std::move(e));
        }
    }

    // ---- FFT buffers and twiddles
    {
        const int G = pp.G, N = pp.N, KX = N / 2 + 1;
        int64_t gsz = 1;
        for (int k = 0; k < d; ++k) gsz *= G;
        pl.grid.alloc(gsz);
        if (d >= 2) pl.specA.alloc((gsz / G) * KX);
        if (d == 3) pl.specB.alloc((int64_t)G * (N + 1) * KX);
        std::vector<float2> tw(G / 2);
        for (int q = 0; q < G / 2; ++q) {
            double a = -2.0 * M_PI * q / G;
            tw[q] = make_float2((float)std::cos(a), (float)std::sin(a));
        }
        pl.twiddle.alloc(G / 2);
        hs.upload(pl.twiddle.p, tw.data(), tw.size() * sizeof(float2));
        const int S = pp.T + pp.W - 1;
        int64_t box = 1;
        for (int k = 0; k < d; ++k) box *= S;
        const int nch = std::max({pl.X.nchunks, pl.same ? 0 : pl.Y.nchunks, pl.X.n_mblocks,
                                  pl.same ? 0 : pl.Y.n_mblocks});
        pl.scratch.alloc((int64_t)std::max(nch, 1) * box);
    }
    // the stage's destructor synchronises the stream: the plan is complete on return
}

// ------------------------------------------------------------------ apply
namespace {

// The matrix-core spread and gather (d = 3) pay per group of up to 16 nodes; the lane-per-node
// kernels pay per node.  The groups are used when they hold MIN_GROUP_FILL nodes on average.
constexpr int MIN_GROUP_FILL = 4;
// Grids of at most this many tiles are folded whole (untouched tiles write their zeros), which
// saves the separate clearing pass.
constexpr int64_t FOLD_ALL_TILES = 4096;
bool use_mfma(const Plan &pl, const Nodes &nd) {
    return !(pl.flags & FS_FLAG_FORCE_VALU) && nd.n_mblocks > 0 &&
           nd.n >= (int64_t)MIN_GROUP_FILL * nd.n_mgroups;
}

template <int D, int W>
void launch_spread_gather(Plan &pl, const Nodes &src, const Nodes &dst, const float *w,
                          float *t, float *grad, hipStream_t s, const PotWeights *pw = nullptr,
                          const PotUpdate *pu = nullptr) {
    const PlanParams &pp = pl.pp;
    SpreadArgs sa{pp.kb, pp.G, pp.T, pp.G / pp.T, pp.m, pl.wpoly.p, pl.mom_cc.p};
    // the tile side shrinks to the grid size for small grids
    auto run = [&](auto tconst) {
        constexpr int T = decltype(tconst)::value;
        // the spread writes one box per chunk (or per matrix-core block); tile_chunk maps a tile
        // to its boxes and multi_tiles lists the tiles with several
        bool mf = false;
        const int *tile_boxes = src.tile_chunk.p, *multi = src.multi_tiles;
        int n_multi = src.n_multi;
        if (src.nchunks > 0) {
            ProfScope ps("spread", s);
            if constexpr (D == 1) {
                hipLaunchKernelGGL((k_spread<D, W, T>), dim3(src.nchunks), dim3(256), 0, s,
                                   src.rec.p, w, src.chunks.p, sa, pl.scratch.p);
            } else {
                if constexpr (D >= 2 && W + BRICK_X - 1 <= 16) mf = use_mfma(pl, src);
                FS_REQUIRE(!pw || mf, FS_EINVAL, "weights from potentials need the matrix-core spread");
                if (mf) {
                    if constexpr (D == 2 && W + BRICK_X - 1 <= 16) {
                        if (pw)
                            hipLaunchKernelGGL((k_spread_mfma2d<W, T, true>), dim3(src.n_mblocks),
                                               dim3(64 * MW), 0, s, src.rec.p, w, src.mblocks.p,
                                               src.mgroups.p, src.mbnodes.p, sa, pl.scratch.p,
                                               *pw);
                        else
                            hipLaunchKernelGGL((k_spread_mfma2d<W, T, false>), dim3(src.n_mblocks),
                                               dim3(64 * MW), 0, s, src.rec.p, w, src.mblocks.p,
                                               src.mgroups.p, src.mbnodes.p, sa, pl.scratch.p,
                                               PotWeights{});
                    }
                    if constexpr (D == 3 && W + BRICK_X - 1 <= 16) {
                        if (pw)
                            hipLaunchKernelGGL((k_spread_mom16<W, true>), dim3(src.n_mblocks),
                                               dim3(64 * MW), 0, s, src.rec.p, w, src.mblocks.p,
                                               src.mgroups.p, src.mbnodes.p, sa, pl.scratch.p,
                                               *pw);
                        else
                            hipLaunchKernelGGL((k_spread_mom16<W, false>), dim3(src.n_mblocks),
                                               dim3(64 * MW), 0, s, src.rec.p, w, src.mblocks.p,
                                               src.mgroups.p, src.mbnodes.p, sa, pl.scratch.p,
                                               PotWeights{});
                    }
                    tile_boxes = src.mtile_block;
                    multi = src.mmulti_tiles;
                    n_multi = src.n_mmulti;
                } else {
                    hipLaunchKernelGGL((k_spread_wave<D, W, T>), dim3(src.nchunks), dim3(256), 0,
                                       s, src.rec.p, w, src.chunks.p, sa, pl.scratch.p);
                }
            }
            FS_LAUNCHED();
        }
        int64_t gsz = 1;
        for (int k = 0; k < D; ++k) gsz *= pp.G;
        if (src.nchunks > 0) {
            ProfScope ps("fold", s);
            const int S = T + W - 1, ntd = pp.G / T;
            int64_t ntiles = 1;
            for (int k = 0; k < D; ++k) ntiles *= ntd;
            int box = 1;
            for (int k = 0; k < D; ++k) box *= S;
            // one thread per element of the boxes to reduce when that fills the chip, else the
            // chunks are split over four waves per element
            const unsigned nt = (unsigned)std::min(n_multi, 65535);
            if (n_multi > 0 && (int64_t)n_multi * box >= 131072) {
                hipLaunchKernelGGL(k_reduce_chunks, dim3((box + 255) / 256, nt), dim3(256), 0, s,
                                   pl.scratch.p, tile_boxes, multi, n_multi, box);
                FS_LAUNCHED();
            } else if (n_multi > 0) {
                hipLaunchKernelGGL(k_reduce_chunks_split, dim3((box + 63) / 64, nt), dim3(256), 0,
                                   s, pl.scratch.p, tile_boxes, multi, n_multi, box);
                FS_LAUNCHED();
            }
            if (ntd >= 3 && S <= pp.G && pp.m <= T) {
                // the T^d points of a tile are split over blocks of 64 threads; on large grids
                // only the tiles with a chunk in their 3^d neighbourhood are folded and the rest
                // of the grid is cleared, on small ones every tile is folded (zeros included)
                int npts = 1;
                for (int k = 0; k < D; ++k) npts *= T;
                const bool all = src.n_touched == ntiles || ntiles <= FOLD_ALL_TILES;
                if (!all) fill_f32(pl.grid.p, gsz, 0.0f, s);
                const unsigned nfold = all ? (unsigned)ntiles : (unsigned)src.n_touched;
                if (nfold > 0)
                    hipLaunchKernelGGL(k_fold_tiles<D>, dim3(nfold, (unsigned)((npts + 255) / 256)),
                                       dim3(256), 0, s, pl.scratch.p, tile_boxes,
                                       all ? nullptr : src.touched_tiles, pp.G, T, ntd, pp.m, S,
                                       pl.grid.p);
            } else {
                hipLaunchKernelGGL(k_fold<D>, dim3(blocks_for(gsz, 256, 1 << 16)), dim3(256), 0, s,
                                   pl.scratch.p, tile_boxes, pp.G, T, ntd, pp.m, S, pl.grid.p);
            }
            FS_LAUNCHED();
        } else {
            fill_f32(pl.grid.p, gsz, 0.0f, s);
        }
        {
        // FFT -> multiply -> inverse FFT
            ProfScope pf("fft", s);
            FftArgs fa{};
            fa.G = pp.G;
            fa.logG = 0;
            while ((1 << fa.logG) < pp.G) ++fa.logG;
            fa.N = pp.N;
            fa.KX = pp.N / 2 + 1;
            // launch shapes: enough workgroups to cover the chip (about 512), at most FFT_ELEMS
            // complex elements per LDS buffer, threads = butterflies per stage (64..256)
            const int maxcols = FFT_ELEMS / pp.G;
            auto threads_for = [&](int transforms) {
                int t = transforms * pp.G / 2;
                t = std::max(64, std::min(256, (t + 63) / 64 * 64));
                return t;
            };
            if (D == 1) {
                fa.nb = 1;
                hipLaunchKernelGGL(k_fft_1d_conv, dim3(1), dim3(threads_for(1)),
                                   2 * pp.G * sizeof(float2), s, pl.grid.p, fa, pl.twiddle.p, pl.Mk.p);
                FS_LAUNCHED();
            } else {
                const int rows = (int)(gsz / pp.G);
                const int pairs = rows / 2;
                fa.nb = std::max(1, std::min(maxcols, pairs / 512));
                const unsigned xblocks = (pairs + fa.nb - 1) / fa.nb;
                const int ylines = (D == 2) ? 1 : pp.G;  // strided pencils per column block
                int nbx = std::max(1, std::min(maxcols, fa.KX * ylines / 512));
                int nkb = (fa.KX + nbx - 1) / nbx;
                fa.nbx = (fa.KX + nkb - 1) / nkb;  // balanced column blocks
                nkb = (fa.KX + fa.nbx - 1) / fa.nbx;
                const size_t lds_x = 2 * (size_t)fa.nb * pp.G * sizeof(float2);
                const size_t lds_y = 2 * (size_t)fa.nbx * pp.G * sizeof(float2);
                // 3-D on a 64^3 grid: z slabs (forward x and y, the z columns, inverse y and x)
                if (D == 3 && pp.G == 64 && pp.N < pp.G) {
                    const int ncol = (pp.N + 1) * fa.KX;
                    hipLaunchKernelGGL(k_fft_xy_fwd64, dim3(pp.G), dim3(256), 0, s, pl.grid.p, fa,
                                       pl.twiddle.p, pl.specB.p);
                    FS_LAUNCHED();
                    hipLaunchKernelGGL(k_fft_z_conv64, dim3((ncol + FFT_ZCOLS - 1) / FFT_ZCOLS),
                                       dim3(64), 0, s, pl.specB.p, fa, pl.twiddle.p, pl.Mk.p);
                    FS_LAUNCHED();
                    hipLaunchKernelGGL(k_fft_xy_inv64, dim3(pp.G), dim3(256), 0, s, pl.specB.p, fa,
                                       pl.twiddle.p, pl.grid.p);
                    FS_LAUNCHED();
                } else {
                    hipLaunchKernelGGL(k_fft_x_r2c, dim3(xblocks), dim3(threads_for(fa.nb)), lds_x, s,
                                       pl.grid.p, rows, fa, pl.twiddle.p, pl.specA.p);
                    FS_LAUNCHED();
                    if (D == 2) {
                        hipLaunchKernelGGL(k_fft_y<1>, dim3(nkb), dim3(threads_for(fa.nbx)), lds_y, s,
                                           pl.specA.p, pl.specB.p, fa, pl.twiddle.p, pl.Mk.p);
                        FS_LAUNCHED();
                    } else {
                        hipLaunchKernelGGL(k_fft_y<0>, dim3(pp.G * nkb), dim3(threads_for(fa.nbx)),
                                           lds_y, s, pl.specA.p, pl.specB.p, fa, pl.twiddle.p, pl.Mk.p);
                        FS_LAUNCHED();
                        hipLaunchKernelGGL(k_fft_z_conv, dim3((pp.N + 1) * nkb),
                                           dim3(threads_for(fa.nbx)), lds_y, s, pl.specB.p, fa,
                                           pl.twiddle.p, pl.Mk.p);
                        FS_LAUNCHED();
                        hipLaunchKernelGGL(k_fft_y<2>, dim3(pp.G * nkb), dim3(threads_for(fa.nbx)),
                                           lds_y, s, pl.specA.p, pl.specB.p, fa, pl.twiddle.p, pl.Mk.p);
                        FS_LAUNCHED();
                    }
                    hipLaunchKernelGGL(k_fft_x_c2r, dim3(xblocks), dim3(threads_for(fa.nb)), lds_x, s,
                                       pl.specA.p, rows, fa, pl.twiddle.p, pl.grid.p);
                    FS_LAUNCHED();
                }
            }
        }
        if (dst.n > 0) {
            if (dst.nchunks > 0) {
                ProfScope pg("gather", s);
                const float gscale = (float)(pp.G / pp.P);
                const unsigned split = (pp.chunk >= 512) ? 2 : 1;
                bool mf = false;
                if constexpr (D == 2 && W + BRICK_X - 1 <= 16) {
                    mf = !grad && use_mfma(pl, dst);
                    FS_REQUIRE(!pu || mf, FS_EINVAL, "the fused update needs the matrix-core gather");
                    if (mf && pu)
                        hipLaunchKernelGGL((k_gather_mfma2d<W, T, true>), dim3(dst.n_mblocks),
                                           dim3(64 * MW), 0, s, dst.rec.p, dst.mblocks.p,
                                           dst.mgroups.p, sa, pl.grid.p, nullptr, *pu);
                    else if (mf)
                        hipLaunchKernelGGL((k_gather_mfma2d<W, T, false>), dim3(dst.n_mblocks),
                                           dim3(64 * MW), 0, s, dst.rec.p, dst.mblocks.p,
                                           dst.mgroups.p, sa, pl.grid.p, t, PotUpdate{});
                }
                if constexpr (D == 3 && W + BRICK_X - 1 <= 16) {
                    mf = !grad && use_mfma(pl, dst);
                    FS_REQUIRE(!pu || mf, FS_EINVAL, "the fused update needs the matrix-core gather");
                    if (mf && pu)
                        hipLaunchKernelGGL((k_gather_mfma16<W, true>), dim3(dst.n_mblocks),
                                           dim3(64 * MW), 0, s, dst.rec.p, dst.mblocks.p,
                                           dst.mgroups.p, sa, pl.grid.p, nullptr, *pu);
                    else if (mf)
                        hipLaunchKernelGGL((k_gather_mfma16<W, false>), dim3(dst.n_mblocks),
                                           dim3(64 * MW), 0, s, dst.rec.p, dst.mblocks.p,
                                           dst.mgroups.p, sa, pl.grid.p, t, PotUpdate{});
                }
                if (mf) {
                    // launched above
                } else if (grad) {
                    hipLaunchKernelGGL((k_gather<D, W, T, true>), dim3(dst.nchunks, split), dim3(256),
                                       0, s, dst.rec.p, dst.chunks.p, sa, pl.grid.p, t, grad, gscale);
                } else {
                    hipLaunchKernelGGL((k_gather<D, W, T, false>), dim3(dst.nchunks, split),
                                       dim3(256), 0, s, dst.rec.p, dst.chunks.p, sa, pl.grid.p, t,
                                       grad, gscale);
                }
                FS_LAUNCHED();
            }
        }
    };
    if constexpr (D == 3) {
        FS_REQUIRE(pp.T == 8, FS_EUNSUPPORTED, "unsupported tile size %d for d=3", pp.T);
        run(std::integral_constant<int, 8>{});
    } else if constexpr (D == 2) {
        if (pp.T == 32) run(std::integral_constant<int, 32>{});
        else if (pp.T == 16) run(std::integral_constant<int, 16>{});
        else FS_REQUIRE(false, FS_EUNSUPPORTED, "unsupported tile size %d for d=2", pp.T);
    } else {
        switch (pp.T) {
            case 256: run(std::integral_constant<int, 256>{}); break;
            case 128: run(std::integral_constant<int, 128>{}); break;
            case 64: run(std::integral_constant<int, 64>{}); break;
            case 32: run(std::integral_constant<int, 32>{}); break;
            case 16: run(std::integral_constant<int, 16>{}); break;
            default: FS_REQUIRE(false, FS_EUNSUPPORTED, "unsupported tile size %d for d=1", pp.T);
        }
    }
}

template <int D>
void dispatch_w(Plan &pl, const Nodes &src, const Nodes &dst, const float *w, float *t,
                float *grad, hipStream_t s, const PotWeights *pw = nullptr,
                const PotUpdate *pu = nullptr) {
    switch (pl.pp.W) {
        case 4: return launch_spread_gather<D, 4>(pl, src, dst, w, t, grad, s, pw, pu);
        case 6: return launch_spread_gather<D, 6>(pl, src, dst, w, t, grad, s, pw, pu);
        case 8: return launch_spread_gather<D, 8>(pl, src, dst, w, t, grad, s, pw, pu);
        case 10: return launch_spread_gather<D, 10>(pl, src, dst, w, t, grad, s, pw, pu);
        case 12: return launch_spread_gather<D, 12>(pl, src, dst, w, t, grad, s, pw, pu);
        case 14: return launch_spread_gather<D, 14>(pl, src, dst, w, t, grad, s, pw, pu);
        case 16: return launch_spread_gather<D, 16>(pl, src, dst, w, t, grad, s, pw, pu);
        default: FS_REQUIRE(false, FS_EINVAL, "unsupported window %d", pl.pp.W);
    }
}

}  // namespace

bool plan_fuses_weights(const Plan &pl, int transpose) {
    const Nodes &src = pl.src(transpose);
    return (pl.pp.d == 3 || pl.pp.d == 2) && !pl.pp.nearfield && pl.pp.W + BRICK_X - 1 <= 16 &&
           use_mfma(pl, src) && src.nchunks > 0;
}

bool plan_fuses_update(const Plan &pl, int transpose) {
    const Nodes &dst = pl.dst(transpose);
    return plan_fuses_weights(pl, transpose) && use_mfma(pl, dst) && dst.nchunks > 0;
}

int plan_update_parts(const Plan &pl, int transpose) { return pl.dst(transpose).n_mblocks; }

int plan_source_blocks(const Plan &pl, int transpose) { return pl.src(transpose).n_mblocks; }

void plan_block_base_max(const Plan &pl, const float *base_sorted, int transpose, float *out,
                         hipStream_t s) {
    const Nodes &src = pl.src(transpose);
    if (src.n_mblocks == 0) return;
    hipLaunchKernelGGL(k_block_absmax, dim3(src.n_mblocks), dim3(256), 0, s, base_sorted,
                       src.mbnodes.p, out);
    FS_LAUNCHED();
}

void plan_apply_sorted_pot(Plan &pl, const PotWeights &pw, float *t_sorted, int transpose,
                           hipStream_t s, const PotUpdate *pu) {
    FS_REQUIRE(plan_fuses_weights(pl, transpose), FS_EINVAL,
               "weights from potentials need the matrix-core spread without near field");
    FS_REQUIRE(!pu || plan_fuses_update(pl, transpose), FS_EINVAL,
               "the fused update needs the matrix-core gather");
    if (pl.pp.d == 3)
        dispatch_w<3>(pl, pl.src(transpose), pl.dst(transpose), nullptr, t_sorted, nullptr, s, &pw,
                      pu);
    else
        dispatch_w<2>(pl, pl.src(transpose), pl.dst(transpose), nullptr, t_sorted, nullptr, s, &pw,
                      pu);
}

void plan_apply_sorted(Plan &pl, const float *w_sorted, float *t_sorted, float *grad,
                       int transpose, hipStream_t s) {
    const Nodes &src = pl.src(transpose);
    const Nodes &dst = pl.dst(transpose);
    switch (pl.pp.d) {
        case 1: dispatch_w<1>(pl, src, dst, w_sorted, t_sorted, grad, s); break;
        case 2: dispatch_w<2>(pl, src, dst, w_sorted, t_sorted, grad, s); break;
        default: dispatch_w<3>(pl, src, dst, w_sorted, t_sorted, grad, s); break;
    }
    if (pl.pp.nearfield && dst.n > 0 && src.n > 0 && dst.nf_nblocks > 0) {
        const PlanParams &pp = pl.pp;
        NearArgs na{};
        na.kind = pp.kind;
        na.p = pp.p;
        na.d = pp.d;
        na.lambda_inv = (float)(pp.kind == FS_LAPLACE ? -M_LOG2E / pp.lambda : 0.0);
        na.lambda_lin = (float)(pp.kind == FS_LAPLACE ? -1.0 / pp.lambda : 0.0);
        na.c2 = (float)(pp.kind == FS_IMQ ? pp.lambda * pp.lambda : 0.0);
        const double r = pp.epsI * pp.P;
        na.rinv = (float)(1.0 / r);
        na.r2max = (float)(r * r);
        for (int k = 0; k < 16; ++k) na.ci[k] = (k < pp.p) ? (float)pp.ci[k] : 0.0f;
        for (int k = 0; k + 1 < 16; ++k)
            na.dci[k] = (k + 1 < pp.p) ? (float)(2.0 * (k + 1) * pp.ci[k + 1]) : 0.0f;
        na.h_inv = (float)(1.0 / pp.nf_h);
        for (int k = 0; k < 3; ++k) {
            na.lo[k] = (float)pp.nf_lo[k];
            na.dims[k] = pp.nf_dims[k];
        }
        const float rr = (float)((r / pp.nf_h) * (r / pp.nf_h));
        ProfScope pn("nearfield", s);
        hipLaunchKernelGGL(k_nf_pack, dim3(blocks_for(src.n + 4, 256, int64_t(1) << 30)),
                           dim3(256), 0, s, src.nf_xs.p, src.nf_order.p, w_sorted, src.n, pp.d,
                           pl.nf_src.p);
        FS_LAUNCHED();
        const int np = (pp.p <= 4) ? 4 : (pp.p <= 8) ? 8 : (pp.p <= 12) ? 12 : 16;
        // few target blocks (small or low-dimensional sets): split every block's sources over
        // several waves so that the launch still fills the chip
        // (deterministic mode: one wave per block, the partial sums would meet through atomics)
        const int split = pp.stable ? 1 : (int)std::min<int64_t>(64, std::max<int64_t>(1, (8192 + dst.nf_nblocks - 1) / dst.nf_nblocks));
        const dim3 g((unsigned)dst.nf_nblocks, (unsigned)split), b(64);
#define FS_NF(DD, KK, NN, GG)                                                                    \
    hipLaunchKernelGGL((k_nearfield<DD, KK, NN, GG>), g, b, 0, s, dst.nf_blocks.p, dst.nf_xs.p, \
                       dst.nf_order.p, src.nf_cell_start.p, pl.nf_src.p, na, pp.nf_R, rr,     \
                       t_sorted, grad)
#define FS_NF_NP(DD, KK, GG)                                \
    do {                                                    \
        if (np == 4) FS_NF(DD, KK, 4, GG);                  \
        else if (np == 8) FS_NF(DD, KK, 8, GG);             \
        else if (np == 12) FS_NF(DD, KK, 12, GG);           \
        else FS_NF(DD, KK, 16, GG);                         \
    } while (0)
#define FS_NF_K(DD, GG)                                                                       \
    do {                                                                                      \
        if (pp.kind == FS_LAPLACE) FS_NF_NP(DD, FS_LAPLACE, GG);                               \
        else if (pp.kind == FS_IMQ) FS_NF_NP(DD, FS_IMQ, GG);                                  \
        else FS_NF_NP(DD, FS_ENERGY, GG);                                                      \
    } while (0)
        if (grad) {
            if (pp.d == 1) FS_NF_K(1, true); else if (pp.d == 2) FS_NF_K(2, true); else FS_NF_K(3, true);
        } else {
            if (pp.d == 1) FS_NF_K(1, false); else if (pp.d == 2) FS_NF_K(2, false); else FS_NF_K(3, false);
        }
#undef FS_NF_K
#undef FS_NF_NP
#undef FS_NF
        FS_LAUNCHED();
    }
}

}  // namespace fs
