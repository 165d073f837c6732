// Unbalanced Sinkhorn (Algorithm 2), MMD (eq. (1205)), Sinkhorn divergence (eq. (586)) and the
// envelope gradients, on top of the kernel-sum operators.
//
// Precision split: the kernel sums (spread / FFT / gather, or the direct pair loop) run in FP32;
// the potential updates, the weights' exponent shift and every final reduction run in FP64.
//
// Log-domain bookkeeping.  With k_ij = exp(-C_ij / eps) and kappa = rho / (rho + eps), the beta
// half-step of eq. (Sinkhorn_uot_iteration) is
//     f_i = -eps kappa log sum_j k_ij b_j e^{g_j/eps}.
// The sum is formed with shifted weights  w_j = b_j e^{(g_j - gmax)/eps} in (0, b_j]  (so FP32
// cannot overflow), and the shift is added back in FP64:
//     f_i = -kappa (gmax + eps log t_i),   t_i = sum_j k_ij w_j.
#include <cfloat>

#include "solver.h"

#include <vector>

namespace fs {

// =====================================================================================
//                                        kernels
// =====================================================================================
namespace {

constexpr int RT = 256;     // threads for reductions
constexpr int RBLK = 1024;  // max blocks for reductions

__device__ __forceinline__ void nadd(double &s, double &c, double v) {
    double t = s + v;
    if (fabs(s) >= fabs(v)) c += (s - t) + v; else c += (v - t) + s;
    s = t;
}

// Largest v over the workgroup (wave shuffles, then one value per wave through `red`, which must
// hold blockDim.x / 64 doubles); every thread gets the result.
__device__ __forceinline__ double block_max(double v, double *red) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    __syncthreads();  // red may still be read by a previous call
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double m = red[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) m = fmax(m, red[i]);
    return m;
}

// w_k = base_k exp((pot_k - pmax) / eps)  (weight_exp: FP64 exponent, FP32 result), pmax the max
// of the nparts per-block maxima written by the update kernel (or a single value, nparts = 1).
__global__ void __launch_bounds__(256) k_weights(const float *__restrict__ base,
                                                 const double *__restrict__ pot,
                                                 const double *__restrict__ parts, int nparts,
                                                 double inv_eps, int64_t n, float *__restrict__ w) {
    __shared__ double red[4];
    double mx = -INFINITY;
    for (int b = threadIdx.x; b < nparts; b += blockDim.x) mx = fmax(mx, parts[b]);
    mx = block_max(mx, red);
    const double pm = (mx == -INFINITY) ? 0.0 : mx;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        w[i] = weight_exp(base[i], (pot[i] - pm) * inv_eps);
}

// u_k = (log base_k + (pot_k - pmax) / eps) log2 e in FP64, rounded to FP32 (-inf for a zero
// weight): the log source weights of the log-domain direct sums, in log2 units.
__global__ void __launch_bounds__(256) k_log_weights(const float *__restrict__ base,
                                                     const double *__restrict__ pot,
                                                     const double *__restrict__ parts, int nparts,
                                                     double inv_eps, int64_t n,
                                                     float *__restrict__ u) {
    __shared__ double red[4];
    double mx = -INFINITY;
    for (int b = threadIdx.x; b < nparts; b += blockDim.x) mx = fmax(mx, parts[b]);
    mx = block_max(mx, red);
    const double pm = (mx == -INFINITY) ? 0.0 : mx;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float b = base[i];
        u[i] = b > 0.0f ? (float)((log((double)b) + (pot[i] - pm) * inv_eps) * 1.4426950408889634)
                        : -INFINITY;
    }
}

// pot_i = -kappa (shift + eps log t_i) in FP64, shift = max of the other potential (the max of
// nshift per-block maxima); writes one block maximum of the new potential per block.  Non-positive
// sums are counted in *nbad and replaced by the smallest normal float.
constexpr int UPD_BLOCKS = 1024;
// With DELTA the per-block maxima of |new - old| go to delta_parts (stopping rule).
template <bool DELTA>
__global__ void __launch_bounds__(RT) k_update(const float *__restrict__ t, int64_t n,
                                               const double *__restrict__ shift_parts, int nshift,
                                               double kappa, double eps, double *__restrict__ pot,
                                               double *__restrict__ out_parts,
                                               int *__restrict__ nbad,
                                               double *__restrict__ delta_parts) {
    __shared__ double red[RT / 64];
    double sh = -INFINITY;
    for (int b = threadIdx.x; b < nshift; b += RT) sh = fmax(sh, shift_parts[b]);
    sh = block_max(sh, red);
    if (sh == -INFINITY) sh = 0.0;
    double mx = -INFINITY, dmx = 0.0;
    int bad = 0;
    // four elements per thread and step, their loads issued together
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i0 < n; i0 += 4 * stride) {
        float v[4];
        double o[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t i = i0 + k * stride;
            v[k] = (i < n) ? t[i] : 1.0f;
            o[k] = (DELTA && i < n) ? pot[i] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t i = i0 + k * stride;
            if (i < n) {
                float vk = v[k];
                if (!(vk > 0.0f)) { bad++; vk = FLT_MIN; }
                const double f = -kappa * (sh + eps * sum_log(vk));
                if (DELTA) dmx = fmax(dmx, fabs(f - o[k]));
                pot[i] = f;
                mx = fmax(mx, f);
            }
        }
    }
    if (bad) atomicAdd(nbad, bad);
    mx = block_max(mx, red);
    if (threadIdx.x == 0) out_parts[blockIdx.x] = mx;
    if (DELTA) {
        dmx = block_max(dmx, red);
        if (threadIdx.x == 0) delta_parts[blockIdx.x] = dmx;
    }
}

// The same update from log t_i given in FP64 (the log-domain direct sums); a row with no
// positive term (log t = -inf) is counted in *nbad and treated like the smallest normal float.
template <bool DELTA>
__global__ void __launch_bounds__(RT) k_update_log(const double *__restrict__ logt, int64_t n,
                                                   const double *__restrict__ shift_parts,
                                                   int nshift, double kappa, double eps,
                                                   double *__restrict__ pot,
                                                   double *__restrict__ out_parts,
                                                   int *__restrict__ nbad,
                                                   double *__restrict__ delta_parts) {
    __shared__ double red[RT / 64];
    double sh = -INFINITY;
    for (int b = threadIdx.x; b < nshift; b += RT) sh = fmax(sh, shift_parts[b]);
    sh = block_max(sh, red);
    if (sh == -INFINITY) sh = 0.0;
    double mx = -INFINITY, dmx = 0.0;
    int bad = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double l = logt[i];
        if (!(l > -INFINITY) || l != l) {
            bad++;
            l = log((double)FLT_MIN);
        }
        const double f = -kappa * (sh + eps * l);
        if (DELTA) dmx = fmax(dmx, fabs(f - pot[i]));
        pot[i] = f;
        mx = fmax(mx, f);
    }
    if (bad) atomicAdd(nbad, bad);
    mx = block_max(mx, red);
    if (threadIdx.x == 0) out_parts[blockIdx.x] = mx;
    if (DELTA) {
        dmx = block_max(dmx, red);
        if (threadIdx.x == 0) delta_parts[blockIdx.x] = dmx;
    }
}

// ------------------------------------------------------------------ floor rows
// The fast sum's absolute error is a small fraction (about 2e-7 measured) of the largest sum of a
// launch, so a row whose sum is far below the largest (a target far from every weighted source)
// carries that floor as a large relative error.  With rho >> eps the plan keeps such a row's mass,
// so its potential and its envelope gradient would inherit the error.  Rows whose sum is below
// FLOOR_REL of the largest are therefore re-evaluated directly, in the log domain, against every
// source (a wave per row): the Sinkhorn update from L_i = log sum_j b_j e^{(g_j - gmax - C_ij)/eps}
// and the gradient from the same softmax weights.
constexpr float FLOOR_REL = 1e-2f;

// Source side of a direct re-evaluation, in operator order: coordinates, base weights and the
// potential that forms the weights base_j e^{(pot_j - shift)/eps}.
struct FloorSrc {
    const float *xt;    // target coordinates (n x d)
    const float *ys;    // source coordinates (m x d)
    const float *base;  // source base weights (m)
    const double *pot;  // source potential (m)
    int64_t m;
    int d, r;           // dimension, cost exponent (C = |x - y|^r)
    double inv_eps;
};

// Per-block maxima of a float array (UPD_BLOCKS-sized launch); also clears *counter (nullable),
// the number of rows the following re-evaluation kernel has taken.
__global__ void __launch_bounds__(RT) k_max_f32(const float *__restrict__ t, int64_t n,
                                                double *__restrict__ parts,
                                                int *__restrict__ counter) {
    __shared__ double red[RT / 64];
    if (counter && blockIdx.x == 0 && threadIdx.x == 0) *counter = 0;
    double mx = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        mx = fmax(mx, (double)t[i]);
    mx = block_max(mx, red);
    if (threadIdx.x == 0) parts[blockIdx.x] = mx;
}

// The whole wave evaluates target `row`: returns (on every lane) L = log sum_j e^{e_j} with
// e_j = log base_j + (pot_j - shift) inv_eps - C_ij inv_eps, and, when G is non-null, the softmax
// mean of grad_x C_ij (d <= 3) in G.
// Exponents in log2 units, e_j = log2 base_j + ((pot_j - shift) / eps - C_ij / eps) log2 e (the
// potential difference in FP64, the rest in FP32), taken in chunks of FCH sources per lane: the
// running maximum is raised at most once per chunk, then each term costs one exp2.
constexpr int FCH = 8;
__device__ void floor_row_lse(const FloorSrc &src, int64_t row, double shift, int lane, double &L,
                              double *G) {
    float xi[3] = {0.0f, 0.0f, 0.0f};
    for (int k = 0; k < src.d; ++k) xi[k] = src.xt[row * src.d + k];
    const float cs = (float)(src.inv_eps * 1.4426950408889634);
    const double ps = src.inv_eps * 1.4426950408889634;
    float M = -FLT_MAX;
    double S = 0.0, g[3] = {0.0, 0.0, 0.0};
    for (int64_t j0 = lane; j0 < src.m; j0 += 64 * FCH) {
        float e[FCH], gw[FCH][3];
        float mx = -FLT_MAX;
#pragma unroll
        for (int c = 0; c < FCH; ++c) {
            const int64_t j = j0 + 64 * c;
            e[c] = -INFINITY;
            gw[c][0] = gw[c][1] = gw[c][2] = 0.0f;
            if (j < src.m) {
                float df[3] = {0.0f, 0.0f, 0.0f}, r2 = 0.0f;
                for (int k = 0; k < src.d; ++k) {
                    df[k] = xi[k] - src.ys[j * src.d + k];
                    r2 = fmaf(df[k], df[k], r2);
                }
                const float rr = __builtin_sqrtf(r2);
                const float b = src.base[j];
                if (b > 0.0f)
                    e[c] = __builtin_amdgcn_logf(b) + (float)((src.pot[j] - shift) * ps) -
                           (src.r == 2 ? r2 : rr) * cs;
                if (G) {
                    // grad_x C: r = 2: 2 (x - y); r = 1: (x - y) / |x - y| (0 at coincident points)
                    const float gs = src.r == 2 ? 2.0f : (rr > 0.0f ? 1.0f / rr : 0.0f);
                    for (int k = 0; k < src.d; ++k) gw[c][k] = gs * df[k];
                }
                mx = fmaxf(mx, e[c]);
            }
        }
        if (mx > M) {
            const double sc = exp2((double)M - (double)mx);
            S *= sc;
            for (int k = 0; k < 3; ++k) g[k] *= sc;
            M = mx;
        }
        float ps_ = 0.0f, pg[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int c = 0; c < FCH; ++c) {
            const float wgt = exp2f(e[c] - M);
            ps_ += wgt;
            if (G)
                for (int k = 0; k < 3; ++k) pg[k] = fmaf(wgt, gw[c][k], pg[k]);
        }
        S += ps_;
        if (G)
            for (int k = 0; k < 3; ++k) g[k] += pg[k];
    }
    float Mw = M;
    for (int o = 32; o > 0; o >>= 1) Mw = fmaxf(Mw, __shfl_xor(Mw, o, 64));
    const double sc = (M == -FLT_MAX) ? 0.0 : exp2((double)M - (double)Mw);
    S *= sc;
    for (int k = 0; k < 3; ++k) g[k] *= sc;
    for (int o = 32; o > 0; o >>= 1) {
        S += __shfl_xor(S, o, 64);
        for (int k = 0; k < 3; ++k) g[k] += __shfl_xor(g[k], o, 64);
    }
    L = (S > 0.0) ? ((double)Mw + log2(S)) * 0.6931471805599453 : -INFINITY;
    if (G)
        for (int k = 0; k < 3; ++k) G[k] = (S > 0.0) ? g[k] / S : 0.0;
}

// The update of k_update, with the rows below FLOOR_REL of the largest sum (and non-positive
// sums) re-evaluated directly.  Rows go in wave-aligned runs of 64 (one per lane); the flagged
// rows of a run are then taken one after the other by the whole wave.
// At most `cap` rows per launch are re-evaluated (the first to claim a slot of *taken); the
// others keep the fast sum (a bounded cost per half-step: cap x m pairs).  The threshold is
// FLOOR_REL of the largest sum of the previous half-step on the same side (tmax_prev; the first
// half-step's own, from k_max_f32); this launch writes its own per-block maxima of t to tmax_out
// and clears the slot counter of the next launch.
template <bool DELTA>
__global__ void __launch_bounds__(RT) k_update_floor(const float *__restrict__ t, int64_t n,
                                                     const double *__restrict__ shift_parts,
                                                     int nshift,
                                                     const double *__restrict__ tmax_prev,
                                                     int ntmax, double *__restrict__ tmax_out,
                                                     double kappa, double eps, FloorSrc src,
                                                     int *__restrict__ taken,
                                                     int *__restrict__ taken_next, int cap,
                                                     double *__restrict__ pot,
                                                     double *__restrict__ out_parts,
                                                     int *__restrict__ nbad,
                                                     double *__restrict__ delta_parts) {
    __shared__ double red[RT / 64];
    if (blockIdx.x == 0 && threadIdx.x == 0) *taken_next = 0;
    double sh = -INFINITY, tm = 0.0;
    for (int b = threadIdx.x; b < nshift; b += RT) sh = fmax(sh, shift_parts[b]);
    for (int b = threadIdx.x; b < ntmax; b += RT) tm = fmax(tm, tmax_prev[b]);
    sh = block_max(sh, red);
    if (sh == -INFINITY) sh = 0.0;
    tm = block_max(tm, red);
    const float thr = (float)(tm * (double)FLOOR_REL);
    double tcur = 0.0;
    const int lane = threadIdx.x & 63;
    double mx = -INFINITY, dmx = 0.0;
    int bad = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i0 = blockIdx.x * (int64_t)blockDim.x + (threadIdx.x & ~63); i0 < n;
         i0 += stride) {
        const int64_t i = i0 + lane;
        const bool ok = i < n;
        const float v = ok ? t[i] : 1.0f;
        if (ok) tcur = fmax(tcur, (double)v);
        bool flag = ok && !(v >= thr && v > 0.0f);
        // claim re-evaluation slots for this run's flagged rows (one atomic per run)
        uint64_t mask = __ballot(flag);
        if (mask) {
            int base = 0;
            if (lane == 0) base = atomicAdd(taken, __popcll(mask));
            base = __shfl(base, 0, 64);
            const int rank = __popcll(mask & ((1ull << lane) - 1ull));
            flag = flag && base + rank < cap;
            mask = __ballot(flag);
        }
        double f = 0.0;
        if (ok && !flag) {
            float vv = v;
            if (!(vv > 0.0f)) {
                bad++;
                vv = FLT_MIN;
            }
            f = -kappa * (sh + eps * sum_log(vv));
        }
        while (mask) {
            const int k = __ffsll((unsigned long long)mask) - 1;
            mask &= mask - 1;
            double L;
            floor_row_lse(src, i0 + k, sh, lane, L, nullptr);
            if (lane == k) {
                if (!(L > -INFINITY)) {
                    bad++;
                    L = log((double)FLT_MIN);
                }
                f = -kappa * (sh + eps * L);
            }
        }
        if (ok) {
            if (DELTA) dmx = fmax(dmx, fabs(f - pot[i]));
            pot[i] = f;
            mx = fmax(mx, f);
        }
    }
    if (bad) atomicAdd(nbad, bad);
    mx = block_max(mx, red);
    if (threadIdx.x == 0) out_parts[blockIdx.x] = mx;
    tcur = block_max(tcur, red);
    if (threadIdx.x == 0) tmax_out[blockIdx.x] = tcur;
    if (DELTA) {
        dmx = block_max(dmx, red);
        if (threadIdx.x == 0) delta_parts[blockIdx.x] = dmx;
    }
}

// Per-block maxima of a double array (warm starts, gradients); combined by the consumer.
__global__ void __launch_bounds__(RT) k_max_parts(const double *__restrict__ v, int64_t n,
                                                  double *__restrict__ parts) {
    __shared__ double sm[RT];
    double mx = -INFINITY;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        mx = fmax(mx, v[i]);
    sm[threadIdx.x] = mx;
    __syncthreads();
    for (int s = RT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) parts[blockIdx.x] = sm[0];
}

// Weighted moments about the reference point ref (the first point of the set), per block:
// parts[b][k] = sum w (p_k - ref_k) (k < d), parts[b][d] = sum w, parts[b][d+1] = sum w |p - ref|^2.
__global__ void __launch_bounds__(RT) k_moments(const float *__restrict__ p, const float *__restrict__ w,
                                                int64_t n, int d, const float *__restrict__ ref,
                                                double *__restrict__ parts) {
    __shared__ double sm[RT];
    for (int k = 0; k < d + 2; ++k) {
        double acc = 0.0;
        for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
             i += (int64_t)gridDim.x * blockDim.x) {
            const double wi = w[i];
            if (k < d) {
                acc += wi * ((double)p[i * d + k] - (double)ref[k]);
            } else if (k == d) {
                acc += wi;
            } else {
                double r2 = 0.0;
                for (int c = 0; c < d; ++c) {
                    const double t = (double)p[i * d + c] - (double)ref[c];
                    r2 += t * t;
                }
                acc += wi * r2;
            }
        }
        sm[threadIdx.x] = acc;
        __syncthreads();
        for (int s = RT / 2; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) parts[(int64_t)blockIdx.x * (d + 2) + k] = sm[0];
        __syncthreads();
    }
}

// out[k] = sum over blocks of parts[b][k] (fixed order), one thread per component
// One block per component: thread t sums blocks t, t + RT, ... in order, then a fixed tree.
__global__ void __launch_bounds__(RT) k_moments_final(const double *__restrict__ parts,
                                                      int nblocks, int ncomp,
                                                      double *__restrict__ out) {
    __shared__ double sm[RT];
    const int k = blockIdx.x;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += RT) acc += parts[(int64_t)b * ncomp + k];
    sm[threadIdx.x] = acc;
    __syncthreads();
    for (int o = RT / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = sm[0];
}

// out = max of nparts maxima (0 if all are -inf), one block
__global__ void __launch_bounds__(RT) k_max_final(const double *__restrict__ parts, int nparts,
                                                  double *__restrict__ out) {
    __shared__ double sm[RT];
    double mx = -INFINITY;
    for (int b = threadIdx.x; b < nparts; b += RT) mx = fmax(mx, parts[b]);
    sm[threadIdx.x] = mx;
    __syncthreads();
    for (int s = RT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = (sm[0] == -INFINITY) ? 0.0 : sm[0];
}

// Compensated FP64 sums of per-element terms.  MODE 0 (objective pieces for one side):
//   out[0] = sum base (1 - e^{-pot/rho}),  out[1] = sum base e^{-pot/rho},  out[2] = sum base
// MODE 1 (dot products):  out[0] = sum u v.   MODE 2:  out[0] = sum u.
// Each block writes (sum, compensation) pairs; k_csum_final folds them with Neumaier sums.
template <int MODE>
__global__ void __launch_bounds__(RT) k_csum(const float *__restrict__ u, const double *__restrict__ pot,
                                             const float *__restrict__ v, int64_t n, double rho,
                                             double *__restrict__ partial) {
    __shared__ double ss[3][RT], sc[3][RT];
    double s[3] = {0, 0, 0}, c[3] = {0, 0, 0};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (MODE == 0) {
            const double bi = u[i], e = exp(-pot[i] / rho);
            nadd(s[0], c[0], -bi * expm1(-pot[i] / rho));
            nadd(s[1], c[1], bi * e);
            nadd(s[2], c[2], bi);
        } else if (MODE == 2) {
            nadd(s[0], c[0], (double)u[i]);
        } else {
            nadd(s[0], c[0], (double)u[i] * (double)v[i]);
        }
    }
    for (int k = 0; k < 3; ++k) { ss[k][threadIdx.x] = s[k]; sc[k][threadIdx.x] = c[k]; }
    __syncthreads();
    // tree: pairwise Neumaier combination of (sum, compensation) pairs
    for (int o = RT / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int k = 0; k < 3; ++k) {
                double S = ss[k][threadIdx.x], C = sc[k][threadIdx.x] + sc[k][threadIdx.x + o];
                nadd(S, C, ss[k][threadIdx.x + o]);
                ss[k][threadIdx.x] = S;
                sc[k][threadIdx.x] = C;
            }
        __syncthreads();
    }
    if (threadIdx.x < 3) {
        partial[(blockIdx.x * 3 + threadIdx.x) * 2] = ss[threadIdx.x][0];
        partial[(blockIdx.x * 3 + threadIdx.x) * 2 + 1] = sc[threadIdx.x][0];
    }
}

// Combination of the per-block (sum, compensation) pairs: thread t takes blocks t, t + RT, ...
// in order, then the same pairwise tree as above (a fixed order: reproducible).
__global__ void __launch_bounds__(RT) k_csum_final(const double *__restrict__ partial, int nblocks,
                                                   double *__restrict__ out) {
    __shared__ double ss[3][RT], sc[3][RT];
    for (int k = 0; k < 3; ++k) {
        double S = 0, C = 0;
        for (int b = threadIdx.x; b < nblocks; b += RT) {
            nadd(S, C, partial[(b * 3 + k) * 2]);
            C += partial[(b * 3 + k) * 2 + 1];
        }
        ss[k][threadIdx.x] = S;
        sc[k][threadIdx.x] = C;
    }
    __syncthreads();
    for (int o = RT / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int k = 0; k < 3; ++k) {
                double S = ss[k][threadIdx.x], C = sc[k][threadIdx.x] + sc[k][threadIdx.x + o];
                nadd(S, C, ss[k][threadIdx.x + o]);
                ss[k][threadIdx.x] = S;
                sc[k][threadIdx.x] = C;
            }
        __syncthreads();
    }
    if (threadIdx.x < 3) out[threadIdx.x] = ss[threadIdx.x][0] + sc[threadIdx.x][0];
}

// Direct gradient sum: g_i = sum_j grad K(x_i - y_j) w_j (and t_i), any d <= 128.
template <int KIND>
__global__ void __launch_bounds__(256) k_direct_grad(const float *__restrict__ x, int64_t n,
                                                     const float *__restrict__ y, int64_t m,
                                                     int d, const float *__restrict__ w,
                                                     float lam_inv, float *__restrict__ t,
                                                     float *__restrict__ g) {
    constexpr int GT = 32;
    __shared__ float sy[GT * 128];
    __shared__ float sw[GT];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const float *xi = x + (i < n ? i : 0) * d;
    double acc = 0.0;
    double gacc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int dd = d < 8 ? d : 8;
    for (int64_t j0 = 0; j0 < m; j0 += GT) {
        const int cnt = (int)((m - j0) < GT ? (m - j0) : GT);
        __syncthreads();
        for (int q = threadIdx.x; q < GT * d; q += blockDim.x) {
            int jj = q / d;
            sy[q] = (jj < cnt) ? y[(j0 + jj) * d + (q - jj * d)] : 0.0f;
        }
        for (int q = threadIdx.x; q < GT; q += blockDim.x) sw[q] = (q < cnt) ? w[j0 + q] : 0.0f;
        __syncthreads();
        float part = 0.0f, gp[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int q = 0; q < cnt; ++q) {
            float r2 = 0.0f;
            for (int k = 0; k < d; ++k) {
                float dv = xi[k] - sy[q * d + k];
                r2 = fmaf(dv, dv, r2);
            }
            const float r = sqrtf(r2);
            float kv, coef;  // K and (dK/dr)/r
            if (KIND == FS_GAUSS) {
                kv = __expf(-r2 * lam_inv);
                coef = -2.0f * lam_inv * kv;
            } else if (KIND == FS_LAPLACE) {
                kv = __expf(-r * lam_inv);
                coef = (r > 0.0f) ? -lam_inv * kv / r : 0.0f;
            } else if (KIND == FS_IMQ) {
                kv = rsqrtf(r2 + lam_inv);  // lam_inv carries c^2 for this kernel
                coef = -kv * kv * kv;
            } else {
                kv = -r;
                coef = (r > 0.0f) ? -1.0f / r : 0.0f;
            }
            part = fmaf(kv, sw[q], part);
            for (int k = 0; k < dd; ++k) gp[k] = fmaf(coef * sw[q], xi[k] - sy[q * d + k], gp[k]);
        }
        acc += (double)part;
        for (int k = 0; k < dd; ++k) gacc[k] += (double)gp[k];
    }
    if (i < n) {
        if (t) t[i] = (float)acc;
        for (int k = 0; k < dd; ++k) g[i * d + k] = (float)gacc[k];
    }
}

// dx_i = coef * a_i * exp((f_i + gmax)/eps) * grad_i  (grad: d per row) and
// da_i = rho (1 - e^{-f_i/rho}) - eps (exp((f_i + gmax)/eps) t_i - Mb)
__global__ void k_uot_grad_rows(const float *__restrict__ a, const double *__restrict__ f,
                                const float *__restrict__ t, const float *__restrict__ grad,
                                int d, int64_t n, const double *__restrict__ gmax, double eps,
                                double rho, const double *__restrict__ Mb, double scale,
                                float *__restrict__ dx, float *__restrict__ da) {
    const double gm = *gmax, mb = *Mb;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double e = exp((f[i] + gm) / eps);
        if (dx)
            for (int k = 0; k < d; ++k)
                dx[i * d + k] = (float)(-scale * eps * (double)a[i] * e * (double)grad[i * d + k]);
        if (da) da[i] = (float)(scale * (-rho * expm1(-f[i] / rho) - eps * (e * (double)t[i] - mb)));
    }
}

// Decade histogram of the rows below FLOOR_REL of the largest sum: bin k < 15 counts
// t_i / max t in [1e-(k+3), 1e-(k+2)), bin 15 everything smaller (or not positive).
constexpr int FLOOR_BINS = 16;
__global__ void __launch_bounds__(RT) k_floor_hist(const float *__restrict__ t, int64_t n,
                                                   const double *__restrict__ tmax_parts,
                                                   int ntmax, int *__restrict__ hist) {
    __shared__ double red[RT / 64];
    __shared__ int h[FLOOR_BINS];
    if (threadIdx.x < FLOOR_BINS) h[threadIdx.x] = 0;
    double tm = 0.0;
    for (int b = threadIdx.x; b < ntmax; b += RT) tm = fmax(tm, tmax_parts[b]);
    tm = block_max(tm, red);  // (its barrier also orders the clearing of h)
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double r = (double)t[i] / tm;
        if (!(r >= (double)FLOOR_REL)) {
            int bin = FLOOR_BINS - 1;
            if (r > 0.0) bin = min(FLOOR_BINS - 1, (int)floor(-log10(r)) - 2);
            atomicAdd(&h[max(bin, 0)], 1);
        }
    }
    __syncthreads();
    if (threadIdx.x < FLOOR_BINS && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

// Rows of k_uot_grad_rows whose sum t_i is below FLOOR_REL of the largest, recomputed directly:
//   dx_i = scale a_i e^{(f_i + gmax)/eps + L_i} Gbar_i,  Gbar_i the softmax mean of grad_x C_ij,
//   da_i = scale (rho (1 - e^{-f_i/rho}) - eps (e^{(f_i + gmax)/eps + L_i} - Mb)).
// The rows with t_i < rel x (largest t) (rel <= FLOOR_REL, chosen by the host from the histogram
// below so that the work stays within a budget), listed for k_uot_grad_floor.
// The list holds at most `cap` rows (the count may run past it; readers clamp).
__global__ void __launch_bounds__(RT) k_floor_list(const float *__restrict__ t, int64_t n,
                                                   const double *__restrict__ tmax_parts,
                                                   int ntmax, double rel, int *__restrict__ count,
                                                   int cap, int *__restrict__ list) {
    __shared__ double red[RT / 64];
    double tm = 0.0;
    for (int b = threadIdx.x; b < ntmax; b += RT) tm = fmax(tm, tmax_parts[b]);
    tm = block_max(tm, red);
    const float thr = (float)(tm * rel);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float v = t[i];
        if (!(v >= thr && v > 0.0f)) {
            const int q = atomicAdd(count, 1);
            if (q < cap) list[q] = (int)i;
        }
    }
}

// One wave per listed row (min(*count, cap) rows).
__global__ void __launch_bounds__(64) k_uot_grad_floor(const float *__restrict__ a,
                                                       const double *__restrict__ f,
                                                       const int *__restrict__ list,
                                                       const int *__restrict__ count, int cap,
                                                       const double *__restrict__ gmax,
                                                       double eps, double rho,
                                                       const double *__restrict__ Mb,
                                                       double scale, FloorSrc src,
                                                       float *__restrict__ dx,
                                                       float *__restrict__ da) {
    const double gm = *gmax, mb = *Mb;
    const int lane = threadIdx.x;
    const int nlist = min(*count, cap);
    for (int q = blockIdx.x; q < nlist; q += gridDim.x) {
        const int64_t row = list[q];
        double L, G[3];
        floor_row_lse(src, row, gm, lane, L, G);
        if (lane == 0) {
            const double e = (L > -INFINITY) ? exp((f[row] + gm) * (1.0 / eps) + L) : 0.0;
            if (dx)
                for (int c = 0; c < src.d; ++c)
                    dx[row * src.d + c] = (float)(scale * (double)a[row] * e * G[c]);
            if (da) da[row] = (float)(scale * (-rho * expm1(-f[row] / rho) - eps * (e - mb)));
        }
    }
}

// out = s1 * u + s2 * v + s3 * c  (float outputs from float inputs; v may be NULL)
__global__ void k_combine(const float *__restrict__ u, const float *__restrict__ v, int64_t n,
                          double s1, double s2, double cst, float *__restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double r = s1 * (double)u[i] + cst;
        if (v) r += s2 * (double)v[i];
        out[i] = (float)r;
    }
}

// MMD gradient rows on the union plan (operator order): with w_k the union weights,
//   dz_k = 2 scale w_k grad s(z_k),   dw_k = 2 scale s(z_k) (sign folded for the b side).
__global__ void k_mmd_grad_rows(const float *__restrict__ ws, const float *__restrict__ ts,
                                const float *__restrict__ gs, const int *__restrict__ perm,
                                int64_t ntot, int64_t n, int d, double scale,
                                float *__restrict__ dx, float *__restrict__ da,
                                float *__restrict__ dy, float *__restrict__ db) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < ntot;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t o = perm ? perm[k] : k;
        const double w = ws[k];
        if (o < n) {
            if (dx)
                for (int c = 0; c < d; ++c) dx[o * d + c] = (float)(2.0 * scale * w * gs[k * d + c]);
            if (da) da[o] = (float)(2.0 * scale * ts[k]);
        } else {
            const int64_t j = o - n;
            if (dy)
                for (int c = 0; c < d; ++c) dy[j * d + c] = (float)(2.0 * scale * w * gs[k * d + c]);
            if (db) db[j] = (float)(-2.0 * scale * ts[k]);
        }
    }
}

__global__ void k_concat_weights(const float *__restrict__ a, int64_t n,
                                 const float *__restrict__ b, int64_t m, float sa, float sb,
                                 float *__restrict__ w) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n + m;
         i += (int64_t)gridDim.x * blockDim.x)
        w[i] = (i < n) ? sa * a[i] : sb * b[i - n];
}

}  // namespace

// =====================================================================================
//                                     operators
// =====================================================================================
std::unique_ptr<Op> make_op(const float *x, int64_t n, const float *y, int64_t m, int d,
                            const fs_params &p, hipStream_t s) {
    auto op = std::make_unique<Op>();
    op->d = d;
    op->kind = p.kernel;
    op->lambda = p.lambda;
    op->flags = p.flags;
    op->n = n;
    op->m = m;
    op->x = x;
    op->y = y;
    op->same = (x == y && n == m);
    FS_REQUIRE(p.kernel == FS_GAUSS || p.kernel == FS_LAPLACE || p.kernel == FS_ENERGY ||
                   p.kernel == FS_IMQ, FS_EINVAL,
               "unknown kernel %d", p.kernel);
    FS_REQUIRE(p.kernel == FS_ENERGY || (p.lambda > 0 && std::isfinite(p.lambda)), FS_EINVAL,
               "lambda must be positive and finite");
    if (p.grid > 0) {
        op->fast = true;
        op->plan = std::make_unique<Plan>();
        plan_build(*op->plan, x, n, y, m, d, p, s);
    } else {
        FS_REQUIRE(d >= 1 && d <= 128, FS_EINVAL, "direct summation supports d in 1..128 (got %d)", d);
        op->mfma = mfma_supported(p.kernel, d) && !(p.flags & FS_FLAG_FORCE_VALU);
        // the Gram path's error grows with the exponent scale: use it only where it meets 1e-5
        if (op->mfma)
            op->mfma = gram_frame(x, n, y, m, op->same, d, p.lambda, op->gcenter, s) <= GRAM_Q_MAX;
        if (op->mfma) {
            gram_prepare(x, n, d, p.lambda, op->gcenter.p, op->gx, s);
            if (!op->same) gram_prepare(y, m, d, p.lambda, op->gcenter.p, op->gy, s);
        }
    }
    return op;
}

void Op::to_op(int side, const float *v, float *vo, hipStream_t s) const {
    const int64_t c = count(side);
    if (fast) gather_to_sorted(side == 0 ? plan->X : (plan->same ? plan->X : plan->Y), v, vo, s);
    else if (c > 0 && v != vo) FS_HIP(hipMemcpyAsync(vo, v, c * sizeof(float), hipMemcpyDeviceToDevice, s));
}
void Op::to_op64(int side, const double *v, double *vo, hipStream_t s) const {
    const int64_t c = count(side);
    if (fast) gather_to_sorted64(side == 0 ? plan->X : (plan->same ? plan->X : plan->Y), v, vo, s);
    else if (c > 0 && v != vo) FS_HIP(hipMemcpyAsync(vo, v, c * sizeof(double), hipMemcpyDeviceToDevice, s));
}
void Op::from_op(int side, const float *vo, float *v, hipStream_t s) const {
    const int64_t c = count(side);
    if (fast) scatter_from_sorted(side == 0 ? plan->X : (plan->same ? plan->X : plan->Y), vo, v, s);
    else if (c > 0 && v != vo) FS_HIP(hipMemcpyAsync(v, vo, c * sizeof(float), hipMemcpyDeviceToDevice, s));
}
void Op::from_op64(int side, const double *vo, double *v, hipStream_t s) const {
    const int64_t c = count(side);
    if (fast) scatter_from_sorted64(side == 0 ? plan->X : (plan->same ? plan->X : plan->Y), vo, v, s);
    else if (c > 0 && v != vo) FS_HIP(hipMemcpyAsync(v, vo, c * sizeof(double), hipMemcpyDeviceToDevice, s));
}
void Op::rows_from_op(int side, const float *vo, float *v, hipStream_t s) const {
    const int64_t c = count(side);
    if (fast) scatter_rows_from_sorted(side == 0 ? plan->X : (plan->same ? plan->X : plan->Y), vo, d, v, s);
    else if (c > 0 && v != vo) FS_HIP(hipMemcpyAsync(v, vo, c * d * sizeof(float), hipMemcpyDeviceToDevice, s));
}
const float *Op::coords(int side) const {
    if (fast) return (side == 0 ? plan->X : (plan->same ? plan->X : plan->Y)).xs.p;
    return side == 0 ? x : y;
}

namespace {
void launch_weights(const float *base, const double *pot, const double *parts, int nparts,
                    double eps, int64_t n, float *w, hipStream_t s);
void launch_log_weights(const float *base, const double *pot, const double *parts, int nparts,
                        double eps, int64_t n, float *u, hipStream_t s);
}  // namespace

bool Op::log_direct() const {
    return !fast && !mfma && (kind == FS_GAUSS || kind == FS_LAPLACE);
}

void Op::apply_pot_log(const float *base, const double *pot, const double *parts, int nparts,
                       double eps, float *u, double *logt, int transpose, hipStream_t s) {
    const int64_t nt = transpose ? m : n, ns = transpose ? n : m;
    if (nt == 0) return;
    if (ns == 0) {
        fill_f64(logt, nt, -INFINITY, s);
        return;
    }
    ProfScope ps("direct", s);
    launch_log_weights(base, pot, parts, nparts, eps, ns, u, s);
    direct_lse(kind, lambda, transpose ? y : x, nt, transpose ? x : y, ns, d, u, logt, s);
}

bool Op::fuses_weights(int transpose) const {
    return fast && count(transpose ? 0 : 1) > 0 && count(transpose ? 1 : 0) > 0 &&
           plan_fuses_weights(*plan, transpose);
}

void Op::apply_pot(const float *base, const double *pot, const double *parts, int nparts,
                   double eps, float *w, float *t, int transpose, hipStream_t s) {
    if (fuses_weights(transpose)) {
        PotWeights pw;
        pw.base = base;
        pw.pot = pot;
        pw.parts = parts;
        pw.nparts = nparts;
        pw.inv_eps = 1.0 / eps;
        plan_apply_sorted_pot(*plan, pw, t, transpose, s);
        return;
    }
    launch_weights(base, pot, parts, nparts, eps, count(transpose ? 0 : 1), w, s);
    apply(w, t, nullptr, transpose, s);
}

bool Op::fuses_update(int transpose) const {
    return fuses_weights(transpose) && plan_fuses_update(*plan, transpose);
}

int Op::update_parts(int transpose) const { return plan_update_parts(*plan, transpose); }

void Op::apply_pot_update(const float *base, const double *pot, const double *parts, int nparts,
                          double eps, const PotUpdate &pu, int transpose, hipStream_t s,
                          const float *bbase) {
    PotWeights pw;
    pw.base = base;
    pw.pot = pot;
    pw.parts = parts;
    pw.nparts = nparts;
    pw.inv_eps = 1.0 / eps;
    pw.bbase = (bbase && nparts == source_blocks(transpose)) ? bbase : nullptr;
    plan_apply_sorted_pot(*plan, pw, nullptr, transpose, s, &pu);
}

int Op::source_blocks(int transpose) const {
    return fast ? plan_source_blocks(*plan, transpose) : 0;
}

void Op::block_base_max(const float *base, int transpose, float *out, hipStream_t s) const {
    if (fast) plan_block_base_max(*plan, base, transpose, out, s);
}

void Op::apply(const float *w, float *t, float *grad, int transpose, hipStream_t s,
               double *ext_partial, size_t ext_count) {
    const int64_t nt = transpose ? m : n, ns = transpose ? n : m;
    if (nt == 0) return;
    if (ns == 0) {
        fill_f32(t, nt, 0.0f, s);
        if (grad) fill_f32(grad, nt * d, 0.0f, s);
        return;
    }
    if (fast) {
        plan_apply_sorted(*plan, w, t, grad, transpose, s);
        return;
    }
    const float *xt = transpose ? y : x, *ys = transpose ? x : y;
    if (grad) {
        FS_REQUIRE(d <= 8, FS_EUNSUPPORTED, "direct gradients support d <= 8 (got %d)", d);
        const float li = (kind == FS_ENERGY) ? 0.0f
                         : (kind == FS_IMQ) ? (float)(lambda * lambda) : (float)(1.0 / lambda);
        dim3 g(blocks_for(nt, 256, int64_t(1) << 30)), b(256);
        if (kind == FS_GAUSS)
            hipLaunchKernelGGL(k_direct_grad<FS_GAUSS>, g, b, 0, s, xt, nt, ys, ns, d, w, li, t, grad);
        else if (kind == FS_LAPLACE)
            hipLaunchKernelGGL(k_direct_grad<FS_LAPLACE>, g, b, 0, s, xt, nt, ys, ns, d, w, li, t, grad);
        else if (kind == FS_IMQ)
            hipLaunchKernelGGL(k_direct_grad<FS_IMQ>, g, b, 0, s, xt, nt, ys, ns, d, w, li, t, grad);
        else
            hipLaunchKernelGGL(k_direct_grad<FS_ENERGY>, g, b, 0, s, xt, nt, ys, ns, d, w, li, t, grad);
        FS_LAUNCHED();
        return;
    }
    ProfScope ps("direct", s);
    if (mfma) {
        const GramOperand &gt = transpose ? (same ? gx : gy) : gx;
        const GramOperand &gs = transpose ? gx : (same ? gx : gy);
        direct_mfma_gauss(gt, gs, w, t, nullptr, s, ext_partial, ext_count);
    } else {
        direct_valu(kind, lambda, xt, nt, ys, ns, d, w, t, nullptr, s);
    }
}

// =====================================================================================
//                                       Sinkhorn
// =====================================================================================
namespace {

// Device scratch of one solve: per-block maxima of both potentials, compensated-sum partials,
// scalar results and the count of non-positive kernel sums.
struct Scalars {
    DevBuf<double> v;       // scalar results: [0] gmax, [1] fmax, [2] Mb, [3] Ma, sums at [8..)
    DevBuf<double> fparts;  // per-block maxima of f
    DevBuf<double> gparts;  // per-block maxima of g
    DevBuf<double> dparts;  // per-block maxima of |change| of f (first half) and g (second half)
    DevBuf<double> partial;  // compensated-sum partials (RBLK x 3 x 2)
    DevBuf<int> nbad;
    int nf = 1, ng = 1;      // number of valid entries in fparts / gparts
    Scalars()
        : v(32), fparts(UPD_BLOCKS), gparts(UPD_BLOCKS), dparts(2 * UPD_BLOCKS),
          partial(RBLK * 6), nbad(1) {}
    void reset(FillBatch &fb) {
        fb.add_f64(v.p, 32, 0.0);
        fb.add_f64(fparts.p, UPD_BLOCKS, 0.0);
        fb.add_f64(gparts.p, UPD_BLOCKS, 0.0);
        fb.add_f64(dparts.p, 2 * UPD_BLOCKS, 0.0);
        fb.add_i32(nbad.p, 1, 0);
        nf = ng = 1;
    }
    void reset(hipStream_t s) {
        FillBatch fb(s);
        reset(fb);
        fb.launch();
    }
};

unsigned red_blocks(int64_t n) { return blocks_for(n, RT, RBLK); }
int upd_blocks(int64_t n) { return (int)blocks_for(n, RT, UPD_BLOCKS); }

// pot = update(t) with shift = max of (shift_parts, nshift); writes per-block maxima of pot
int launch_update(const float *t, int64_t n, const double *shift_parts, int nshift, double kappa,
                  double eps, double *pot, double *out_parts, int *nbad, double *delta_parts,
                  hipStream_t s) {
    ProfScope ps("update", s);
    const int nb = upd_blocks(n);
    if (delta_parts)
        hipLaunchKernelGGL(k_update<true>, dim3(nb), dim3(RT), 0, s, t, n, shift_parts, nshift,
                           kappa, eps, pot, out_parts, nbad, delta_parts);
    else
        hipLaunchKernelGGL(k_update<false>, dim3(nb), dim3(RT), 0, s, t, n, shift_parts, nshift,
                           kappa, eps, pot, out_parts, nbad, delta_parts);
    FS_LAUNCHED();
    return nb;
}

// The update with floor rows re-evaluated (fast path, unfused half-steps).  tmax_parts: scratch
// for UPD_BLOCKS per-block maxima of t.
// Work budget of the floor-row re-evaluation, in (row, source) pairs: per Sinkhorn half-step, and
// per gradient call.
constexpr double FLOOR_PAIRS_HALFSTEP = 1 << 30;
constexpr double FLOOR_PAIRS_GRAD = 1 << 30;

// Floor-row state of one side of a solve: per-block maxima of t and slot counters, both
// alternating between two halves from one half-step of that side to the next (zero at the start).
struct FloorState {
    DevBuf<double> tparts;  // 2 x UPD_BLOCKS
    DevBuf<int> taken;      // 2
    int phase = 0;
    bool first = true;  // the first half-step takes the largest sum of its own t
    void init(FillBatch &fb) {
        tparts.alloc(2 * UPD_BLOCKS);
        taken.alloc(2);
        fb.add_f64(tparts.p, 2 * UPD_BLOCKS, 0.0);
        fb.add_i32(taken.p, 2, 0);
    }
};

int launch_update_floor(const float *t, int64_t n, const double *shift_parts, int nshift,
                        double kappa, double eps, const FloorSrc &src, FloorState &fs,
                        double *pot, double *out_parts, int *nbad, double *delta_parts,
                        hipStream_t s) {
    ProfScope ps("update", s);
    const int nb = upd_blocks(n);
    const int cap = (int)std::min<double>(2e9, FLOOR_PAIRS_HALFSTEP / std::max<int64_t>(src.m, 1));
    const int ph = fs.phase;
    const double *prev = fs.tparts.p + (1 - ph) * UPD_BLOCKS;
    double *cur = fs.tparts.p + ph * UPD_BLOCKS;
    int *tk = fs.taken.p + ph, *tk_next = fs.taken.p + (1 - ph);
    if (fs.first) {
        hipLaunchKernelGGL(k_max_f32, dim3(nb), dim3(RT), 0, s, t, n,
                           fs.tparts.p + (1 - ph) * UPD_BLOCKS, nullptr);
        FS_LAUNCHED();
        fs.first = false;
    }
    if (delta_parts)
        hipLaunchKernelGGL(k_update_floor<true>, dim3(nb), dim3(RT), 0, s, t, n, shift_parts,
                           nshift, prev, UPD_BLOCKS, cur, kappa, eps, src, tk, tk_next, cap, pot,
                           out_parts, nbad, delta_parts);
    else
        hipLaunchKernelGGL(k_update_floor<false>, dim3(nb), dim3(RT), 0, s, t, n, shift_parts,
                           nshift, prev, UPD_BLOCKS, cur, kappa, eps, src, tk, tk_next, cap, pot,
                           out_parts, nbad, delta_parts);
    FS_LAUNCHED();
    fs.phase = 1 - ph;
    return nb;
}

int launch_update_log(const double *logt, int64_t n, const double *shift_parts, int nshift,
                      double kappa, double eps, double *pot, double *out_parts, int *nbad,
                      double *delta_parts, hipStream_t s) {
    ProfScope ps("update", s);
    const int nb = upd_blocks(n);
    if (delta_parts)
        hipLaunchKernelGGL(k_update_log<true>, dim3(nb), dim3(RT), 0, s, logt, n, shift_parts,
                           nshift, kappa, eps, pot, out_parts, nbad, delta_parts);
    else
        hipLaunchKernelGGL(k_update_log<false>, dim3(nb), dim3(RT), 0, s, logt, n, shift_parts,
                           nshift, kappa, eps, pot, out_parts, nbad, delta_parts);
    FS_LAUNCHED();
    return nb;
}

void launch_log_weights(const float *base, const double *pot, const double *parts, int nparts,
                        double eps, int64_t n, float *u, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_log_weights, dim3(blocks_for(n, 256, 8192)), dim3(256), 0, s, base, pot,
                       parts, nparts, 1.0 / eps, n, u);
    FS_LAUNCHED();
}

void launch_weights(const float *base, const double *pot, const double *parts, int nparts,
                    double eps, int64_t n, float *w, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_weights, dim3(blocks_for(n, 256, 8192)), dim3(256), 0, s, base, pot,
                       parts, nparts, 1.0 / eps, n, w);
    FS_LAUNCHED();
}

int launch_max_parts(const double *v, int64_t n, double *parts, hipStream_t s) {
    const int nb = upd_blocks(n);
    hipLaunchKernelGGL(k_max_parts, dim3(nb), dim3(RT), 0, s, v, n, parts);
    FS_LAUNCHED();
    return nb;
}

// compensated sums: MODE 0 objective pieces (3 values), 1 dot, 2 sum -> out[0..2]
void csum(int mode, const float *u, const double *pot, const float *v, int64_t n, double rho,
          Scalars &sc, double *out, hipStream_t s) {
    const unsigned nb = red_blocks(n);
    if (mode == 0)
        hipLaunchKernelGGL(k_csum<0>, dim3(nb), dim3(RT), 0, s, u, pot, v, n, rho, sc.partial.p);
    else if (mode == 1)
        hipLaunchKernelGGL(k_csum<1>, dim3(nb), dim3(RT), 0, s, u, pot, v, n, rho, sc.partial.p);
    else
        hipLaunchKernelGGL(k_csum<2>, dim3(nb), dim3(RT), 0, s, u, pot, v, n, rho, sc.partial.p);
    FS_LAUNCHED();
    hipLaunchKernelGGL(k_csum_final, dim3(1), dim3(RT), 0, s, sc.partial.p, (int)nb, out);
    FS_LAUNCHED();
}

// Envelope-gradient rows at the fast sum's error floor, recomputed directly (k_uot_grad_floor).
// The rows are taken from the smallest sums up, whole decades at a time, within
// FLOOR_PAIRS_GRAD pairs (the decade of the smallest sums is always taken).
void grad_floor_rows(const float *a, const double *f, const float *t, int64_t n,
                     const double *shift, double eps, double rho, const double *mass,
                     double scale, const FloorSrc &src, double *tparts, int *hist, float *dx,
                     float *da, hipStream_t s) {
    if (n == 0 || (!dx && !da)) return;
    const int nb = upd_blocks(n);
    hipLaunchKernelGGL(k_max_f32, dim3(nb), dim3(RT), 0, s, t, n, tparts, nullptr);
    FS_LAUNCHED();
    fill_i32(hist, FLOOR_BINS, 0, s);
    hipLaunchKernelGGL(k_floor_hist, dim3(nb), dim3(RT), 0, s, t, n, tparts, nb, hist);
    FS_LAUNCHED();
    int h[FLOOR_BINS];
    FS_HIP(hipMemcpyAsync(h, hist, sizeof(h), hipMemcpyDeviceToHost, s));
    FS_HIP(hipStreamSynchronize(s));
    const double cap_rows = FLOOR_PAIRS_GRAD / (double)std::max<int64_t>(src.m, 1);
    double rel = 0.0, taken = 0.0;
    for (int k = FLOOR_BINS - 1; k >= 0; --k) {
        if (h[k] == 0) continue;
        if (rel > 0.0 && taken + h[k] > cap_rows) break;
        taken += h[k];
        rel = (k == FLOOR_BINS - 1) ? std::pow(10.0, -(double)(FLOOR_BINS + 1))
                                    : std::pow(10.0, -(double)(k + 2));
    }
    if (taken == 0.0) return;
    // list the rows (counter in hist[0], rows after it), then one wave per row
    DevBuf<int> list((size_t)taken + 1);
    fill_i32(hist, 1, 0, s);
    hipLaunchKernelGGL(k_floor_list, dim3(nb), dim3(RT), 0, s, t, n, tparts, nb, rel, hist,
                       (int)taken, list.p);
    FS_LAUNCHED();
    hipLaunchKernelGGL(k_uot_grad_floor, dim3((unsigned)std::min<double>(taken, 65535.0)),
                       dim3(64), 0, s, a, f, list.p, hist, (int)taken, shift, eps, rho, mass,
                       scale, src, dx, da);
    FS_LAUNCHED();
    list.reset_after(s);
}

}  // namespace

void sinkhorn_solve(Op &op, const float *a_o, const float *b_o, double eps, double rho, int iters,
                    bool warm, double *f_o, double *g_o, double *objective_host, hipStream_t s,
                    double tol, int *sweeps_done) {
    const int64_t n = op.n, m = op.m;
    const double kappa = rho / (rho + eps);
    Scalars sc;
    FillBatch fb(s);  // the solve's initial fills, one launch
    sc.reset(fb);
    DevBuf<float> wX(n + 1), wY(m + 1), tX(n + 1), tY(m + 1);
    // log-domain direct sums (no underflow for rows far from every source) where they apply
    const bool logd = op.log_direct();
    DevBuf<double> lX(logd ? n + 1 : 0), lY(logd ? m + 1 : 0);
    // fast path, unfused half-steps: rows at the fast sum's error floor are re-evaluated directly
    FloorState floorX, floorY;  // targets X (beta half-steps), Y (gamma half-steps)
    if (op.fast) {
        floorX.init(fb);
        floorY.init(fb);
    }
    FloorSrc srcY{}, srcX{};
    if (op.fast) {
        const int r = op.kind == FS_GAUSS ? 2 : 1;
        srcY = FloorSrc{op.coords(0), op.coords(1), b_o, g_o, m, op.d, r, 1.0 / eps};
        srcX = FloorSrc{op.coords(1), op.coords(0), a_o, f_o, n, op.d, r, 1.0 / eps};
    }
    if (warm) {
        fb.launch();  // before the maxima are written into the cleared parts
        if (m > 0) sc.ng = launch_max_parts(g_o, m, sc.gparts.p, s);
        if (n > 0) sc.nf = launch_max_parts(f_o, n, sc.fparts.p, s);
    } else {
        fb.add_f64(g_o, m, 0.0);
        fb.add_f64(f_o, n, 0.0);
        fb.launch();
    }
    // fused half-steps: each side's largest |base| per source block, and whether that side's
    // potential maxima come from a fused update (then they are per source block)
    const bool fuseX = n > 0 && op.fuses_update(0) && op.update_parts(0) <= UPD_BLOCKS;
    const bool fuseY = m > 0 && op.fuses_update(1) && op.update_parts(1) <= UPD_BLOCKS;
    DevBuf<float> bbY(fuseX ? std::max(1, op.source_blocks(0)) : 0);
    DevBuf<float> bbX(fuseY ? std::max(1, op.source_blocks(1)) : 0);
    if (fuseX) op.block_base_max(b_o, 0, bbY.p, s);
    if (fuseY) op.block_base_max(a_o, 1, bbX.p, s);
    bool fblocks = false, gblocks = false;
    // with a tolerance, a sweep that changes no potential by more than tol * eps ends the solve
    const bool track = tol > 0.0;
    double *fd = track ? sc.dparts.p : nullptr, *gd = track ? sc.dparts.p + UPD_BLOCKS : nullptr;
    // On fused half-steps the change of each sweep is read back one sweep late: sweep it + 1 is
    // queued before the change of sweep it arrives, and the state after sweep it (both potentials,
    // their per-block maxima and the count of non-positive sums) is kept, so that a sweep found to
    // follow a converged one is undone.  The solve stops at the same sweep with the same state as
    // with a check after every sweep, without the device draining each time.
    const bool lag = track && fuseX && fuseY;
    DevBuf<double> snapF(lag ? n + 1 : 0), snapG(lag ? m + 1 : 0);
    DevBuf<double> snapP(lag ? 2 * UPD_BLOCKS : 0);
    DevBuf<int> snapB(lag ? 1 : 0);
    HostStage stage(s);
    double *hchange = lag ? static_cast<double *>(stage.pinned(2 * sizeof(double))) : nullptr;
    struct EventPair {
        hipEvent_t e[2] = {nullptr, nullptr};
        ~EventPair() {
            for (hipEvent_t x : e)
                if (x) (void)hipEventDestroy(x);
        }
    } ev;
    if (lag)
        for (hipEvent_t &x : ev.e) FS_HIP(hipEventCreateWithFlags(&x, hipEventDisableTiming));
    auto copy_state = [&](bool save) {
        CopyBatch cb(s);
        const size_t parts = UPD_BLOCKS * sizeof(double);
        if (save) {
            cb.add(snapF.p, f_o, n * sizeof(double));
            cb.add(snapG.p, g_o, m * sizeof(double));
            cb.add(snapP.p, sc.fparts.p, parts);
            cb.add(snapP.p + UPD_BLOCKS, sc.gparts.p, parts);
            cb.add(snapB.p, sc.nbad.p, sizeof(int));
        } else {
            cb.add(f_o, snapF.p, n * sizeof(double));
            cb.add(g_o, snapG.p, m * sizeof(double));
            cb.add(sc.fparts.p, snapP.p, parts);
            cb.add(sc.gparts.p, snapP.p + UPD_BLOCKS, parts);
            cb.add(sc.nbad.p, snapB.p, sizeof(int));
        }
        cb.launch();
    };
    int done = 0;
    for (int it = 0; it < iters; ++it) {
        // beta half-step (Delta odd): t_i = sum_j k_ij b_j e^{g_j/eps}, then the f update
        if (fuseX) {
            PotUpdate pu;
            pu.shift_parts = sc.gparts.p;
            pu.nshift = sc.ng;
            pu.kappa = kappa;
            pu.eps = eps;
            pu.pot = f_o;
            pu.out_parts = sc.fparts.p;
            pu.delta_parts = fd;
            pu.nbad = sc.nbad.p;
            op.apply_pot_update(b_o, g_o, sc.gparts.p, sc.ng, eps, pu, 0, s,
                                gblocks ? bbY.p : nullptr);
            sc.nf = op.update_parts(0);
            fblocks = true;
        } else if (logd) {
            op.apply_pot_log(b_o, g_o, sc.gparts.p, sc.ng, eps, wY.p, lX.p, 0, s);
            if (n > 0)
                sc.nf = launch_update_log(lX.p, n, sc.gparts.p, sc.ng, kappa, eps, f_o,
                                          sc.fparts.p, sc.nbad.p, fd, s);
        } else {
            op.apply_pot(b_o, g_o, sc.gparts.p, sc.ng, eps, wY.p, tX.p, 0, s);
            if (n > 0 && op.fast)
                sc.nf = launch_update_floor(tX.p, n, sc.gparts.p, sc.ng, kappa, eps, srcY,
                                            floorX, f_o, sc.fparts.p, sc.nbad.p, fd, s);
            else if (n > 0)
                sc.nf = launch_update(tX.p, n, sc.gparts.p, sc.ng, kappa, eps, f_o, sc.fparts.p,
                                      sc.nbad.p, fd, s);
        }
        // gamma half-step (Delta even): t~_j = sum_i k_ij a_i e^{f_i/eps}, then the g update
        if (fuseY) {
            PotUpdate pu;
            pu.shift_parts = sc.fparts.p;
            pu.nshift = sc.nf;
            pu.kappa = kappa;
            pu.eps = eps;
            pu.pot = g_o;
            pu.out_parts = sc.gparts.p;
            pu.delta_parts = gd;
            pu.nbad = sc.nbad.p;
            op.apply_pot_update(a_o, f_o, sc.fparts.p, sc.nf, eps, pu, 1, s,
                                fblocks ? bbX.p : nullptr);
            sc.ng = op.update_parts(1);
            gblocks = true;
        } else if (logd) {
            op.apply_pot_log(a_o, f_o, sc.fparts.p, sc.nf, eps, wX.p, lY.p, 1, s);
            if (m > 0)
                sc.ng = launch_update_log(lY.p, m, sc.fparts.p, sc.nf, kappa, eps, g_o,
                                          sc.gparts.p, sc.nbad.p, gd, s);
        } else {
            op.apply_pot(a_o, f_o, sc.fparts.p, sc.nf, eps, wX.p, tY.p, 1, s);
            if (m > 0 && op.fast)
                sc.ng = launch_update_floor(tY.p, m, sc.fparts.p, sc.nf, kappa, eps, srcX,
                                            floorY, g_o, sc.gparts.p, sc.nbad.p, gd, s);
            else if (m > 0)
                sc.ng = launch_update(tY.p, m, sc.fparts.p, sc.nf, kappa, eps, g_o, sc.gparts.p,
                                      sc.nbad.p, gd, s);
        }
        ++done;
        if (lag) {
            hipLaunchKernelGGL(k_max_final, dim3(1), dim3(RT), 0, s, sc.dparts.p, 2 * UPD_BLOCKS,
                               sc.v.p + 24);
            FS_LAUNCHED();
            FS_HIP(hipMemcpyAsync(hchange + it % 2, sc.v.p + 24, sizeof(double),
                                  hipMemcpyDeviceToHost, s));
            FS_HIP(hipEventRecord(ev.e[it % 2], s));
            if (it > 0) {
                // the previous sweep's change (it arrives while this sweep runs)
                FS_HIP(hipEventSynchronize(ev.e[(it - 1) % 2]));
                if (hchange[(it - 1) % 2] <= tol * eps) {
                    copy_state(false);  // back to the state after the converged sweep
                    --done;
                    break;
                }
            }
            if (it + 1 < iters) copy_state(true);
        } else if (track) {
            hipLaunchKernelGGL(k_max_final, dim3(1), dim3(RT), 0, s, sc.dparts.p, 2 * UPD_BLOCKS,
                               sc.v.p + 24);
            FS_LAUNCHED();
            double change = 0.0;
            FS_HIP(hipMemcpyAsync(&change, sc.v.p + 24, sizeof(double), hipMemcpyDeviceToHost, s));
            FS_HIP(hipStreamSynchronize(s));
            if (change <= tol * eps) break;
        }
    }
    if (sweeps_done) *sweeps_done = done;
    int nbad = 0;
    if (objective_host) {
        // Dual value of Theorem "dualization" at (f, g).  After a gamma half-step the double sum
        // sum_ij a_i b_j e^{(f_i + g_j - C_ij)/eps} = sum_j b_j e^{g_j/eps} t~_j equals
        // sum_j b_j e^{-g_j/rho} (the update makes e^{g_j/eps} t~_j = e^{-g_j/rho}), so no extra
        // kernel sum is needed:  D = rho sum a (1 - e^{-f/rho}) + rho sum b (1 - e^{-g/rho})
        //                            - eps (sum b e^{-g/rho} - Ma Mb).
        // With no sweep done (f = g = 0 or the warm start) the double sum is formed explicitly.
        double *sx = sc.v.p + 8, *sy = sc.v.p + 12, *sd = sc.v.p + 16;
        double *gmax = sc.v.p + 0, *fmax = sc.v.p + 1;
        csum(0, a_o, f_o, nullptr, n, rho, sc, sx, s);
        csum(0, b_o, g_o, nullptr, m, rho, sc, sy, s);
        if (iters == 0) {
            // sum_i a_i e^{f_i/eps} sum_j k_ij b_j e^{g_j/eps}, shifted by fmax and gmax
            hipLaunchKernelGGL(k_max_final, dim3(1), dim3(RT), 0, s, sc.gparts.p, sc.ng, gmax);
            hipLaunchKernelGGL(k_max_final, dim3(1), dim3(RT), 0, s, sc.fparts.p, sc.nf, fmax);
            FS_LAUNCHED();
            launch_weights(b_o, g_o, sc.gparts.p, sc.ng, eps, m, wY.p, s);
            op.apply(wY.p, tX.p, nullptr, 0, s);
            launch_weights(a_o, f_o, sc.fparts.p, sc.nf, eps, n, wX.p, s);
            csum(1, wX.p, nullptr, tX.p, n, rho, sc, sd, s);
        }
        double h[20];
        FS_HIP(hipMemcpyAsync(h, sc.v.p, sizeof(h), hipMemcpyDeviceToHost, s));
        FS_HIP(hipMemcpyAsync(&nbad, sc.nbad.p, sizeof(int), hipMemcpyDeviceToHost, s));
        FS_HIP(hipStreamSynchronize(s));
        const double Ma = h[10], Mb = h[14];
        double dsum = h[13];
        if (iters == 0) dsum = h[16] * std::exp((h[1] + h[0]) / eps);
        *objective_host = rho * h[8] + rho * h[12] - eps * (dsum - Ma * Mb);
    } else {
        FS_HIP(hipMemcpyAsync(&nbad, sc.nbad.p, sizeof(int), hipMemcpyDeviceToHost, s));
        FS_HIP(hipStreamSynchronize(s));
    }
    FS_REQUIRE(nbad == 0, FS_ENUMERIC,
               "%d kernel sums were not positive (points too far apart for lambda, or the fast "
               "summation is not accurate enough for them)", nbad);
}

// =====================================================================================
//                           reductions, gradients and MMD drivers
// =====================================================================================
double device_sum(const float *u, int64_t n, hipStream_t s) {
    if (n <= 0) return 0.0;
    Scalars sc;
    sc.reset(s);
    csum(2, u, nullptr, nullptr, n, 0.0, sc, sc.v.p, s);
    double h = 0.0;
    FS_HIP(hipMemcpyAsync(&h, sc.v.p, sizeof(double), hipMemcpyDeviceToHost, s));
    FS_HIP(hipStreamSynchronize(s));
    return h;
}

double device_dot(const float *u, const float *v, int64_t n, hipStream_t s) {
    if (n <= 0) return 0.0;
    Scalars sc;
    sc.reset(s);
    csum(1, u, nullptr, v, n, 0.0, sc, sc.v.p, s);
    double h = 0.0;
    FS_HIP(hipMemcpyAsync(&h, sc.v.p, sizeof(double), hipMemcpyDeviceToHost, s));
    FS_HIP(hipStreamSynchronize(s));
    return h;
}

void combine(const float *u, const float *v, int64_t n, double s1, double s2, double cst,
             float *out, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_combine, dim3(blocks_for(n, 256, 8192)), dim3(256), 0, s, u, v, n, s1, s2,
                       cst, out);
    FS_LAUNCHED();
}

double pair_cost_mean(const float *x, const float *a, int64_t n, const float *y, const float *b,
                      int64_t m, int d, int r, const fs_params &p, double *Ma, double *Mb,
                      hipStream_t s) {
    FS_REQUIRE(n > 0 && m > 0, FS_EINVAL, "both measures need at least one point");
    // masses and, for r = 2, the first and second moments about x_0 (translation invariant)
    const unsigned nbx = blocks_for(n, RT, RBLK), nby = blocks_for(m, RT, RBLK);
    DevBuf<double> px((size_t)nbx * (d + 2)), py((size_t)nby * (d + 2)), mx(d + 2), my(d + 2);
    hipLaunchKernelGGL(k_moments, dim3(nbx), dim3(RT), 0, s, x, a, n, d, x, px.p);
    hipLaunchKernelGGL(k_moments, dim3(nby), dim3(RT), 0, s, y, b, m, d, x, py.p);
    hipLaunchKernelGGL(k_moments_final, dim3(d + 2), dim3(RT), 0, s, px.p,
                       (int)nbx, d + 2, mx.p);
    hipLaunchKernelGGL(k_moments_final, dim3(d + 2), dim3(RT), 0, s, py.p,
                       (int)nby, d + 2, my.p);
    FS_LAUNCHED();
    std::vector<double> hx(d + 2), hy(d + 2);
    FS_HIP(hipMemcpyAsync(hx.data(), mx.p, (d + 2) * sizeof(double), hipMemcpyDeviceToHost, s));
    FS_HIP(hipMemcpyAsync(hy.data(), my.p, (d + 2) * sizeof(double), hipMemcpyDeviceToHost, s));
    FS_HIP(hipStreamSynchronize(s));
    *Ma = hx[d];
    *Mb = hy[d];
    if (r == 2) {
        // sum_ij a_i b_j |x_i - y_j|^2 = Mb sum a |x|^2 + Ma sum b |y|^2 - 2 (sum a x).(sum b y)
        double cross = 0.0;
        for (int k = 0; k < d; ++k) cross += hx[k] * hy[k];
        return *Mb * hx[d + 1] + *Ma * hy[d + 1] - 2.0 * cross;
    }
    // r = 1: sum_ij a_i b_j |x_i - y_j| = -<a, K_energy b>, one energy kernel sum
    fs_params q = p;
    q.kernel = FS_ENERGY;
    q.lambda = 1.0;
    auto op = make_op(x, n, y, m, d, q, s);
    DevBuf<float> ao(n + 1), bo(m + 1), t(n + 1);
    op->to_op(0, a, ao.p, s);
    op->to_op(1, b, bo.p, s);
    op->apply(bo.p, t.p, nullptr, 0, s);
    return -device_dot(ao.p, t.p, n, s);
}

void uot_grad_core(Op &op, const float *a, const float *b, const double *f, const double *g,
                   double eps, double rho, double scale, float *dx, float *da, float *dy,
                   float *db, hipStream_t s) {
    const int64_t n = op.n, m = op.m;
    const int d = op.d;
    Scalars sc;
    sc.reset(s);
    double *gmax = sc.v.p + 0, *fmax = sc.v.p + 1, *Mb = sc.v.p + 2, *Ma = sc.v.p + 3;
    DevBuf<float> ao(n + 1), bo(m + 1), w(std::max(n, m) + 1), t(std::max(n, m) + 1),
        gr((std::max(n, m) + 1) * d), ox((std::max(n, m) + 1) * d), o1(std::max(n, m) + 1);
    DevBuf<double> fo(n + 1), go(m + 1), tparts(UPD_BLOCKS);
    DevBuf<int> fhist(FLOOR_BINS);
    const int r = op.kind == FS_GAUSS ? 2 : 1;
    op.to_op(0, a, ao.p, s);
    op.to_op(1, b, bo.p, s);
    op.to_op64(0, f, fo.p, s);
    op.to_op64(1, g, go.p, s);
    if (m > 0) sc.ng = launch_max_parts(go.p, m, sc.gparts.p, s);
    if (n > 0) sc.nf = launch_max_parts(fo.p, n, sc.fparts.p, s);
    hipLaunchKernelGGL(k_max_final, dim3(1), dim3(RT), 0, s, sc.gparts.p, sc.ng, gmax);
    hipLaunchKernelGGL(k_max_final, dim3(1), dim3(RT), 0, s, sc.fparts.p, sc.nf, fmax);
    FS_LAUNCHED();
    {
        double *tmp = sc.v.p + 8;
        csum(2, bo.p, nullptr, nullptr, m, 0.0, sc, tmp, s);
        FS_HIP(hipMemcpyAsync(Mb, tmp, sizeof(double), hipMemcpyDeviceToDevice, s));
        csum(2, ao.p, nullptr, nullptr, n, 0.0, sc, tmp, s);
        FS_HIP(hipMemcpyAsync(Ma, tmp, sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    if ((dx || da) && n > 0) {
        launch_weights(bo.p, go.p, gmax, 1, eps, m, w.p, s);
        op.apply(w.p, t.p, gr.p, 0, s);
        hipLaunchKernelGGL(k_uot_grad_rows, dim3(blocks_for(n, 256, 8192)), dim3(256), 0, s, ao.p,
                           fo.p, t.p, gr.p, d, n, gmax, eps, rho, Mb, scale,
                           dx ? ox.p : nullptr, da ? o1.p : nullptr);
        FS_LAUNCHED();
        if (op.fast)
            grad_floor_rows(ao.p, fo.p, t.p, n, gmax, eps, rho, Mb, scale,
                            FloorSrc{op.coords(0), op.coords(1), bo.p, go.p, m, d, r, 1.0 / eps},
                            tparts.p, fhist.p, dx ? ox.p : nullptr, da ? o1.p : nullptr, s);
        if (dx) op.rows_from_op(0, ox.p, dx, s);
        if (da) op.from_op(0, o1.p, da, s);
    }
    if ((dy || db) && m > 0) {
        launch_weights(ao.p, fo.p, fmax, 1, eps, n, w.p, s);
        op.apply(w.p, t.p, gr.p, 1, s);
        hipLaunchKernelGGL(k_uot_grad_rows, dim3(blocks_for(m, 256, 8192)), dim3(256), 0, s, bo.p,
                           go.p, t.p, gr.p, d, m, fmax, eps, rho, Ma, scale,
                           dy ? ox.p : nullptr, db ? o1.p : nullptr);
        FS_LAUNCHED();
        if (op.fast)
            grad_floor_rows(bo.p, go.p, t.p, m, fmax, eps, rho, Ma, scale,
                            FloorSrc{op.coords(1), op.coords(0), ao.p, fo.p, n, d, r, 1.0 / eps},
                            tparts.p, fhist.p, dy ? ox.p : nullptr, db ? o1.p : nullptr, s);
        if (dy) op.rows_from_op(1, ox.p, dy, s);
        if (db) op.from_op(1, o1.p, db, s);
    }
    FS_HIP(hipStreamSynchronize(s));
}

namespace {

// union point set z = (x, y) in caller order
void make_union(const float *x, int64_t n, const float *y, int64_t m, int d, DevBuf<float> &z,
                hipStream_t s) {
    z.alloc((n + m) * d + 1);
    if (n > 0) FS_HIP(hipMemcpyAsync(z.p, x, n * d * sizeof(float), hipMemcpyDeviceToDevice, s));
    if (m > 0)
        FS_HIP(hipMemcpyAsync(z.p + n * d, y, m * d * sizeof(float), hipMemcpyDeviceToDevice, s));
}

void concat_weights(const float *a, int64_t n, const float *b, int64_t m, float sa, float sb,
                    float *w, hipStream_t s) {
    if (n + m == 0) return;
    hipLaunchKernelGGL(k_concat_weights, dim3(blocks_for(n + m, 256, 8192)), dim3(256), 0, s, a, n,
                       b, m, sa, sb, w);
    FS_LAUNCHED();
}

}  // namespace

void mmd_core(const float *x, const float *a, int64_t n, const float *y, const float *b,
              int64_t m, int d, const fs_params &p, double *mmd2, double *terms3, hipStream_t s) {
    const int64_t nz = n + m;
    if (nz == 0) {
        if (mmd2) *mmd2 = 0.0;
        if (terms3) terms3[0] = terms3[1] = terms3[2] = 0.0;
        return;
    }
    DevBuf<float> z, wz(nz + 1), wo(nz + 1), to(nz + 1);
    make_union(x, n, y, m, d, z, s);
    auto op = make_op(z.p, nz, z.p, nz, d, p, s);
    Scalars sc;
    sc.reset(s);
    double h[8] = {0};
    if (!terms3) {
        // one kernel sum with the signed weights w = (a, -b):  MMD^2 = w . K w
        concat_weights(a, n, b, m, 1.0f, -1.0f, wz.p, s);
        op->to_op(0, wz.p, wo.p, s);
        op->apply(wo.p, to.p, nullptr, 0, s);
        csum(1, wo.p, nullptr, to.p, nz, 0.0, sc, sc.v.p, s);
        FS_HIP(hipMemcpyAsync(h, sc.v.p, sizeof(double), hipMemcpyDeviceToHost, s));
        FS_HIP(hipStreamSynchronize(s));
        if (mmd2) *mmd2 = h[0];
        return;
    }
    // two kernel sums, K (a, 0) and K (0, b), give the three double sums of eq. (1205)
    DevBuf<float> w2(nz + 1), t2(nz + 1);
    concat_weights(a, n, b, m, 1.0f, 0.0f, wz.p, s);
    op->to_op(0, wz.p, wo.p, s);
    op->apply(wo.p, to.p, nullptr, 0, s);
    concat_weights(a, n, b, m, 0.0f, 1.0f, wz.p, s);
    op->to_op(0, wz.p, w2.p, s);
    op->apply(w2.p, t2.p, nullptr, 0, s);
    csum(1, wo.p, nullptr, to.p, nz, 0.0, sc, sc.v.p + 8, s);   // a K a
    csum(1, wo.p, nullptr, t2.p, nz, 0.0, sc, sc.v.p + 12, s);  // a K b
    csum(1, w2.p, nullptr, t2.p, nz, 0.0, sc, sc.v.p + 16, s);  // b K b
    double hv[20];
    FS_HIP(hipMemcpyAsync(hv, sc.v.p, sizeof(hv), hipMemcpyDeviceToHost, s));
    FS_HIP(hipStreamSynchronize(s));
    terms3[0] = hv[8];
    terms3[1] = hv[12];
    terms3[2] = hv[16];
    if (mmd2) *mmd2 = hv[8] - 2.0 * hv[12] + hv[16];
}

void mmd_grad_core(const float *x, const float *a, int64_t n, const float *y, const float *b,
                   int64_t m, int d, const fs_params &p, double scale, float *dx, float *da,
                   float *dy, float *db, hipStream_t s) {
    const int64_t nz = n + m;
    if (nz == 0) return;
    DevBuf<float> z, wz(nz + 1), wo(nz + 1), to(nz + 1), go(nz * d + 1);
    make_union(x, n, y, m, d, z, s);
    auto op = make_op(z.p, nz, z.p, nz, d, p, s);
    concat_weights(a, n, b, m, 1.0f, -1.0f, wz.p, s);
    op->to_op(0, wz.p, wo.p, s);
    op->apply(wo.p, to.p, go.p, 0, s);
    const int *perm = op->fast ? op->plan->X.perm.p : nullptr;
    hipLaunchKernelGGL(k_mmd_grad_rows, dim3(blocks_for(nz, 256, 8192)), dim3(256), 0, s, wo.p,
                       to.p, go.p, perm, nz, n, d, scale, dx, da, dy, db);
    FS_LAUNCHED();
    FS_HIP(hipStreamSynchronize(s));
}

}  // namespace fs
