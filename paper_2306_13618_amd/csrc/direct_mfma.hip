// Gaussian kernel sum for high dimension (d a multiple of 16) with the whole exponent on the
// matrix cores.  The kernel depends only on differences, so both point sets are first shifted
// by a common centre c (the midpoint of their joint bounding box).  With s = sqrt(2 log2(e) /
// lambda), p' = p - c and a_i = -(log2(e) / lambda) |x'_i|^2,
//   log2 K_ij = -(log2(e) / lambda) |x_i - y_j|^2 = (s x'_i).(s y'_j) + a_i + b_j,
// so one Gram tile of augmented vectors gives the exponent directly:
//   * each scaled coordinate is split into FP16 hi = f16(v) and lo = f16(v - hi) (22 significant
//     bits); the dot product is hi.hi + hi.lo + lo.hi accumulated in FP32 on the FP16 matrix
//     instructions (the dropped lo.lo term is ~2^-22 of the product);
//   * the norm terms ride in one extra K step on the BF16 matrix instruction (BF16 keeps the
//     exponent range of FP32 for large |a|): a_i is split into three BF16 pieces (24 bits),
//     A_i = [a_h, a_m, a_l, 1, 1, 1] against B_j = [1, 1, 1, b_h, b_m, b_l].
// Then K_ij = exp2(g_ij), and sum_j K_ij w_j is accumulated per lane in FP32 over two stages of
// column tiles and in FP64 beyond.
//
// Accuracy.  Near pairs, which dominate a row sum, get g ~ 0 from terms of size up to
// Q = (log2(e) / lambda) (R_x + R_y)^2 (R: largest centred norm of a set), so the absolute error
// of g grows with Q (splits and FP32 accumulation).  An emulation of this arithmetic on uniform,
// Gaussian, shifted and clustered clouds in d = 16 ... 128 keeps the relative error of the sums
// at or below 2.5e-6 for Q <= 64; gram_frame measures Q and the Gram path is used only there
// (the FP32 VALU kernel otherwise).
//
// Wave tile: 32 target rows x 32 source columns, v_mfma_f32_32x32x16_f16 / _bf16 (gfx950).
// Operand layout of those instructions (per lane l of the wave):
//   A (32 x 16):  row l % 32, k = 8 (l / 32) .. 8 (l / 32) + 7
//   B (16 x 32):  column l % 32, same k range
//   D (32 x 32):  register r holds row 8 (r / 4) + 4 (l / 32) + (r % 4), column l % 32
// The packed operand array stores, per tile of 32 points and per part, the 16 bytes each lane
// loads, so a wave's operand load is one contiguous 1 KB read.  Parts: hi for each K step, lo for
// each K step, the A-role norm step, the B-role norm step.
//
// A workgroup of 4 waves takes 128 rows and one split of the column tiles; the column tiles are
// staged through LDS (double buffered, one barrier per stage) and shared by the 4 waves.  Within
// a stage the MFMAs of the next tile are issued before the exponentials of the current one.
#include "direct.h"

namespace fs {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

template <int D>
struct GramShape {
    static constexpr int KS = D / 16;                 // K steps of 16
    static constexpr int PARTS = 2 * KS + 2;          // stored parts per tile
    static constexpr int UPARTS = 2 * KS + 1;         // parts one role uses
    static constexpr int TPS = D <= 32 ? 4 : (D == 64 ? 2 : 1);  // column tiles per stage
    static constexpr int UNITS = TPS * UPARTS * 64;   // 16-byte units per stage
    static constexpr int NLD = (UNITS + 255) / 256;   // units per thread per stage
};

__device__ __forceinline__ uint16_t f2bf_bits(float v) {
    // round to nearest even (inputs are finite)
    uint32_t u = __float_as_uint(v);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf_bits2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ uint16_t f2h_bits(float v) {
    return __builtin_bit_cast(uint16_t, (_Float16)v);  // round to nearest even
}
__device__ __forceinline__ float h_bits2f(uint16_t b) { return (float)__builtin_bit_cast(_Float16, b); }

// One thread per (point, half): writes that lane's units of every part.  Points beyond `count`
// (the tail of the last tile) get all-zero parts.  Coordinates are centred on `center` (d).
__global__ void k_gram_pack(const float *__restrict__ p, int64_t count, int d, int parts,
                            double scale, double anorm, const float *__restrict__ center,
                            int64_t padded, u16x8 *__restrict__ packed) {
    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (gid >= 2 * padded) return;
    const int64_t i = gid >> 1;
    const int h = (int)(gid & 1);
    const int ks = d / 16;
    const int64_t tile = i / 32;
    const int lane = (int)(i % 32) + 32 * h;
    u16x8 *base = packed + tile * parts * 64 + lane;
    const bool ok = i < count;
    double a = 0.0;
    if (ok) {
        for (int k = 0; k < d; ++k) {
            const double v = (double)p[i * d + k] - (double)center[k];
            a = fma(v, v, a);
        }
        a *= -anorm;
    }
    for (int s = 0; s < ks; ++s) {
        u16x8 hi = {}, lo = {};
        if (ok)
            for (int e = 0; e < 8; ++e) {
                const int k = 16 * s + 8 * h + e;
                const float v = (float)(scale * ((double)p[i * d + k] - (double)center[k]));
                const uint16_t hb = f2h_bits(v);
                hi[e] = hb;
                lo[e] = f2h_bits(v - h_bits2f(hb));
            }
        base[(int64_t)s * 64] = hi;
        base[(int64_t)(ks + s) * 64] = lo;
    }
    u16x8 augA = {}, augB = {};
    if (ok && h == 0) {
        const uint16_t one = 0x3f80;
        const uint16_t ah = f2bf_bits((float)a);
        const double r1 = a - (double)bf_bits2f(ah);
        const uint16_t am = f2bf_bits((float)r1);
        const uint16_t al = f2bf_bits((float)(r1 - (double)bf_bits2f(am)));
        augA[0] = ah; augA[1] = am; augA[2] = al; augA[3] = one; augA[4] = one; augA[5] = one;
        augB[0] = one; augB[1] = one; augB[2] = one; augB[3] = ah; augB[4] = am; augB[5] = al;
    }
    base[(int64_t)(2 * ks) * 64] = augA;
    base[(int64_t)(2 * ks + 1) * 64] = augB;
}

template <int D>
__device__ __forceinline__ f32x16 gram_tile(const f16x8 *ah, const f16x8 *al, bf16x8 aaug,
                                            const u16x8 *sb, int lane) {
    using S = GramShape<D>;
    f32x16 g = {};
    g = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aaug, __builtin_bit_cast(bf16x8, sb[2 * S::KS * 64 + lane]), g, 0, 0, 0);
#pragma unroll
    for (int s = 0; s < S::KS; ++s) {
        const f16x8 bh = __builtin_bit_cast(f16x8, sb[s * 64 + lane]);
        const f16x8 bl = __builtin_bit_cast(f16x8, sb[(S::KS + s) * 64 + lane]);
        g = __builtin_amdgcn_mfma_f32_32x32x16_f16(al[s], bh, g, 0, 0, 0);
        g = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah[s], bl, g, 0, 0, 0);
        g = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah[s], bh, g, 0, 0, 0);
    }
    return g;
}

template <int D>
__global__ void __launch_bounds__(256) k_gram_gauss(
    const u16x8 *__restrict__ A, int64_t n, const u16x8 *__restrict__ B, int64_t m,
    const float *__restrict__ w, int tiles_per_split, double *__restrict__ partial,
    float *__restrict__ out, double *__restrict__ out64) {
    using S = GramShape<D>;
    __shared__ u16x8 sB[2][S::TPS][S::UPARTS * 64];
    __shared__ float sw[2][S::TPS][32];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int half = lane >> 5;
    const int64_t ntn = (n + 31) / 32, ntm = (m + 31) / 32;
    const int64_t rt = (int64_t)blockIdx.x * 4 + wave;  // row tile of this wave
    const bool rows_ok = rt < ntn;

    f16x8 ah[S::KS], al[S::KS];
    bf16x8 aaug;
    {
        const u16x8 *a = A + (rows_ok ? rt : 0) * S::PARTS * 64 + lane;
        const u16x8 z = {};
#pragma unroll
        for (int s = 0; s < S::KS; ++s) {
            ah[s] = __builtin_bit_cast(f16x8, rows_ok ? a[s * 64] : z);
            al[s] = __builtin_bit_cast(f16x8, rows_ok ? a[(S::KS + s) * 64] : z);
        }
        aaug = __builtin_bit_cast(bf16x8, rows_ok ? a[2 * S::KS * 64] : z);
    }

    const int64_t c0 = (int64_t)blockIdx.y * tiles_per_split;
    const int64_t c1 = c0 + tiles_per_split < ntm ? c0 + tiles_per_split : ntm;

    u16x8 pre[S::NLD];
    float prew = 0.0f;
    auto load_stage = [&](int64_t st) {
#pragma unroll
        for (int q = 0; q < S::NLD; ++q) {
            const int u = tid + 256 * q;
            const int t = u / (S::UPARTS * 64), rem = u % (S::UPARTS * 64);
            const int part = rem / 64;  // B role: parts 0 .. 2KS-1, then the B-role norm step
            const int sp = part < 2 * S::KS ? part : 2 * S::KS + 1;
            const int64_t ct = st + t;
            if (u < S::UNITS && ct < c1) {
                pre[q] = B[(ct * S::PARTS + sp) * 64 + (rem % 64)];
            } else {
                const u16x8 z = {};
                pre[q] = z;
            }
        }
        if (tid < S::TPS * 32) {
            const int64_t j = (st + tid / 32) * 32 + (tid % 32);
            prew = (st + tid / 32 < c1 && j < m) ? w[j] : 0.0f;
        }
    };
    auto store_stage = [&](int buf) {
#pragma unroll
        for (int q = 0; q < S::NLD; ++q) {
            const int u = tid + 256 * q;
            if (u < S::UNITS) sB[buf][u / (S::UPARTS * 64)][u % (S::UPARTS * 64)] = pre[q];
        }
        if (tid < S::TPS * 32) sw[buf][tid / 32][tid % 32] = prew;
    };

    // per-lane FP32 partial sums over two stages (up to 8 tiles = 256 terms), FP64 beyond
    float part[16];
    double acc[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        acc[r] = 0.0;
        part[r] = 0.0f;
    }

    if (c0 < c1) load_stage(c0);
    int buf = 0;
    for (int64_t st = c0; st < c1; st += S::TPS, buf ^= 1) {
        store_stage(buf);
        __syncthreads();
        if (st + S::TPS < c1) load_stage(st + S::TPS);
        f32x16 g = gram_tile<D>(ah, al, aaug, sB[buf][0], lane);
#pragma unroll
        for (int t = 0; t < S::TPS; ++t) {
            f32x16 gn = {};
            if (t + 1 < S::TPS) gn = gram_tile<D>(ah, al, aaug, sB[buf][t + 1], lane);
            const float wj = sw[buf][t][lane & 31];
#pragma unroll
            for (int r = 0; r < 16; ++r) part[r] = fmaf(__builtin_amdgcn_exp2f(g[r]), wj, part[r]);
            g = gn;
        }
        if (buf == 1 || st + S::TPS >= c1) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                acc[r] += (double)part[r];
                part[r] = 0.0f;
            }
        }
    }
    // reduce over the 32 lanes of each half-wave (they hold the same rows, different columns)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        double v = acc[r];
#pragma unroll
        for (int off = 16; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        acc[r] = v;
    }
    if ((lane & 31) == 0 && rows_ok) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t row = rt * 32 + 8 * (r / 4) + 4 * half + (r % 4);
            if (row < n) {
                if (partial) {
                    partial[(int64_t)blockIdx.y * n + row] = acc[r];
                } else {
                    if (out) out[row] = (float)acc[r];
                    if (out64) out64[row] = acc[r];
                }
            }
        }
    }
}

__global__ void k_gram_combine(const double *__restrict__ partial, int64_t n, int splits,
                               float *__restrict__ out, double *__restrict__ out64) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v = 0.0;
    for (int k = 0; k < splits; ++k) v += partial[(int64_t)k * n + i];
    if (out) out[i] = (float)v;
    if (out64) out64[i] = v;
}

// Per-workgroup minimum and maximum of every coordinate (d divides 256): thread t of a workgroup
// always reads coordinate t % d of the row-major array, so the loads are contiguous.
__global__ void __launch_bounds__(256) k_coord_minmax(const float *__restrict__ p, int64_t count,
                                                      int d, float *__restrict__ part) {
    __shared__ float lo_s[256], hi_s[256];
    const int tid = threadIdx.x;
    float lo = INFINITY, hi = -INFINITY;
    const int64_t total = count * d;
    for (int64_t f = (int64_t)blockIdx.x * 256 + tid; f < total; f += (int64_t)gridDim.x * 256) {
        const float v = p[f];
        lo = fminf(lo, v);
        hi = fmaxf(hi, v);
    }
    lo_s[tid] = lo;
    hi_s[tid] = hi;
    __syncthreads();
    if (tid < d) {
        for (int t = tid + d; t < 256; t += d) {
            lo = fminf(lo, lo_s[t]);
            hi = fmaxf(hi, hi_s[t]);
        }
        part[(int64_t)blockIdx.x * 2 * d + tid] = lo;
        part[(int64_t)blockIdx.x * 2 * d + d + tid] = hi;
    }
}

// Per-workgroup maximum of |p_i - c|^2 (FP64 sums, rounded up to float).
__global__ void __launch_bounds__(256) k_centered_norm2_max(const float *__restrict__ p,
                                                            int64_t count, int d,
                                                            const float *__restrict__ center,
                                                            float *__restrict__ part) {
    __shared__ float m_s[256];
    const int tid = threadIdx.x;
    double mx = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + tid; i < count; i += (int64_t)gridDim.x * 256) {
        double a = 0.0;
        for (int k = 0; k < d; ++k) {
            const double v = (double)p[i * d + k] - (double)center[k];
            a = fma(v, v, a);
        }
        mx = fmax(mx, a);
    }
    m_s[tid] = (float)(mx * (1.0 + 1e-6));
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) m_s[tid] = fmaxf(m_s[tid], m_s[tid + w]);
        __syncthreads();
    }
    if (tid == 0) part[blockIdx.x] = m_s[0];
}

constexpr int FRAME_BLOCKS = 256;

}  // namespace

bool mfma_supported(int kind, int d) { return kind == FS_GAUSS && (d == 16 || d == 32 || d == 64 || d == 128); }

double gram_frame(const float *x, int64_t n, const float *y, int64_t m, bool same, int d,
                  double lambda, DevBuf<float> &center, hipStream_t s) {
    FS_REQUIRE(mfma_supported(FS_GAUSS, d), FS_EINVAL, "MFMA path needs d in {16,32,64,128}");
    const int nsets = same ? 1 : 2;
    const float *pts[2] = {x, y};
    const int64_t cnt[2] = {n, m};
    DevBuf<float> part((size_t)nsets * FRAME_BLOCKS * 2 * d);
    HostStage hs(s);
    std::vector<const float *> got(nsets);
    std::vector<int> nb(nsets);
    for (int k = 0; k < nsets; ++k) {
        nb[k] = (int)blocks_for(cnt[k] * d, 256, FRAME_BLOCKS);
        if (cnt[k] > 0) {
            hipLaunchKernelGGL(k_coord_minmax, dim3(nb[k]), dim3(256), 0, s, pts[k], cnt[k], d,
                               part.p + (size_t)k * FRAME_BLOCKS * 2 * d);
            FS_LAUNCHED();
        }
        got[k] = hs.download(part.p + (size_t)k * FRAME_BLOCKS * 2 * d, (size_t)nb[k] * 2 * d);
    }
    FS_HIP(hipStreamSynchronize(s));
    std::vector<float> c(d);
    for (int j = 0; j < d; ++j) {
        double lo = INFINITY, hi = -INFINITY;
        for (int k = 0; k < nsets; ++k)
            for (int b = 0; cnt[k] > 0 && b < nb[k]; ++b) {
                lo = std::min(lo, (double)got[k][(size_t)b * 2 * d + j]);
                hi = std::max(hi, (double)got[k][(size_t)b * 2 * d + d + j]);
            }
        c[j] = std::isfinite(lo) && std::isfinite(hi) ? (float)(0.5 * (lo + hi)) : 0.0f;
    }
    center.alloc(d);
    hs.upload(center.p, c.data(), d * sizeof(float));
    for (int k = 0; k < nsets; ++k) {
        nb[k] = (int)blocks_for(cnt[k], 256, FRAME_BLOCKS);
        if (cnt[k] > 0) {
            hipLaunchKernelGGL(k_centered_norm2_max, dim3(nb[k]), dim3(256), 0, s, pts[k], cnt[k],
                               d, center.p, part.p + (size_t)k * FRAME_BLOCKS);
            FS_LAUNCHED();
        }
        got[k] = hs.download(part.p + (size_t)k * FRAME_BLOCKS, (size_t)nb[k]);
    }
    FS_HIP(hipStreamSynchronize(s));
    double r[2] = {0.0, 0.0};
    for (int k = 0; k < nsets; ++k)
        for (int b = 0; cnt[k] > 0 && b < nb[k]; ++b) r[k] = std::max(r[k], (double)got[k][b]);
    if (same) r[1] = r[0];
    const double l2e = 1.4426950408889634;
    const double rs = std::sqrt(r[0]) + std::sqrt(r[1]);
    return l2e / lambda * rs * rs;
}

void gram_prepare(const float *pts, int64_t count, int d, double lambda, const float *center,
                  GramOperand &op, hipStream_t s) {
    FS_REQUIRE(mfma_supported(FS_GAUSS, d), FS_EINVAL, "MFMA path needs d in {16,32,64,128}");
    op.count = count;
    op.d = d;
    op.parts = 2 * (d / 16) + 2;
    const int64_t tiles = (count + 31) / 32;
    op.packed.alloc((size_t)(std::max<int64_t>(tiles, 1) * op.parts * 64 * 8));
    if (count == 0) return;
    const double l2e = 1.4426950408889634;
    const double scale = std::sqrt(2.0 * l2e / lambda);
    const double anorm = l2e / lambda;
    hipLaunchKernelGGL(k_gram_pack, dim3(blocks_for(2 * tiles * 32, 256, int64_t(1) << 30)),
                       dim3(256), 0, s, pts, count, d, op.parts, scale, anorm, center, tiles * 32,
                       reinterpret_cast<u16x8 *>(op.packed.p));
    FS_LAUNCHED();
}

void direct_mfma_gauss(const GramOperand &x, const GramOperand &y, const float *w, float *out,
                       double *out64, hipStream_t s, double *ext_partial, size_t ext_count) {
    FS_REQUIRE(x.d == y.d && mfma_supported(FS_GAUSS, x.d), FS_EINVAL,
               "MFMA path needs matching d in {16,32,64,128}");
    if (x.count == 0) return;
    const int64_t ntn = (x.count + 31) / 32, ntm = (y.count + 31) / 32;
    const int64_t rblocks = (ntn + 3) / 4;
    FS_REQUIRE(rblocks < (int64_t(1) << 31), FS_EINVAL, "too many rows for the MFMA path");
    // split the columns so that the launch holds about 8192 workgroups (several rounds of the
    // chip), keeping at least 64 column tiles per workgroup
    int64_t splits = std::max<int64_t>(1, (8192 + rblocks - 1) / rblocks);
    splits = std::min<int64_t>(splits, std::max<int64_t>(1, ntm / 64));
    splits = std::min<int64_t>(splits, 65535);
    // a caller-provided partial-sum buffer bounds the number of splits (one split needs none)
    if (ext_partial) splits = std::min<int64_t>(splits, std::max<int64_t>(1, (int64_t)(ext_count / (size_t)x.count)));
    const int64_t per = (ntm + splits - 1) / splits;
    splits = std::max<int64_t>(1, (ntm + per - 1) / per);
    DevBuf<double> partial;
    if (splits > 1 && !ext_partial) partial.alloc((size_t)(splits * x.count));
    double *part = ext_partial ? ext_partial : partial.p;
    const u16x8 *A = reinterpret_cast<const u16x8 *>(x.packed.p);
    const u16x8 *B = reinterpret_cast<const u16x8 *>(y.packed.p);
    dim3 grid((unsigned)rblocks, (unsigned)splits), block(256);
#define FS_GRAM(DD)                                                                           \
    hipLaunchKernelGGL(k_gram_gauss<DD>, grid, block, 0, s, A, x.count, B, y.count, w,       \
                       (int)per, splits > 1 ? part : nullptr, out, out64)
    switch (x.d) {
        case 16: FS_GRAM(16); break;
        case 32: FS_GRAM(32); break;
        case 64: FS_GRAM(64); break;
        default: FS_GRAM(128); break;
    }
#undef FS_GRAM
    FS_LAUNCHED();
    if (splits > 1) {
        hipLaunchKernelGGL(k_gram_combine, dim3(blocks_for(x.count, 256, int64_t(1) << 30)),
                           dim3(256), 0, s, part, x.count, (int)splits, out, out64);
        FS_LAUNCHED();
    }
    // the two kernels above are still queued: the partial sums go back to the workspace cache
    // only once the stream has passed them
    partial.reset_after(s);
}

}  // namespace fs
