// NFFT fast summation plan (eq. (1724)): torus scaling, kernel regularisation and Fourier
// multiplier, node binning, and the spread / FFT / gather / near-field passes.
#pragma once
#include "internal.h"

namespace fs {

// A point set mapped to the torus and sorted by grid tile.
struct Nodes {
    int64_t n = 0;
    DevBuf<float4> rec;     // sorted: fractional grid offsets (x, y, z) and packed grid cell in .w
    DevBuf<int> perm;       // sorted position -> original index
    DevBuf<float> xs;       // sorted coordinates (n x d, data units)
    DevBuf<int4> chunks;    // (tile, first node, node count, 0)
    int nchunks = 0;
    // per tile: [first chunk, chunk count] (then the binning's totals and groups per tile)
    DevBuf<int> tile_chunk;
    // tile lists built on the host in one upload; the pointers below point into it
    DevBuf<int> tile_lists;
    const int *multi_tiles = nullptr;  // tiles holding more than one chunk
    int n_multi = 0;
    const int *touched_tiles = nullptr;  // tiles with a chunk in their 3^d neighbourhood
    int n_touched = 0;
    // near-field cell list (sources only): cell-sorted index -> tile-sorted position
    DevBuf<int> nf_cell_start;  // ncells + 1
    DevBuf<int> nf_order;       // cell-sorted k -> tile-sorted position
    DevBuf<float> nf_xs;        // cell-sorted coordinates
    DevBuf<int4> nf_blocks;     // target blocks (<= 64 targets inside one row of cells)
    int nf_nblocks = 0;
    // matrix-core groups (d = 3): up to 16 consecutive nodes inside one brick of BRICK_X cells
    // along x (same y and z cell); groups (first node, count, brick offset in the tile's box, 0)
    // and blocks of groups inside one tile (tile, first group, group count, 0)
    DevBuf<int4> mgroups, mblocks;
    DevBuf<int2> mbnodes;  // per block: first node, node count
    int n_mgroups = 0, n_mblocks = 0;
    const int *mtile_block = nullptr;   // per tile: [first block, block count]
    const int *mmulti_tiles = nullptr;  // tiles holding more than one block
    int n_mmulti = 0;
};

constexpr int BRICK_X = 4;
// Waves per workgroup of the 3-D matrix-core spread and gather (each wave takes a contiguous run
// of the workgroup's groups; the workgroup shares one box of the tile).
constexpr int MW = 8;
constexpr int MIN_GROUPS_PER_BLOCK = MW;  // one per wave

enum Regime { REGIME_CUBE = 0, REGIME_BALL = 1 };

// Window segment polynomials: on the unit cell of a node (fractional offset t in [0, 1)), the
// window value at grid offset a is phi(t + m - 1 - a), written as a degree-(WPOLY-1)
// polynomial in u = 2t - 1 (fitted in FP64 per plan).
constexpr int WPOLY = 8;

struct PlanParams {
    int d = 0, kind = FS_GAUSS;
    double lambda = 1.0;
    int G = 0, N = 0, sigma = 2, m = 6, W = 12, p = 8;
    int T = 8;          // tile side (grid points)
    int chunk = 1024;   // nodes per spread/gather chunk
    double P = 1.0;     // period in data units (torus unit)
    double center[3] = {0, 0, 0};
    int regime = REGIME_CUBE;
    double epsI = 0.0;  // inner regularisation radius (torus units), 0 = none
    double epsB = 0.0;  // boundary zone width (torus units), 0 = none
    double ci[16] = {0};  // inner polynomial  sum_k ci[k] r^(2k), k < p   (torus units)
    double cb[32] = {0};  // boundary polynomial sum_k cb[k] (r - 1/2)^k, k <= 2p-2
    bool nearfield = false;
    bool stable = false;  // deterministic mode: stable node order, no atomic partial sums
    // near-field cell grid (data units)
    double nf_h = 0.0;
    int nf_R = 2;  // stencil half-width in cells: nf_R * nf_h >= radius
    int nf_dims[3] = {1, 1, 1};
    double nf_lo[3] = {0, 0, 0};
    KB kb{};
};

struct Plan {
    PlanParams pp;
    unsigned flags = 0;
    Nodes X, Y;          // targets and sources (transpose swaps the roles)
    bool same = false;   // Y is X (symmetric problems): Y aliases X
    DevBuf<float> Mk;    // multiplier (N/2+1)^d
    DevBuf<float> grid;  // G^d real
    DevBuf<float2> specA, specB;
    DevBuf<float2> twiddle;  // exp(-2 pi i q / G), q < G/2
    DevBuf<uint4> mom_cc;    // 3-D moment-form spread: Chebyshev transform operands
    DevBuf<float> wpoly;     // window segments as polynomials: value (W x WPOLY) then derivative
    DevBuf<float> scratch;   // per-chunk spread boxes
    DevBuf<float4> nf_src;   // near-field source records (cell order) for the current weights
    const Nodes &src(int transpose) const { return transpose ? X : (same ? X : Y); }
    const Nodes &dst(int transpose) const { return transpose ? (same ? X : Y) : X; }
};

// Plan creation: x (n x d) targets, y (m x d) sources (y == x allowed: symmetric plan).
void plan_build(Plan &pl, const float *x, int64_t n, const float *y, int64_t m, int d,
                const fs_params &p, hipStream_t s);

// Fast kernel sum in sorted order: w_sorted (source order) -> t_sorted (target order), float32.
// transpose = 0: sources Y, targets X.  With `grad` != NULL also writes the gradient of the sum
// with respect to the target position (n x d, data units).
void plan_apply_sorted(Plan &pl, const float *w_sorted, float *t_sorted, float *grad,
                       int transpose, hipStream_t s);

// Source weights given as w_k = base_k exp((pot_k - pmax) / eps), FP64 exponent, FP32 result
// (a Sinkhorn half-step), pmax the largest of nparts per-block maxima (0 when all are -inf).
// With bbase set, parts are instead the per-block maxima of pot over the source set's matrix-core
// blocks (as the fused update over that set writes them) and bbase the blocks' largest |base|; the
// 3-D spread then bounds its block's largest weight by them instead of reading the block's nodes.
struct PotWeights {
    const float *base = nullptr;
    const double *pot = nullptr, *parts = nullptr;
    int nparts = 0;
    double inv_eps = 1.0;
    const float *bbase = nullptr;
};

// The potential update of a Sinkhorn half-step applied to the kernel sums t_k as they are
// formed: pot_k = -kappa (shift + eps log t_k), shift the largest of nshift maxima (0 when all
// are -inf); one maximum of the new potential per workgroup goes to out_parts (and of |new - old|
// to delta_parts when it is not null); non-positive sums are counted in *nbad and replaced by the
// smallest normal float.
struct PotUpdate {
    const double *shift_parts = nullptr;
    int nshift = 0;
    double kappa = 1.0, eps = 1.0;
    double *pot = nullptr, *out_parts = nullptr, *delta_parts = nullptr;
    int *nbad = nullptr;
};

// True when the kernel sum of this direction evaluates such weights inside its spread (2-D or
// 3-D matrix-core spread, no near field); plan_apply_sorted_pot then needs no weight array.
bool plan_fuses_weights(const Plan &pl, int transpose);
// True when, in addition, the gather forms the potential update itself (matrix-core gather);
// plan_update_parts is then the number of maxima it writes.
bool plan_fuses_update(const Plan &pl, int transpose);
int plan_update_parts(const Plan &pl, int transpose);
// Largest |base_k| over each matrix-core block of the direction's source set (base in sorted
// order; out: plan_source_blocks values), for PotWeights::bbase.
int plan_source_blocks(const Plan &pl, int transpose);
void plan_block_base_max(const Plan &pl, const float *base_sorted, int transpose, float *out,
                         hipStream_t s);
// With pu the sums are not stored: the gather applies the update (t_sorted may be null).
void plan_apply_sorted_pot(Plan &pl, const PotWeights &pw, float *t_sorted, int transpose,
                           hipStream_t s, const PotUpdate *pu = nullptr);
// Inspection: the multiplier M_k ((N/2+1)^d floats, k >= 0 in every coordinate, first coordinate
// fastest), the window transform phihat(k) used in its deconvolution (N/2+1 values), the torus
// period in data units and the bandwidth N.  Either array may be null.
void plan_multiplier(const Plan &pl, float *mult_host, double *phihat_host, int64_t count,
                     double *period, int *bandwidth, hipStream_t s);
// Drop the cached multipliers of recent plans (after a device synchronisation).
void plan_release_mult_cache();

// Permutations between caller order and a node set's sorted order.
void gather_to_sorted(const Nodes &nd, const float *v, float *v_sorted, hipStream_t s);
void scatter_from_sorted(const Nodes &nd, const float *v_sorted, float *v, hipStream_t s);
void gather_to_sorted64(const Nodes &nd, const double *v, double *v_sorted, hipStream_t s);
void scatter_from_sorted64(const Nodes &nd, const double *v_sorted, double *v, hipStream_t s);
void scatter_rows_from_sorted(const Nodes &nd, const float *v_sorted, int d, float *v,
                              hipStream_t s);

}  // namespace fs
