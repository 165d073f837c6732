// Operators (direct or NFFT) and the Sinkhorn / MMD drivers built on them.
#pragma once
#include <memory>

#include "direct.h"
#include "nfft.h"

namespace fs {

// A kernel-sum operator between a target set X (n) and a source set Y (m).  "Operator order" is
// the order in which the operator wants its vectors: tile-sorted for the NFFT path, the caller's
// order for the direct path.
struct Op {
    bool fast = false;
    bool mfma = false;
    int d = 0, kind = FS_GAUSS;
    double lambda = 1.0;
    unsigned flags = 0;
    int64_t n = 0, m = 0;
    const float *x = nullptr, *y = nullptr;  // caller order (direct path)
    bool same = false;
    std::unique_ptr<Plan> plan;
    GramOperand gx, gy;
    DevBuf<float> gcenter;  // common centre of the Gram path's point sets (d)
    DevBuf<float> xcopy, ycopy;  // direct path keeps copies only when asked to

    int64_t count(int side) const { return side == 0 ? n : m; }  // 0: X, 1: Y
    // caller order -> operator order (side 0: X, 1: Y)
    void to_op(int side, const float *v, float *vo, hipStream_t s) const;
    void to_op64(int side, const double *v, double *vo, hipStream_t s) const;
    void from_op(int side, const float *vo, float *v, hipStream_t s) const;
    void from_op64(int side, const double *vo, double *v, hipStream_t s) const;
    void rows_from_op(int side, const float *vo, float *v, hipStream_t s) const;
    // coordinates of a side in operator order (n x d)
    const float *coords(int side) const;
    // transpose = 0: t (X, op order) = K w (Y, op order); 1: t (Y) = K^T w (X).
    // grad (nullable): gradient of t with respect to the target positions (op order, x d).
    // ext_partial / ext_count: caller-owned scratch for the direct matrix-core path's partial
    // sums (no allocation then); ignored elsewhere.
    void apply(const float *w, float *t, float *grad, int transpose, hipStream_t s,
               double *ext_partial = nullptr, size_t ext_count = 0);
    // The same sum with source weights base_k exp((pot_k - max) / eps) (max: the largest of
    // nparts per-block maxima), formed inside the spread where the plan supports it
    // (fuses_weights), else through the weight array w.
    bool fuses_weights(int transpose) const;
    void apply_pot(const float *base, const double *pot, const double *parts, int nparts,
                   double eps, float *w, float *t, int transpose, hipStream_t s);
    // Direct Gauss/Laplace sums on the VALU: the Sinkhorn half-step's sums are taken in the log
    // domain (per-row running maximum), logt (FP64) = log of the same sums as apply_pot's t.
    bool log_direct() const;
    void apply_pot_log(const float *base, const double *pot, const double *parts, int nparts,
                       double eps, float *u, double *logt, int transpose, hipStream_t s);
    // The same, with the potential update applied to the sums inside the gather (no t): only
    // where fuses_update; update_parts maxima are then written.
    bool fuses_update(int transpose) const;
    int update_parts(int transpose) const;
    // bbase (nullable): the source blocks' largest |base| (block_base_max), given when parts are
    // the per-block maxima that the previous fused update over the same set wrote.
    void apply_pot_update(const float *base, const double *pot, const double *parts, int nparts,
                          double eps, const PotUpdate &pu, int transpose, hipStream_t s,
                          const float *bbase = nullptr);
    // Matrix-core blocks of the direction's source set and their largest |base| (fast path).
    int source_blocks(int transpose) const;
    void block_base_max(const float *base, int transpose, float *out, hipStream_t s) const;
};

std::unique_ptr<Op> make_op(const float *x, int64_t n, const float *y, int64_t m, int d,
                            const fs_params &p, hipStream_t s);

struct SinkhornResult {
    double objective = 0.0;
};

// Sinkhorn in operator order.  a_o (n), b_o (m) float weights; f_o, g_o double potentials
// (in/out; used as starting values when warm).
// tol > 0: stop after the first sweep that changes no potential by more than tol * eps;
// sweeps_done (nullable) receives the number of sweeps run.
void sinkhorn_solve(Op &op, const float *a_o, const float *b_o, double eps, double rho, int iters,
                    bool warm, double *f_o, double *g_o, double *objective_host, hipStream_t s,
                    double tol = 0.0, int *sweeps_done = nullptr);

// Envelope gradients of the UOT dual at given potentials (caller order in and out); any output
// may be NULL.  Scaled by `scale`.
void uot_grad_core(Op &op, const float *a, const float *b, const double *f, const double *g,
                   double eps, double rho, double scale, float *dx, float *da, float *dy,
                   float *db, hipStream_t s);

// MMD^2 on the union z = (x, y) with weights (a, -b); terms3 (nullable) gets the three sums.
void mmd_core(const float *x, const float *a, int64_t n, const float *y, const float *b,
              int64_t m, int d, const fs_params &p, double *mmd2, double *terms3, hipStream_t s);
void mmd_grad_core(const float *x, const float *a, int64_t n, const float *y, const float *b,
                   int64_t m, int d, const fs_params &p, double scale, float *dx, float *da,
                   float *dy, float *db, hipStream_t s);

// <mu x nu, d^r> = sum_ij a_i b_j |x_i - y_j|^r (eq. (561)): r = 2 from moments in FP64, r = 1
// through one energy-kernel sum with the grid settings of p; also returns the two masses.
double pair_cost_mean(const float *x, const float *a, int64_t n, const float *y, const float *b,
                      int64_t m, int d, int r, const fs_params &p, double *Ma, double *Mb,
                      hipStream_t s);

// Compensated FP64 sum / dot of float vectors on the device, returned to the host.
double device_sum(const float *u, int64_t n, hipStream_t s);
double device_dot(const float *u, const float *v, int64_t n, hipStream_t s);
// out = s1 u + s2 v + cst  (v nullable)
void combine(const float *u, const float *v, int64_t n, double s1, double s2, double cst,
             float *out, hipStream_t s);

}  // namespace fs
