/*
 * fastuot: fast radial-kernel summation on one MI355X (gfx950), and the unbalanced Sinkhorn and
 * MMD computations built on it.
 *
 * Method: Lakshmanan & Pichler, "Unbalanced Optimal Transport and Maximum Mean Discrepancies:
 * Interconnections and Rapid Evaluation" (arXiv 2306.13618).  The product computed everywhere is
 * the kernel sum of eq. (fast_sum),
 *        s_i = sum_j K(x_i - y_j) v_j,    K radial,
 * evaluated either directly (O(n m)) or by NFFT fast summation (eq. (1724), Section "NFFT fast
 * summation"): spreading of the weighted source nodes onto an oversampled grid with a
 * Kaiser-Bessel window, an FFT, a pointwise product with the kernel's Fourier coefficients b_k,
 * an inverse FFT and an interpolation (gather) at the target nodes, plus a near-field correction
 * for the kernels that are not smooth at the origin.
 *
 * Conventions for every entry point
 * ---------------------------------
 *  - Array arguments are DEVICE pointers owned by the caller (HIP device memory, e.g. the data of
 *    torch tensors), contiguous, row-major.  Points are float32 (count x d); weights float32;
 *    dual potentials float64.  Outputs are preallocated by the caller.  Scalars written to
 *    `*_host` pointers are host memory.
 *  - `stream` is a hipStream_t (may be NULL for the default stream).  Work is enqueued on it;
 *    calls that return a host scalar, fastsum_apply and plan creation synchronise that stream;
 *    fs_plan_apply does not (it is stream-ordered: its temporaries are reused only after the
 *    stream has passed them).
 *  - The library allocates its own workspace (device memory) and keeps freed blocks in a cache
 *    for reuse until fs_release_cache() or process exit.  Calls are not thread-safe.
 *  - Return value: FS_OK (0) on success, a negative fs_status on failure; fs_last_error() then
 *    describes the failure.  Outputs are unspecified after a failure.
 *  - Interface choices: the kernel kind and width, which the problem statement passes as a
 *    separate kernel argument, are fields of fs_params with the grid settings; fs_plan_apply
 *    takes the stream it enqueues on (a plan may be applied on a stream other than the one it
 *    was created on).
 *  - Parameters use the temperature convention: the Gibbs kernel of the transport cost |x-y|^r is
 *    exp(-|x-y|^r / lambda), i.e. lambda here is the reciprocal of the paper's lambda (the paper
 *    writes exp(-lambda d^r) with an inverse temperature, eq. (W4)).  rho is the paper's marginal
 *    penalty eta (eta_1 = eta_2 = rho, Remark "hyperparameter tuning").
 */
#ifndef FASTUOT_H
#define FASTUOT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FS_OK = 0,
    FS_EINVAL = -1,       /* bad argument (size, pointer, parameter out of range)           */
    FS_EDOMAIN = -2,      /* points cannot be mapped into the torus / d unsupported          */
    FS_ENOMEM = -3,       /* device allocation failed                                       */
    FS_EHIP = -4,         /* a HIP runtime call or kernel launch failed                      */
    FS_ENUMERIC = -5,     /* a kernel sum that must be positive was not (log of <= 0)        */
    FS_EUNSUPPORTED = -6  /* combination not implemented                                     */
} fs_status;

/* Radial kernels (Table "prominent kernels" and eq. (1492)), r = |x - y| */
enum {
    FS_GAUSS = 0,   /* exp(-r^2 / lambda)  (lambda = ell^2 of the table)      */
    FS_LAPLACE = 1, /* exp(-r / lambda)    (lambda = ell of the table)        */
    FS_ENERGY = 2,  /* -r                  (lambda unused)                    */
    FS_IMQ = 3      /* 1 / sqrt(r^2 + c^2) (lambda = c of the table)          */
};

/* flags */
#define FS_FLAG_WARM_START 0x1u   /* uot_sinkhorn: f and g hold starting potentials on entry     */
#define FS_FLAG_FORCE_VALU 0x2u   /* use the FP32 VALU kernels even where matrix-core ones apply */
#define FS_FLAG_DETERMINISTIC 0x4u /* bitwise reproducible results: nodes that share a grid cell
                                      or a near-field cell keep their input order (stable sorts in
                                      the plan build), and the near field adds no partial sums
                                      through atomics; costs a radix sort per point set */

/* Parameters of one kernel sum.  Zero-initialise and set what you need; zeros mean defaults. */
typedef struct fs_params {
    int kernel;              /* FS_GAUSS, FS_LAPLACE, FS_ENERGY or FS_IMQ                         */
    int grid;                /* oversampled FFT grid points per dimension (even, 16..512);
                                0 selects direct summation                                         */
    int window;              /* Kaiser-Bessel window cutoff m: support 2m grid points per dim,
                                2..8 (0 -> 6)                                                      */
    int oversampling;        /* sigma = grid / bandwidth N, integer >= 2 (0 -> 2); see bandwidth  */
    int smoothness;          /* p: derivatives matched by the regularisation polynomials (0 -> 8) */
    unsigned flags;          /* FS_FLAG_*                                                         */
    double lambda;           /* kernel width (see the kernel list); > 0 for Gauss, Laplace, IMQ   */
    double nearfield_radius; /* Laplace/energy/IMQ: radius (data units) inside which the kernel is
                                summed directly; 0 -> smoothness / bandwidth in torus units        */
    int bandwidth;           /* N, the trigonometric polynomial's bandwidth (even, <= grid - 2);
                                0 -> grid / oversampling.  Overrides oversampling when set; the
                                window shape follows the effective ratio grid / N.                 */
} fs_params;

/* Opaque plan: two point sets mapped to the torus, binned by grid tile, and the kernel's
 * Fourier multiplier.  Holds device workspace until fs_plan_destroy. */
typedef struct fs_plan_s *fs_plan;

/* Message for the last non-OK status returned on this thread ("" if none). */
const char *fs_last_error(void);

/* Library version, (major << 16) | minor. */
int fs_version(void);

/* Release the cached device memory of the calling process: workspace blocks and the multipliers
 * kept from recent plans (the latter after a device synchronisation). */
void fs_release_cache(void);

/* Pass timing (instrumentation, not part of the method).  fs_profile_enable(1) makes every
 * subsequent launch of the named passes ("spread", "fold", "fft", "gather", "nearfield",
 * "update", "direct") record a pair of HIP events on the stream the pass is launched on;
 * fs_profile_query waits for the recorded events and returns the summed duration in
 * milliseconds and the launch count for one pass name (0 and 0 if none); fs_profile_reset
 * discards the records.  fs_profile_select(pass, period) restricts the recording to the passes
 * named `pass` (NULL or "": all) and to every period-th of them (period >= 1; sampling keeps the
 * events' own cost out of a timed run); it restarts the count.  Returns FS_OK or FS_EINVAL (NULL
 * argument, period < 1). */
int fs_profile_enable(int enable);
int fs_profile_select(const char *pass, int period);
int fs_profile_query(const char *pass, double *total_ms, int64_t *count);
void fs_profile_reset(void);

/* Kernel sum, eq. (fast_sum):  out_i = sum_j K(x_i - y_j) v_j,  i < n, j < m.
 *   x (n x d), y (m x d), v (m), out (n): device, float32.  d in 1..3 for the fast path
 *   (Section "Curse of dimensionality": the method is restricted to d <= 3); any d in 1..128 for
 *   direct summation (grid = 0), where a Gaussian kernel with d a multiple of 16 forms the
 *   exponent on the matrix cores (centred coordinates as FP16 hi/lo split products accumulated
 *   in FP32) when the exponent scale (log2 e / lambda) (R_x + R_y)^2 (R: largest centred norm of
 *   a set) is at most 64, where that arithmetic stays within 1e-5, and the FP32 VALU kernel
 *   otherwise or with FS_FLAG_FORCE_VALU.  In 2-D and 3-D the fast path spreads onto and
 *   interpolates from the grid with FP16 matrix-core products of split operands (hi + lo, about
 *   22 significant bits, summed in FP32; within 2e-6 of the FP32 VALU kernels) where the nodes
 *   fill groups of up to 16 per brick of 4 cells (unless FS_FLAG_FORCE_VALU).
 *   n = 0 or m = 0 is valid (out is zero-filled when m = 0). */
int fastsum_apply(const float *x, int64_t n, const float *y, int64_t m, int d, const float *v,
                  float *out, const fs_params *p, void *stream);

/* Plans: fs_plan_create maps x (targets) and y (sources) to the torus and bins them (the plan
 * keeps copies; the caller may free x and y afterwards).  fs_plan_apply computes
 *   transpose = 0:  out (n) = K_xy v,  v of length m
 *   transpose = 1:  out (m) = K_yx v,  v of length n
 * with K symmetric (radial), so the transpose is the same operator with the roles swapped.
 * fs_plan_apply is stream-ordered and returns without waiting; a plan holds scratch buffers, so
 * applications of one plan must be ordered (one stream, or synchronised between streams).
 * fs_plan_destroy waits for the device before releasing the plan.  A 3-D plan whose window
 * segments' Chebyshev transform (the 3-D spread's moment form) would leave FP16 range fails with
 * FS_EUNSUPPORTED; the Kaiser-Bessel windows built here stay well inside it. */
int fs_plan_create(const float *x, int64_t n, const float *y, int64_t m, int d,
                   const fs_params *p, void *stream, fs_plan *plan_out);
int fs_plan_apply(fs_plan plan, const float *v, float *out, int transpose, void *stream);
void fs_plan_destroy(fs_plan plan);

/* Inspection of a fast-summation plan (eq. (ansatz_NFFT)): the Fourier multiplier applied
 * between the forward and the inverse transform,
 *   M_k = b_k / (G^2 phihat(k_1)^2 ... phihat(k_d)^2) x (1/2 per coordinate with |k_i| = N/2),
 *   b_k = N^-d sum_{j in I_N} K_R(j/N) e^{-2 pi i j.k/N}  (real and even),
 * for k in [0, N/2]^d (first coordinate fastest; the values at negative k are the same), as
 * float32 into mult_host (count >= (N/2+1)^d), the window transform phihat(k), k = 0..N/2, into
 * phihat_host (float64, N/2+1 values), the torus period in data units (torus coordinates are
 * data coordinates divided by it) and N.  Host pointers; any may be NULL except that count must
 * cover the multiplier.  Synchronises the stream.  FS_EINVAL for a direct-summation plan. */
int fs_plan_multiplier(fs_plan plan, float *mult_host, double *phihat_host, int64_t count,
                       double *period_host, int *bandwidth_host, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): fs_plan_apply with no allocation of any kind.  Same
 * arguments, result and kernels as fs_plan_apply; its temporaries (the operator-order weights
 * and sums of the fast path, the partial row sums of the direct matrix-core path) live in a
 * static 16 MiB device array, one copy per GPU, held until the process ends.  Limit: on the fast
 * path 4 (ns + 1) + 4 (nt + 1) bytes, each rounded up to 256, must fit (about 4.19 million
 * source plus target points); larger plans return FS_EINVAL with a message, and nothing is
 * launched.  On the direct matrix-core path the array bounds the column splits instead (no
 * size limit).  Every call on one GPU shares that GPU's array: calls that overlap on one GPU
 * (other streams or threads) race and must be ordered by the caller.  The calling thread's
 * current device must be the stream's device.  Pass timing (fs_profile_enable) creates events
 * and should stay off in such callers. */
int fs_plan_apply_noalloc(fs_plan plan, const float *v, float *out, int transpose,
                          void *stream);

/* Unbalanced Sinkhorn, Algorithm 2 (the NFFT-accelerated form of Algorithm 1):
 *   iters full sweeps; each sweep does the beta half-step then the gamma half-step,
 *     f_i = -(rho lambda/(rho + lambda)) log sum_j k_ij b_j exp(g_j/lambda)
 *     g_j = -(rho lambda/(rho + lambda)) log sum_i k_ij a_i exp(f_i/lambda)
 *   with k_ij = exp(-|x_i - y_j|^r / lambda), r = 2 for FS_GAUSS and r = 1 for FS_LAPLACE
 *   (eq. (Sinkhorn_uot_iteration) with the paper's lambda replaced by 1/lambda).
 *   Starts from g = 0 (f = 0) unless FS_FLAG_WARM_START.  a (n), b (m): nonnegative weights.
 *   f (n), g (m): device float64, the potentials beta and gamma of the paper.
 *   objective_host (nullable): the dual value of Theorem "dualization" at (f, g), summed in FP64
 *   with compensation.  The kernel sums run in FP32, the potential updates in FP64. */
int uot_sinkhorn(const float *x, const float *a, int64_t n, const float *y, const float *b,
                 int64_t m, int d, const fs_params *p, double rho, int iters, double *f, double *g,
                 double *objective_host, void *stream);

/* Upper bound of Proposition "Optimal independent measure" and the remark on upper bounds:
 *   c* = exp(-<mu x nu, d^r> / (Ma Mb (2 rho + lambda))) Ma^(-rho/(2 rho + lambda))
 *        Mb^(-rho/(2 rho + lambda))                          (eq. (561), eta_1 = eta_2 = rho)
 *   bound = objective of eq. (W4) at pi = c* mu x nu  >=  UOT_lambda(mu, nu),
 * with Ma, Mb the masses and r = 2 (FS_GAUSS) or 1 (FS_LAPLACE).  For r = 2, <mu x nu, d^2>
 * comes from FP64 first and second moments; for r = 1 it is one energy-kernel sum with the grid,
 * window and near-field settings of p (direct when grid = 0).  cstar_host and bound_host are
 * host doubles (nullable).  Synchronises the stream. */
int uot_upper_bound(const float *x, const float *a, int64_t n, const float *y, const float *b,
                    int64_t m, int d, const fs_params *p, double rho, double *cstar_host,
                    double *bound_host, void *stream);

/* Starting potentials of uot_sinkhorn_scaling */
#define FS_INIT_ZERO 0  /* g = 0                                                           */
#define FS_INIT_CSTAR 1 /* g = lambda_0 log c*, c* of eq. (561) at the first temperature,
                           f = 0 (the remark on initialisation, read as e^{g/lambda} = c*) */
#define FS_INIT_WARM 2  /* f and g hold the starting potentials on entry                  */

/* lambda-scaling (Section "lambda-scaling"): the problem of uot_sinkhorn solved for the
 * temperatures eps_stages[0..nstages) in turn (p->lambda is ignored), each stage warm-started
 * from the potentials of the previous one.  A stage ends after the first sweep that changes no
 * potential by more than tol * eps_stages[k] (the potentials enter the kernel sums as
 * exp(f / eps); tol = 0 runs max_sweeps sweeps), or after max_sweeps sweeps.  The FP32 kernel
 * sums leave a floor of about 1e-7 in this measure: use tol >= 1e-6.  Each stage builds its own plan (the torus period follows the temperature).
 * sweeps_host (nullable, nstages ints) receives the sweeps run per stage; objective_host
 * (nullable) the dual value at the last temperature.  f (n), g (m): device float64. */
int uot_sinkhorn_scaling(const float *x, const float *a, int64_t n, const float *y, const float *b,
                         int64_t m, int d, const fs_params *p, const double *eps_stages,
                         int nstages, double rho, int max_sweeps, double tol, int init, double *f,
                         double *g, int *sweeps_host, double *objective_host, void *stream);

/* Gradients of the UOT value at converged potentials (envelope theorem on the dual of Theorem
 * "dualization"), scaled by `scale`:
 *   dx_i = scale * sum_j pi_ij grad_x |x_i - y_j|^r,    pi_ij = a_i b_j exp((f_i + g_j - C_ij)/lambda)
 *   da_i = scale * (rho (1 - exp(-f_i/rho)) - lambda sum_j b_j (exp((f_i + g_j - C_ij)/lambda) - 1))
 *   and symmetrically dy, db.  Any of dx, da, dy, db may be NULL (not computed).  float32 outputs. */
int uot_sinkhorn_grad(const float *x, const float *a, int64_t n, const float *y, const float *b,
                      int64_t m, int d, const fs_params *p, double rho, const double *f,
                      const double *g, double scale, float *dx, float *da, float *dy, float *db,
                      void *stream);

/* Sinkhorn divergence, eq. (586):
 *   S = UOT(a,b) - UOT(a,a)/2 - UOT(b,b)/2 + (lambda/2) (sum a - sum b)^2,
 *   each UOT value the dual value after `iters` sweeps.  Potentials of the three problems are
 *   written to f_ab (n), g_ab (m), f_aa (n), f_bb (m) (device float64; each may be NULL) for the
 *   backward pass; terms3_host (nullable) receives the three UOT values.  The three problems are
 *   independent and run side by side: UOT(a,b) on `stream`, the self terms on two streams the
 *   library keeps per device (default priority) from host threads of its own, all ordered after
 *   the work already queued on `stream`.  The call returns when all three have finished; an error
 *   in any of them is returned with its message. */
int sinkhorn_divergence(const float *x, const float *a, int64_t n, const float *y, const float *b,
                        int64_t m, int d, const fs_params *p, double rho, int iters,
                        double *f_ab, double *g_ab, double *f_aa, double *f_bb,
                        double *value_host, double *terms3_host, void *stream);

/* Gradient of the Sinkhorn divergence from the potentials written by sinkhorn_divergence
 * (the symmetric problems contribute twice their one-slot envelope gradient), scaled by `scale`.
 * The envelope gradients run side by side as the three problems do in sinkhorn_divergence
 * (the (a,b) term's two sides and the two self terms, on `stream` and three library streams);
 * the call returns when the gradients are written. */
int sinkhorn_divergence_grad(const float *x, const float *a, int64_t n, const float *y,
                             const float *b, int64_t m, int d, const fs_params *p, double rho,
                             const double *f_ab, const double *g_ab, const double *f_aa,
                             const double *f_bb, double scale, float *dx, float *da, float *dy,
                             float *db, void *stream);

/* Squared MMD, eq. (1205), as one kernel sum on the union z = (x, y) with weights w = (a, -b):
 *   MMD^2 = sum_ij w_i w_j K(z_i - z_j)   (V-statistic, diagonal included; signed for the
 *   energy kernel, which is only conditionally positive definite).  The final dot product is
 *   summed in FP64 with compensation.  terms3_host (nullable) receives sum a a K, sum a b K,
 *   sum b b K computed from the same kernel sum. */
int mmd(const float *x, const float *a, int64_t n, const float *y, const float *b, int64_t m,
        int d, const fs_params *p, double *mmd2_host, double *terms3_host, void *stream);

/* Gradient of MMD^2, scaled by `scale`:
 *   dx_i = 2 scale a_i [sum_j a_j gradK(x_i - x_j) - sum_j b_j gradK(x_i - y_j)],
 *   da_i = 2 scale [sum_j a_j K(x_i - x_j) - sum_j b_j K(x_i - y_j)], and symmetrically for y, b
 *   (with the sign of b).  Any output may be NULL.  float32 outputs. */
int mmd_grad(const float *x, const float *a, int64_t n, const float *y, const float *b, int64_t m,
             int d, const fs_params *p, double scale, float *dx, float *da, float *dy, float *db,
             void *stream);

#ifdef __cplusplus
}
#endif

#endif /* FASTUOT_H */
