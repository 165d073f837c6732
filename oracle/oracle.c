/*
 * CPU oracle for radial-kernel summation, unbalanced Sinkhorn and MMD.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct FP64 reference that
 * the GPU library is checked against.  Only the tests, the smoke check and the benchmark's CPU
 * baseline may load it.  It shares no code, header, table or constant with the GPU library.
 *
 * Everything is written from the paper (Lakshmanan & Pichler, "Unbalanced Optimal Transport and
 * Maximum Mean Discrepancies: Interconnections and Rapid Evaluation", arXiv 2306.13618) in its own
 * notation:
 *   - measures  mu = sum_i mu_i delta_{x_i} (i < n),  nu = sum_j nu_j delta_{xt_j} (j < nt);
 *   - cost      d_ij^r with d the Euclidean distance (eq. (dist));
 *   - lam       the paper's lambda, an INVERSE temperature: the Gibbs kernel is k = exp(-lam d^r)
 *               and the entropy term carries 1/lam (Definition "entropy regularized UOT", eq. (W4)).
 *               Callers pass eps = 1/lam (the temperature); the code converts once.
 *   - eta       the marginal penalty, eta_1 = eta_2 = eta (Remark "hyperparameter tuning").
 *   - beta, gamma  the dual potentials (Theorem "dualization", eq. (dual_euot)).
 *
 * Kernels for fast summation and MMD (Table "prominent kernels", eq. (1492)), r = |x - y|:
 *   kind 0  Gauss    exp(-r^2 / ell2)     (ell2 = ell^2, passed as `lam_k`)
 *   kind 1  Laplace  exp(-r / ell)        (ell passed as `lam_k`)
 *   kind 2  energy   -r                    (lam_k unused)
 *   kind 3  IMQ      1 / sqrt(r^2 + c^2)  (c passed as `lam_k`)
 *
 * All sums use Neumaier (improved Kahan) compensated accumulation.
 * Parallelism is plain OpenMP over output rows; no blocking, fusion or reordering.
 *
 * Parity notes: every function here is pinned by CPU tests against closed forms, brute force in
 * extended precision, independent O(n log n) 1-D algorithms and invariants of the method.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- compensated sums */
typedef struct { double s, c; } nsum;
static inline void nadd(nsum *a, double v) {
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v; else a->c += (v - t) + a->s;
    a->s = t;
}
static inline double nval(const nsum *a) { return a->s + a->c; }

/* ---------------------------------------------------------------- distances and kernels */
static double dist(const double *p, const double *q, int d) {
    double s = 0.0;
    for (int k = 0; k < d; ++k) { double t = p[k] - q[k]; s += t * t; }
    return sqrt(s);
}

/* Radial kernels of Table "prominent kernels" (energy kernel with the table's minus sign). */
double orc_kernel(int kind, double lam_k, double r) {
    switch (kind) {
        case 0: return exp(-r * r / lam_k);
        case 1: return exp(-r / lam_k);
        case 2: return -r;
        case 3: return 1.0 / sqrt(r * r + lam_k * lam_k);
        default: return NAN;
    }
}

/* Gradient of the radial kernel K(y) with respect to y, at y = p - q.  Written out from the
 * kernel definitions: Gauss -2/ell2 y K, Laplace -(y/(ell |y|)) K, energy -y/|y| (0 at y = 0),
 * IMQ -y / (|y|^2 + c^2)^(3/2). */
static void kernel_grad(int kind, double lam_k, const double *p, const double *q, int d,
                        double *out) {
    double r = dist(p, q, d);
    for (int k = 0; k < d; ++k) {
        double y = p[k] - q[k];
        switch (kind) {
            case 0: out[k] = -2.0 / lam_k * y * exp(-r * r / lam_k); break;
            case 1: out[k] = (r > 0) ? -(y / (lam_k * r)) * exp(-r / lam_k) : 0.0; break;
            case 2: out[k] = (r > 0) ? -y / r : 0.0; break;
            case 3: out[k] = -y / pow(r * r + lam_k * lam_k, 1.5); break;
            default: out[k] = NAN;
        }
    }
}

/* ---------------------------------------------------------------- direct summation
 * eq. (fast_sum): s(x_i) = sum_j K(x_i - xt_j) alpha_j, evaluated directly in O(n nt d). */
void orc_direct_sum(const double *x, int64_t n, const double *y, int64_t m, int d,
                    const double *alpha, int kind, double lam_k, double *s) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        nsum acc = {0, 0};
        for (int64_t j = 0; j < m; ++j)
            nadd(&acc, orc_kernel(kind, lam_k, dist(x + i * d, y + j * d, d)) * alpha[j]);
        s[i] = nval(&acc);
    }
}

/* Same sum for a subset of rows (sampled checks at full problem size). */
void orc_direct_sum_rows(const double *x, const int64_t *rows, int64_t nrows, const double *y,
                         int64_t m, int d, const double *alpha, int kind, double lam_k,
                         double *s) {
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < nrows; ++t) {
        const double *xi = x + rows[t] * d;
        nsum acc = {0, 0};
        for (int64_t j = 0; j < m; ++j)
            nadd(&acc, orc_kernel(kind, lam_k, dist(xi, y + j * d, d)) * alpha[j]);
        s[t] = nval(&acc);
    }
}

/* Gradient of the direct sum with respect to the target position:
 * grad_x s(x_i) = sum_j (grad K)(x_i - xt_j) alpha_j.  Output (n x d). */
void orc_direct_sum_grad(const double *x, int64_t n, const double *y, int64_t m, int d,
                         const double *alpha, int kind, double lam_k, double *gs) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        nsum acc[64];
        double gk[64];
        for (int k = 0; k < d; ++k) acc[k].s = acc[k].c = 0.0;
        for (int64_t j = 0; j < m; ++j) {
            kernel_grad(kind, lam_k, x + i * d, y + j * d, d, gk);
            for (int k = 0; k < d; ++k) nadd(&acc[k], gk[k] * alpha[j]);
        }
        for (int k = 0; k < d; ++k) gs[i * d + k] = nval(&acc[k]);
    }
}

/* ---------------------------------------------------------------- unbalanced Sinkhorn
 * One half-step of the alternating maximisation, eq. (Sinkhorn_uot_iteration) / Algorithm 1:
 *     beta_i <- -(eta/(1+eta lam)) log( sum_j k_ij exp(lam gamma_j) nu_j ),  k_ij = exp(-lam d_ij^r).
 * The logarithm of the sum is evaluated as a log-sum-exp over j of
 *     -lam d_ij^r + lam gamma_j + log nu_j
 * (the same number, written so that it cannot overflow or underflow).
 * `src` are the points summed over (with weights w and potential pot), `dst` the points updated. */
static void half_step(const double *dst, int64_t nd, const double *src, const double *w,
                      const double *pot, int64_t ns, int d, int r, double lam, double eta,
                      double *out) {
    const double fac = eta / (1.0 + eta * lam);
#pragma omp parallel
    {
        double *e = (double *)malloc(sizeof(double) * (size_t)(ns > 0 ? ns : 1));
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < nd; ++i) {
            double mx = -INFINITY;
            for (int64_t j = 0; j < ns; ++j) {
                double dij = dist(dst + i * d, src + j * d, d);
                double c = (r == 2) ? dij * dij : dij;
                e[j] = -lam * c + lam * pot[j] + log(w[j]);
                if (e[j] > mx) mx = e[j];
            }
            nsum acc = {0, 0};
            for (int64_t j = 0; j < ns; ++j) nadd(&acc, exp(e[j] - mx));
            out[i] = -fac * (mx + log(nval(&acc)));
        }
        free(e);
    }
}

/* Algorithm 1 with a fixed number of half-steps.  Half-step Delta = 1, 3, ... updates beta
 * (Delta odd), Delta = 2, 4, ... updates gamma.  gamma holds the starting value on entry
 * (zero in the paper's default, gamma^(0) = 0).  eps = 1/lam is the temperature. */
void orc_uot_sinkhorn_halfsteps(const double *x, const double *mu, int64_t n, const double *y,
                                const double *nu, int64_t m, int d, int r, double eps,
                                double eta, int64_t nhalf, double *beta, double *gamma) {
    const double lam = 1.0 / eps;
    for (int64_t delta = 1; delta <= nhalf; ++delta) {
        if (delta % 2 == 1)
            half_step(x, n, y, nu, gamma, m, d, r, lam, eta, beta);
        else
            half_step(y, m, x, mu, beta, n, d, r, lam, eta, gamma);
    }
}

/* Full sweeps (beta then gamma) starting from gamma = 0, beta = 0. */
void orc_uot_sinkhorn(const double *x, const double *mu, int64_t n, const double *y,
                      const double *nu, int64_t m, int d, int r, double eps, double eta,
                      int64_t sweeps, double *beta, double *gamma) {
    for (int64_t i = 0; i < n; ++i) beta[i] = 0.0;
    for (int64_t j = 0; j < m; ++j) gamma[j] = 0.0;
    orc_uot_sinkhorn_halfsteps(x, mu, n, y, nu, m, d, r, eps, eta, 2 * sweeps, beta, gamma);
}

/* beta-half-step for selected rows only: beta_i from a given gamma (sampled full-size checks). */
void orc_uot_beta_rows(const double *x, const int64_t *rows, int64_t nrows, const double *y,
                       const double *nu, const double *gamma, int64_t m, int d, int r,
                       double eps, double eta, double *beta_rows) {
    double *xs = (double *)malloc(sizeof(double) * (size_t)(nrows * d + 1));
    for (int64_t t = 0; t < nrows; ++t)
        for (int k = 0; k < d; ++k) xs[t * d + k] = x[rows[t] * d + k];
    half_step(xs, nrows, y, nu, gamma, m, d, r, 1.0 / eps, eta, beta_rows);
    free(xs);
}

/* Dual function of Theorem "dualization" (eq. (dual_euot)), evaluated by its definition:
 *   D = -eta sum_i e^{-beta_i/eta} mu_i - eta sum_j e^{-gamma_j/eta} nu_j + eta sum mu + eta sum nu
 *       - (1/lam) sum_ij mu_i (e^{lam beta_i} e^{-lam d_ij^r} e^{lam gamma_j} - 1) nu_j.      */
double orc_uot_dual(const double *x, const double *mu, int64_t n, const double *y,
                    const double *nu, int64_t m, int d, int r, double eps, double eta,
                    const double *beta, const double *gamma) {
    const double lam = 1.0 / eps;
    nsum t1 = {0, 0};
    for (int64_t i = 0; i < n; ++i) nadd(&t1, -eta * exp(-beta[i] / eta) * mu[i] + eta * mu[i]);
    for (int64_t j = 0; j < m; ++j) nadd(&t1, -eta * exp(-gamma[j] / eta) * nu[j] + eta * nu[j]);
    double *rowsum = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        nsum acc = {0, 0};
        for (int64_t j = 0; j < m; ++j) {
            double dij = dist(x + i * d, y + j * d, d);
            double c = (r == 2) ? dij * dij : dij;
            nadd(&acc, mu[i] * (exp(lam * beta[i] - lam * c + lam * gamma[j]) - 1.0) * nu[j]);
        }
        rowsum[i] = nval(&acc);
    }
    nsum t2 = {0, 0};
    for (int64_t i = 0; i < n; ++i) nadd(&t2, rowsum[i]);
    free(rowsum);
    return nval(&t1) - nval(&t2) / lam;
}

/* Primal objective of the discrete problem (Section "Unbalanced optimal transport", discrete
 * form of eq. (W4)) at the plan pi = e^{lam beta} k e^{lam gamma} (mu x nu):
 *   sum d^r pi + (1/lam)(sum pi log(pi/(mu nu)) + sum mu nu - sum pi)
 *   + eta (sum_i P_i log(P_i/mu_i) + sum mu - sum P) + eta (sum_j Q_j log(Q_j/nu_j) + sum nu - sum Q)
 * with P = pi 1 and Q = pi^T 1.  O(n m); meant for small problems (duality-gap checks). */
double orc_uot_primal(const double *x, const double *mu, int64_t n, const double *y,
                      const double *nu, int64_t m, int d, int r, double eps, double eta,
                      const double *beta, const double *gamma) {
    const double lam = 1.0 / eps;
    double *P = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    double *Q = (double *)calloc((size_t)(m > 0 ? m : 1), sizeof(double));
    nsum cost = {0, 0}, ent = {0, 0};
    double Mmu = 0, Mnu = 0;
    for (int64_t i = 0; i < n; ++i) Mmu += mu[i];
    for (int64_t j = 0; j < m; ++j) Mnu += nu[j];
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < m; ++j) {
            double dij = dist(x + i * d, y + j * d, d);
            double c = (r == 2) ? dij * dij : dij;
            double logratio = lam * beta[i] - lam * c + lam * gamma[j]; /* log(pi_ij/(mu_i nu_j)) */
            double pij = mu[i] * nu[j] * exp(logratio);
            P[i] += pij;
            Q[j] += pij;
            nadd(&cost, c * pij);
            nadd(&ent, pij * logratio - pij);
        }
    }
    nsum mar1 = {0, 0}, mar2 = {0, 0};
    for (int64_t i = 0; i < n; ++i) nadd(&mar1, P[i] * log(P[i] / mu[i]) + mu[i] - P[i]);
    for (int64_t j = 0; j < m; ++j) nadd(&mar2, Q[j] * log(Q[j] / nu[j]) + nu[j] - Q[j]);
    free(P);
    free(Q);
    return nval(&cost) + (nval(&ent) + Mmu * Mnu) / lam + eta * nval(&mar1) + eta * nval(&mar2);
}

/* Marginals of the plan pi = e^{lam beta} k e^{lam gamma} (mu x nu): P = pi 1, Q = pi^T 1. */
void orc_uot_marginals(const double *x, const double *mu, int64_t n, const double *y,
                       const double *nu, int64_t m, int d, int r, double eps, const double *beta,
                       const double *gamma, double *P, double *Q) {
    const double lam = 1.0 / eps;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        nsum acc = {0, 0};
        for (int64_t j = 0; j < m; ++j) {
            double dij = dist(x + i * d, y + j * d, d);
            double c = (r == 2) ? dij * dij : dij;
            nadd(&acc, mu[i] * nu[j] * exp(lam * beta[i] - lam * c + lam * gamma[j]));
        }
        P[i] = nval(&acc);
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < m; ++j) {
        nsum acc = {0, 0};
        for (int64_t i = 0; i < n; ++i) {
            double dij = dist(x + i * d, y + j * d, d);
            double c = (r == 2) ? dij * dij : dij;
            nadd(&acc, mu[i] * nu[j] * exp(lam * beta[i] - lam * c + lam * gamma[j]));
        }
        Q[j] = nval(&acc);
    }
}

/* Optimal independent measure, Proposition "optimal independent measure", eq. (561):
 *   c* = exp(-<mu x nu, d^r> / (mu(X) nu(X) (eta1 + eta2 + 1/lam)))
 *        * mu(X)^(-eta2/(eta1+eta2+1/lam)) * nu(X)^(-eta1/(eta1+eta2+1/lam)),
 * with eta1 = eta2 = eta.  Also returns the primal objective at pi = c* mu x nu, an upper bound on
 * the regularised UOT value (Remark "upper bounds"). */
double orc_uot_cstar(const double *x, const double *mu, int64_t n, const double *y,
                     const double *nu, int64_t m, int d, int r, double eps, double eta,
                     double *upper_bound) {
    const double lam = 1.0 / eps;
    nsum cc = {0, 0};
    double Mmu = 0, Mnu = 0;
    for (int64_t i = 0; i < n; ++i) Mmu += mu[i];
    for (int64_t j = 0; j < m; ++j) Mnu += nu[j];
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < m; ++j) {
            double dij = dist(x + i * d, y + j * d, d);
            nadd(&cc, mu[i] * nu[j] * ((r == 2) ? dij * dij : dij));
        }
    const double s = 2.0 * eta + 1.0 / lam;
    const double cstar = exp(-nval(&cc) / (Mmu * Mnu * s)) * pow(Mmu, -eta / s) * pow(Mnu, -eta / s);
    if (upper_bound) {
        /* objective at pi = c mu x nu: c<mu x nu,d^r> + (1/lam) Mmu Mnu (c log c - c + 1)
         * + eta Mmu (c Mnu log(c Mnu) - c Mnu + 1) + eta Mnu (c Mmu log(c Mmu) - c Mmu + 1) */
        const double c = cstar;
        *upper_bound = c * nval(&cc) + Mmu * Mnu * (c * log(c) - c + 1.0) / lam +
                       eta * Mmu * (c * Mnu * log(c * Mnu) - c * Mnu + 1.0) +
                       eta * Mnu * (c * Mmu * log(c * Mmu) - c * Mmu + 1.0);
    }
    return cstar;
}

/* Sinkhorn divergence, eq. (586):
 *   sd = UOT(mu,nu) - 1/2 UOT(mu,mu) - 1/2 UOT(nu,nu) + (1/(2 lam)) (mu(X) - nu(X))^2,
 * each UOT value taken as the dual value after `sweeps` full sweeps (strong duality). */
double orc_sinkhorn_divergence(const double *x, const double *mu, int64_t n, const double *y,
                               const double *nu, int64_t m, int d, int r, double eps,
                               double eta, int64_t sweeps, double *terms3) {
    double *bx = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    double *gx = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    double *by = (double *)malloc(sizeof(double) * (size_t)(m + 1));
    double *gy = (double *)malloc(sizeof(double) * (size_t)(m + 1));
    orc_uot_sinkhorn(x, mu, n, y, nu, m, d, r, eps, eta, sweeps, bx, gy);
    double uxy = orc_uot_dual(x, mu, n, y, nu, m, d, r, eps, eta, bx, gy);
    orc_uot_sinkhorn(x, mu, n, x, mu, n, d, r, eps, eta, sweeps, bx, gx);
    double uxx = orc_uot_dual(x, mu, n, x, mu, n, d, r, eps, eta, bx, gx);
    orc_uot_sinkhorn(y, nu, m, y, nu, m, d, r, eps, eta, sweeps, by, gy);
    double uyy = orc_uot_dual(y, nu, m, y, nu, m, d, r, eps, eta, by, gy);
    double Mmu = 0, Mnu = 0;
    for (int64_t i = 0; i < n; ++i) Mmu += mu[i];
    for (int64_t j = 0; j < m; ++j) Mnu += nu[j];
    free(bx); free(gx); free(by); free(gy);
    if (terms3) { terms3[0] = uxy; terms3[1] = uxx; terms3[2] = uyy; }
    return uxy - 0.5 * uxx - 0.5 * uyy + 0.5 * eps * (Mmu - Mnu) * (Mmu - Mnu);
}

/* Envelope gradients of the dual value at given potentials (derivatives of eq. (dual_euot) with
 * the potentials held fixed, which equal the derivatives of the optimal value at the optimum):
 *   dD/dx_i  = sum_j pi_ij grad_x d^r(x_i, xt_j)
 *   dD/dmu_i = eta (1 - e^{-beta_i/eta}) - (1/lam) sum_j (e^{lam(beta_i + gamma_j - d_ij^r)} - 1) nu_j
 * and symmetrically for xt_j, nu_j.  grad of d^r: r=2 -> 2(x-y); r=1 -> (x-y)/|x-y| (0 at 0). */
void orc_uot_grad(const double *x, const double *mu, int64_t n, const double *y,
                  const double *nu, int64_t m, int d, int r, double eps, double eta,
                  const double *beta, const double *gamma, double *dx, double *dmu, double *dy,
                  double *dnu) {
    const double lam = 1.0 / eps;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        nsum g[64], s = {0, 0};
        for (int k = 0; k < d; ++k) g[k].s = g[k].c = 0;
        for (int64_t j = 0; j < m; ++j) {
            double dij = dist(x + i * d, y + j * d, d);
            double c = (r == 2) ? dij * dij : dij;
            double e = exp(lam * (beta[i] + gamma[j] - c));
            double pij = mu[i] * nu[j] * e;
            for (int k = 0; k < d; ++k) {
                double diff = x[i * d + k] - y[j * d + k];
                double gc = (r == 2) ? 2.0 * diff : (dij > 0 ? diff / dij : 0.0);
                nadd(&g[k], pij * gc);
            }
            nadd(&s, (e - 1.0) * nu[j]);
        }
        for (int k = 0; k < d; ++k) dx[i * d + k] = nval(&g[k]);
        dmu[i] = eta * (1.0 - exp(-beta[i] / eta)) - nval(&s) / lam;
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < m; ++j) {
        nsum g[64], s = {0, 0};
        for (int k = 0; k < d; ++k) g[k].s = g[k].c = 0;
        for (int64_t i = 0; i < n; ++i) {
            double dij = dist(x + i * d, y + j * d, d);
            double c = (r == 2) ? dij * dij : dij;
            double e = exp(lam * (beta[i] + gamma[j] - c));
            double pij = mu[i] * nu[j] * e;
            for (int k = 0; k < d; ++k) {
                double diff = y[j * d + k] - x[i * d + k];
                double gc = (r == 2) ? 2.0 * diff : (dij > 0 ? diff / dij : 0.0);
                nadd(&g[k], pij * gc);
            }
            nadd(&s, (e - 1.0) * mu[i]);
        }
        for (int k = 0; k < d; ++k) dy[j * d + k] = nval(&g[k]);
        dnu[j] = eta * (1.0 - exp(-gamma[j] / eta)) - nval(&s) / lam;
    }
}

/* Envelope gradient rows (as orc_uot_grad, first slot only) for selected rows of x. */
void orc_uot_grad_rows(const double *x, const double *mu, const int64_t *rows, int64_t nrows,
                       const double *y, const double *nu, int64_t m, int d, int r, double eps,
                       double eta, const double *beta, const double *gamma, double *dx,
                       double *dmu) {
    const double lam = 1.0 / eps;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < nrows; ++t) {
        const int64_t i = rows[t];
        nsum g[64], s = {0, 0};
        for (int k = 0; k < d; ++k) g[k].s = g[k].c = 0;
        for (int64_t j = 0; j < m; ++j) {
            double dij = dist(x + i * d, y + j * d, d);
            double c = (r == 2) ? dij * dij : dij;
            double e = exp(lam * (beta[i] + gamma[j] - c));
            double pij = mu[i] * nu[j] * e;
            for (int k = 0; k < d; ++k) {
                double diff = x[i * d + k] - y[j * d + k];
                double gc = (r == 2) ? 2.0 * diff : (dij > 0 ? diff / dij : 0.0);
                nadd(&g[k], pij * gc);
            }
            nadd(&s, (e - 1.0) * nu[j]);
        }
        for (int k = 0; k < d; ++k) dx[t * d + k] = nval(&g[k]);
        dmu[t] = eta * (1.0 - exp(-beta[i] / eta)) - nval(&s) / lam;
    }
}

/* ---------------------------------------------------------------- MMD
 * eq. (1205): MMD^2 = sum_ij mu_i mu_j k(x_i,x_j) - 2 sum_ij mu_i nu_j k(x_i,xt_j)
 *                     + sum_ij nu_i nu_j k(xt_i,xt_j)   (diagonal included; signed for the
 * energy kernel, which is only conditionally positive definite).  terms3 receives the three
 * double sums (without the factor -2). */
double orc_mmd2(const double *x, const double *mu, int64_t n, const double *y, const double *nu,
                int64_t m, int d, int kind, double lam_k, double *terms3) {
    double *s = (double *)malloc(sizeof(double) * (size_t)((n > m ? n : m) + 1));
    double t[3];
    nsum acc;
    orc_direct_sum(x, n, x, n, d, mu, kind, lam_k, s);
    acc.s = acc.c = 0; for (int64_t i = 0; i < n; ++i) nadd(&acc, mu[i] * s[i]); t[0] = nval(&acc);
    orc_direct_sum(x, n, y, m, d, nu, kind, lam_k, s);
    acc.s = acc.c = 0; for (int64_t i = 0; i < n; ++i) nadd(&acc, mu[i] * s[i]); t[1] = nval(&acc);
    orc_direct_sum(y, m, y, m, d, nu, kind, lam_k, s);
    acc.s = acc.c = 0; for (int64_t j = 0; j < m; ++j) nadd(&acc, nu[j] * s[j]); t[2] = nval(&acc);
    free(s);
    if (terms3) { terms3[0] = t[0]; terms3[1] = t[1]; terms3[2] = t[2]; }
    return t[0] - 2.0 * t[1] + t[2];
}

/* Gradients of eq. (1205), differentiated term by term:
 *   dMMD2/dx_i  = 2 mu_i [sum_j mu_j gradK(x_i - x_j) - sum_j nu_j gradK(x_i - xt_j)]
 *   dMMD2/dmu_i = 2 [sum_j mu_j K(x_i - x_j) - sum_j nu_j K(x_i - xt_j)]
 * and with the roles exchanged for xt, nu. */
void orc_mmd2_grad(const double *x, const double *mu, int64_t n, const double *y,
                   const double *nu, int64_t m, int d, int kind, double lam_k, double *dx,
                   double *dmu, double *dy, double *dnu) {
    double *g1 = (double *)malloc(sizeof(double) * (size_t)((n > m ? n : m) * d + 1));
    double *g2 = (double *)malloc(sizeof(double) * (size_t)((n > m ? n : m) * d + 1));
    double *s1 = (double *)malloc(sizeof(double) * (size_t)((n > m ? n : m) + 1));
    double *s2 = (double *)malloc(sizeof(double) * (size_t)((n > m ? n : m) + 1));
    orc_direct_sum_grad(x, n, x, n, d, mu, kind, lam_k, g1);
    orc_direct_sum_grad(x, n, y, m, d, nu, kind, lam_k, g2);
    orc_direct_sum(x, n, x, n, d, mu, kind, lam_k, s1);
    orc_direct_sum(x, n, y, m, d, nu, kind, lam_k, s2);
    for (int64_t i = 0; i < n; ++i) {
        for (int k = 0; k < d; ++k) dx[i * d + k] = 2.0 * mu[i] * (g1[i * d + k] - g2[i * d + k]);
        dmu[i] = 2.0 * (s1[i] - s2[i]);
    }
    orc_direct_sum_grad(y, m, y, m, d, nu, kind, lam_k, g1);
    orc_direct_sum_grad(y, m, x, n, d, mu, kind, lam_k, g2);
    orc_direct_sum(y, m, y, m, d, nu, kind, lam_k, s1);
    orc_direct_sum(y, m, x, n, d, mu, kind, lam_k, s2);
    for (int64_t j = 0; j < m; ++j) {
        for (int k = 0; k < d; ++k) dy[j * d + k] = 2.0 * nu[j] * (g1[j * d + k] - g2[j * d + k]);
        dnu[j] = 2.0 * (s1[j] - s2[j]);
    }
    free(g1); free(g2); free(s1); free(s2);
}

/* Gradient rows of eq. (1205) for selected rows of x (first measure):
 *   dx_i = 2 mu_i [sum_j mu_j gradK(x_i - x_j) - sum_j nu_j gradK(x_i - xt_j)],
 *   dmu_i = 2 [sum_j mu_j K(x_i - x_j) - sum_j nu_j K(x_i - xt_j)]. */
void orc_mmd2_grad_rows(const double *x, const double *mu, int64_t n, const int64_t *rows,
                        int64_t nrows, const double *y, const double *nu, int64_t m, int d,
                        int kind, double lam_k, double *dx, double *dmu) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < nrows; ++t) {
        const int64_t i = rows[t];
        nsum g[64], s = {0, 0};
        double gk[64];
        for (int k = 0; k < d; ++k) g[k].s = g[k].c = 0;
        for (int64_t j = 0; j < n; ++j) {
            kernel_grad(kind, lam_k, x + i * d, x + j * d, d, gk);
            for (int k = 0; k < d; ++k) nadd(&g[k], gk[k] * mu[j]);
            nadd(&s, orc_kernel(kind, lam_k, dist(x + i * d, x + j * d, d)) * mu[j]);
        }
        for (int64_t j = 0; j < m; ++j) {
            kernel_grad(kind, lam_k, x + i * d, y + j * d, d, gk);
            for (int k = 0; k < d; ++k) nadd(&g[k], -gk[k] * nu[j]);
            nadd(&s, -orc_kernel(kind, lam_k, dist(x + i * d, y + j * d, d)) * nu[j]);
        }
        for (int k = 0; k < d; ++k) dx[t * d + k] = 2.0 * mu[i] * nval(&g[k]);
        dmu[t] = 2.0 * nval(&s);
    }
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
