"""Pins of the FP64 CPU oracle against what the paper and mathematics fix (CPU only).

Each test checks the oracle against something other than itself: extended-precision brute force,
an independent O(n log n) algorithm, a closed form, or an invariant of the method.  The tests are
chosen so that a dropped term, a wrong sign, a wrong factor or a transposed operand in the oracle
fails at least one of them.
"""
import json
import math
import os

import mpmath as mp
import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


# --------------------------------------------------------------------------- direct sums

def _mp_kernel(kind, lam, r):
    if kind == "gauss":
        return mp.e ** (-r * r / lam)
    if kind == "laplace":
        return mp.e ** (-r / lam)
    if kind == "imq":
        return 1 / mp.sqrt(r * r + lam * lam)
    return -r


@pytest.mark.parametrize("kind,lam", [("gauss", 0.02), ("laplace", 0.05), ("energy", 0.0),
                                      ("imq", 0.3), ("imq", 0.01)])
@pytest.mark.parametrize("d", [1, 2, 3])
def test_direct_sum_vs_mpmath_bruteforce(kind, lam, d):
    """eq. (fast_sum) evaluated in 40-digit arithmetic on n, m <= 24."""
    rng = np.random.default_rng([7, d])
    x = rng.uniform(-0.25, 0.25, (17, d))
    y = rng.uniform(-0.25, 0.25, (23, d))
    v = rng.uniform(-1, 1, 23)
    got = oracle.direct_sum(x, y, v, kind, lam if lam else 1.0)
    mp.mp.dps = 40
    ref = []
    for i in range(len(x)):
        acc = mp.mpf(0)
        for j in range(len(y)):
            r = mp.sqrt(sum((mp.mpf(float(x[i, k])) - mp.mpf(float(y[j, k]))) ** 2 for k in range(d)))
            acc += _mp_kernel(kind, lam if lam else 1.0, r) * mp.mpf(float(v[j]))
        ref.append(float(acc))
    assert rel(got, ref) < 1e-13


@pytest.mark.parametrize("c", [0.05, 0.5])
def test_direct_sum_imq_as_gaussian_scale_mixture(c):
    """IMQ through the Gaussian kernel: 1/sqrt(r^2 + c^2) = (2/sqrt(pi)) int_0^inf e^{-u^2 c^2}
    e^{-u^2 r^2} du, so the IMQ sum is a quadrature over Gaussian sums (lambda = 1/u^2) that the
    oracle evaluates through its independently pinned Gaussian kernel."""
    from scipy.integrate import quad_vec
    rng = np.random.default_rng([8, int(100 * c)])
    x = rng.uniform(-0.25, 0.25, (15, 3))
    y = rng.uniform(-0.25, 0.25, (21, 3))
    v = rng.uniform(-1, 1, 21)

    def f(t):  # u = t / (1 - t) maps [0, 1) onto [0, inf)
        if t <= 0.0:
            return np.zeros(len(x))
        if t >= 1.0:
            return np.zeros(len(x))
        u = t / (1.0 - t)
        return (2 / math.sqrt(math.pi)) * math.exp(-u * u * c * c) * \
            oracle.direct_sum(x, y, v, "gauss", 1.0 / (u * u)) / (1.0 - t) ** 2

    ref, _ = quad_vec(f, 0.0, 1.0, epsabs=1e-13, epsrel=1e-12)
    got = oracle.direct_sum(x, y, v, "imq", c)
    assert rel(got, ref) < 1e-9


def _laplace_1d_two_sided(x, y, v, ell):
    """Independent O((n+m) log) evaluation of sum_j exp(-|x_i-y_j|/ell) v_j in 1-D by two
    exponential recurrences over the sorted points (left-to-right and right-to-left)."""
    order = np.argsort(y, kind="stable")
    ys, vs = y[order], v[order]
    xo = np.argsort(x, kind="stable")
    out = np.zeros(len(x))
    # left part: sum_{y_j <= x} exp(-(x - y_j)/ell) v_j
    acc, pos, j = 0.0, -np.inf, 0
    for i in xo:
        xi = x[i]
        while j < len(ys) and ys[j] <= xi:
            acc = acc * math.exp(-(ys[j] - pos) / ell) if pos > -np.inf else 0.0
            acc += vs[j]
            pos = ys[j]
            j += 1
        out[i] += acc * math.exp(-(xi - pos) / ell) if pos > -np.inf else 0.0
    # right part: sum_{y_j > x} exp(-(y_j - x)/ell) v_j
    acc, pos, j = 0.0, np.inf, len(ys) - 1
    for i in xo[::-1]:
        xi = x[i]
        while j >= 0 and ys[j] > xi:
            acc = acc * math.exp(-(pos - ys[j]) / ell) if pos < np.inf else 0.0
            acc += vs[j]
            pos = ys[j]
            j -= 1
        out[i] += acc * math.exp(-(pos - xi) / ell) if pos < np.inf else 0.0
    return out


def test_direct_sum_1d_laplace_vs_recurrence():
    rng = np.random.default_rng(11)
    x = rng.uniform(-0.25, 0.25, 3000)
    y = rng.normal(0.05, 0.08, 2500)
    v = rng.uniform(0.5, 1.5, 2500)
    for ell in (0.01, 0.2):
        got = oracle.direct_sum(x, y, v, "laplace", ell)
        ref = _laplace_1d_two_sided(x, y, v, ell)
        assert rel(got, ref) < 1e-12


def test_direct_sum_1d_energy_vs_prefix_sums():
    """sum_j -|x - y_j| v_j = -[x (A_le - A_gt) - (B_le - B_gt)], A = sum v, B = sum y v."""
    rng = np.random.default_rng(12)
    x = rng.uniform(-0.25, 0.25, 3000)
    y = rng.uniform(-0.25, 0.25, 2800)
    v = rng.uniform(-1, 1, 2800)
    order = np.argsort(y)
    ys, vs = y[order], v[order]
    A = np.concatenate([[0.0], np.cumsum(vs)])
    B = np.concatenate([[0.0], np.cumsum(vs * ys)])
    k = np.searchsorted(ys, x, side="right")
    ref = -(x * (A[k] - (A[-1] - A[k])) - (B[k] - (B[-1] - B[k])))
    got = oracle.direct_sum(x, y, v, "energy", 1.0)
    assert rel(got, ref) < 1e-11


@pytest.mark.parametrize("kind", ["gauss", "laplace", "energy", "imq"])
def test_direct_sum_adjoint_symmetry(kind):
    """<u, K_xy v> = <K_yx u, v>: the kernel matrix of a radial kernel is symmetric."""
    rng = np.random.default_rng(13)
    x = rng.uniform(-0.25, 0.25, (300, 3))
    y = rng.uniform(-0.25, 0.25, (200, 3))
    u, v = rng.normal(size=300), rng.normal(size=200)
    lhs = u @ oracle.direct_sum(x, y, v, kind, 0.03)
    rhs = oracle.direct_sum(y, x, u, kind, 0.03) @ v
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)


@pytest.mark.parametrize("kind", ["gauss", "laplace", "energy", "imq"])
def test_direct_sum_grad_vs_central_differences(kind):
    rng = np.random.default_rng(14)
    x = rng.uniform(-0.25, 0.25, (6, 3))
    y = rng.uniform(-0.25, 0.25, (40, 3))
    v = rng.uniform(0.5, 1.5, 40)
    g = oracle.direct_sum_grad(x, y, v, kind, 0.05)
    h = 1e-6
    for i in range(6):
        for k in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, k] += h
            xm[i, k] -= h
            fd = (oracle.direct_sum(xp[i:i + 1], y, v, kind, 0.05)[0]
                  - oracle.direct_sum(xm[i:i + 1], y, v, kind, 0.05)[0]) / (2 * h)
            assert abs(fd - g[i, k]) < 1e-6 * (1 + abs(fd))


# Rows in scrambled order, with a repeat and a gap: a row function that used the position t in
# the list instead of rows[t] fails every case below.
_ROWS = np.array([37, 2, 19, 2, 40, 0, 23])


@pytest.mark.parametrize("kind,lam", [("gauss", 0.02), ("laplace", 0.05), ("energy", 1.0),
                                      ("imq", 0.3)])
@pytest.mark.parametrize("d", [1, 3])
def test_direct_sum_rows_are_the_selected_rows(kind, lam, d):
    """The sampled-row sum of eq. (fast_sum) is row rows[t] of the full direct sum, and those rows
    agree with a 40-digit brute force of the definition (an independent pin of the row function)."""
    rng = np.random.default_rng([11, d])
    x = rng.uniform(-0.25, 0.25, (41, d))
    y = rng.uniform(-0.25, 0.25, (29, d))
    v = rng.uniform(-1, 1, 29)
    got = oracle.direct_sum_rows(x, _ROWS, y, v, kind, lam)
    full = oracle.direct_sum(x, y, v, kind, lam)
    assert np.max(np.abs(got - full[_ROWS])) <= 1e-15 * np.max(np.abs(full))
    mp.mp.dps = 40
    for t in (0, 2, 4):
        i = int(_ROWS[t])
        acc = mp.mpf(0)
        for j in range(len(y)):
            r = mp.sqrt(sum((mp.mpf(float(x[i, k])) - mp.mpf(float(y[j, k]))) ** 2 for k in range(d)))
            acc += _mp_kernel(kind, lam, r) * mp.mpf(float(v[j]))
        assert abs(got[t] - float(acc)) <= 1e-13 * max(abs(float(acc)), 1e-300)


# --------------------------------------------------------------------------- unbalanced Sinkhorn

def _single_point(r_cost, A, B, eps, eta, sweeps):
    """n = m = 1: with C the cost, the half-steps are affine,
    beta <- kappa (C - gamma - eps log B), gamma <- kappa (C - beta - eps log A), kappa = eta/(eta+eps).
    Fixed point by solving the 2x2 linear system; iterate after T sweeps by the geometric error
    contraction beta_T - beta* = kappa^(2(T-1)) (beta_1 - beta*)."""
    kap = eta / (eta + eps)
    C = r_cost
    bstar = (kap * (C - eps * math.log(B)) - kap ** 2 * (C - eps * math.log(A))) / (1 - kap ** 2)
    gstar = (kap * (C - eps * math.log(A)) - kap ** 2 * (C - eps * math.log(B))) / (1 - kap ** 2)
    b1 = kap * (C - eps * math.log(B))
    bT = bstar + kap ** (2 * (sweeps - 1)) * (b1 - bstar)
    g1 = kap * (C - b1 - eps * math.log(A))
    gT = gstar + kap ** (2 * (sweeps - 1)) * (g1 - gstar)
    return bT, gT, bstar, gstar


@pytest.mark.parametrize("r", [1, 2])
def test_uot_single_point_closed_form(r):
    x = np.array([[0.1, -0.05]])
    y = np.array([[-0.07, 0.12]])
    dist = float(np.linalg.norm(x - y))
    C = dist ** r
    A, B, eps, eta = 0.7, 1.9, 0.05, 1.0
    for T in (1, 2, 5, 40):
        beta, gamma = oracle.uot_sinkhorn(x, [A], y, [B], eps, eta, T, r=r)
        bT, gT, _, _ = _single_point(C, A, B, eps, eta, T)
        assert abs(beta[0] - bT) < 1e-13 and abs(gamma[0] - gT) < 1e-13


def test_uot_coincident_points_reduce_to_single_point():
    """Point clouds collapsed to one location each behave like one point of the total mass."""
    x = np.tile([[0.1, -0.05]], (5, 1))
    y = np.tile([[-0.07, 0.12]], (3, 1))
    mu = np.array([0.1, 0.2, 0.15, 0.05, 0.2])
    nu = np.array([0.5, 0.9, 0.5])
    eps, eta = 0.05, 1.0
    beta, gamma = oracle.uot_sinkhorn(x, mu, y, nu, eps, eta, 7)
    bT, gT, _, _ = _single_point(float(np.sum((x[0] - y[0]) ** 2)), mu.sum(), nu.sum(), eps, eta, 7)
    assert np.allclose(beta, bT, atol=1e-13) and np.allclose(gamma, gT, atol=1e-13)


def _small_problem(seed=21, n=24, m=19, d=2):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-0.25, 0.25, (n, d))
    y = rng.normal(0.05, 0.1, (m, d))
    mu = rng.uniform(0.5, 1.5, n)
    nu = rng.uniform(0.5, 1.5, m)
    return x, mu / mu.sum(), y, 1.3 * nu / nu.sum()


@pytest.mark.parametrize("r", [1, 2])
def test_uot_halfstep_is_exact_block_maximiser(r):
    """Each half-step maximises the dual of Theorem 'dualization' over one block exactly:
    after a beta-update, dD/dbeta = 0; after a gamma-update, dD/dgamma = 0 (checked by central
    differences of the separately written dual), and D never decreases."""
    x, mu, y, nu = _small_problem()
    eps, eta = 0.03, 0.7
    beta, gamma = np.zeros(len(x)), np.zeros(len(y))
    prev = oracle.uot_dual(x, mu, y, nu, eps, eta, beta, gamma, r=r)
    h = 1e-6
    for delta in range(1, 9):
        beta, gamma = oracle.uot_halfsteps(x, mu, y, nu, eps, eta, 1, beta, gamma, r=r) \
            if delta % 2 == 1 else _gamma_step(x, mu, y, nu, eps, eta, beta, gamma, r)
        D = oracle.uot_dual(x, mu, y, nu, eps, eta, beta, gamma, r=r)
        assert D >= prev - 1e-14
        prev = D
        blk = beta if delta % 2 == 1 else gamma
        for i in (0, 3, 7):
            bp, bm = blk.copy(), blk.copy()
            bp[i] += h
            bm[i] -= h
            if delta % 2 == 1:
                gd = (oracle.uot_dual(x, mu, y, nu, eps, eta, bp, gamma, r=r)
                      - oracle.uot_dual(x, mu, y, nu, eps, eta, bm, gamma, r=r)) / (2 * h)
            else:
                gd = (oracle.uot_dual(x, mu, y, nu, eps, eta, beta, bp, r=r)
                      - oracle.uot_dual(x, mu, y, nu, eps, eta, beta, bm, r=r)) / (2 * h)
            assert abs(gd) < 1e-8


def _gamma_step(x, mu, y, nu, eps, eta, beta, gamma, r):
    # a gamma half-step is a beta half-step of the transposed problem
    g2, b2 = oracle.uot_halfsteps(y, nu, x, mu, eps, eta, 1, gamma, beta, r=r)
    return b2, g2


@pytest.mark.parametrize("r", [1, 2])
def test_uot_beta_rows_are_rows_of_a_beta_halfstep(r):
    """The sampled-row beta update (eq. (Sinkhorn_uot_iteration)) is row rows[t] of a full beta
    half-step taken from the same gamma, which the closed-form and block-maximiser pins above fix."""
    x, mu, y, nu = _small_problem(n=41, m=29)
    eps, eta = 0.03, 0.7
    beta, gamma = oracle.uot_sinkhorn(x, mu, y, nu, eps, eta, 3, r=r)
    full, _ = oracle.uot_halfsteps(x, mu, y, nu, eps, eta, 1, beta, gamma, r=r)
    got = oracle.uot_beta_rows(x, _ROWS, y, nu, gamma, eps, eta, r=r)
    assert np.max(np.abs(got - full[_ROWS])) <= 1e-15 * np.max(np.abs(full))


def test_uot_beta_rows_single_point_closed_form():
    """n = m = 1: beta = kappa (C - gamma - eps log B) exactly, for any gamma."""
    x = np.array([[0.1, -0.05], [0.2, 0.01]])
    y = np.array([[-0.07, 0.12]])
    B, eps, eta, g0 = 1.9, 0.05, 1.0, 0.013
    kap = eta / (eta + eps)
    got = oracle.uot_beta_rows(x, np.array([1, 0]), y, [B], [g0], eps, eta, r=2)
    for t, i in enumerate((1, 0)):
        C = float(np.sum((x[i] - y[0]) ** 2))
        assert abs(got[t] - kap * (C - g0 - eps * math.log(B))) < 1e-15


def test_uot_weak_and_strong_duality():
    """D(beta, gamma) <= primal(pi) for every iterate (weak duality); the gap closes at
    convergence (strong duality for eta > 0, Theorem 'dualization')."""
    x, mu, y, nu = _small_problem()
    eps, eta = 0.05, 1.0
    gaps = []
    for sweeps in (1, 3, 10, 400):
        b, g = oracle.uot_sinkhorn(x, mu, y, nu, eps, eta, sweeps)
        D = oracle.uot_dual(x, mu, y, nu, eps, eta, b, g)
        P = oracle.uot_primal(x, mu, y, nu, eps, eta, b, g)
        assert D <= P + 1e-13
        gaps.append(P - D)
    assert gaps[-1] < 1e-11 and gaps[0] > gaps[-1]


def test_uot_fixed_point_marginals():
    """At the optimum, the plan's first marginal is P_i = mu_i exp(-beta_i/eta) and the second
    Q_j = nu_j exp(-gamma_j/eta) (first-order conditions of the dual)."""
    x, mu, y, nu = _small_problem()
    eps, eta = 0.05, 0.5
    b, g = oracle.uot_sinkhorn(x, mu, y, nu, eps, eta, 600)
    P, Q = oracle.uot_marginals(x, mu, y, nu, eps, b, g)
    assert rel(P, mu * np.exp(-b / eta)) < 1e-10
    assert rel(Q, nu * np.exp(-g / eta)) < 1e-10


def test_uot_large_eta_recovers_balanced_marginals():
    """eta -> infinity with equal masses: the marginals approach mu and nu (Remark on eta -> inf:
    the marginal penalties enforce the constraints); the violation shrinks like 1/eta."""
    x, mu, y, nu = _small_problem(n=16, m=12)
    nu = nu / nu.sum()
    eps = 0.1
    errs = []
    for eta in (10.0, 100.0):
        kap = eta / (eta + eps)
        sweeps = int(30 / (1 - kap * kap)) + 50
        b, g = oracle.uot_sinkhorn(x, mu, y, nu, eps, eta, sweeps)
        P, Q = oracle.uot_marginals(x, mu, y, nu, eps, b, g)
        errs.append(max(rel(P, mu), rel(Q, nu)))
    assert errs[1] < errs[0] / 5 and errs[1] < 3e-3


def test_uot_cstar_upper_bound():
    """Proposition 'optimal independent measure' (eq. 561): the objective at c* mu x nu bounds the
    regularised UOT value from above, and c* makes the derivative of that objective vanish."""
    x, mu, y, nu = _small_problem()
    for r in (1, 2):
        eps, eta = 0.05, 1.0
        c, ub = oracle.uot_cstar(x, mu, y, nu, eps, eta, r=r)
        b, g = oracle.uot_sinkhorn(x, mu, y, nu, eps, eta, 500, r=r)
        D = oracle.uot_dual(x, mu, y, nu, eps, eta, b, g, r=r)
        assert D <= ub + 1e-13
        # stationarity of phi(c) = c K + Mm Mn (c log c - c + 1)/lam + eta Mm (c Mn log(c Mn) - c Mn + 1)
        #                          + eta Mn (c Mm log(c Mm) - c Mm + 1), K = <mu x nu, d^r>
        Kc = sum(mu[i] * nu[j] * np.linalg.norm(x[i] - y[j]) ** r
                 for i in range(len(x)) for j in range(len(y)))
        Mm, Mn = mu.sum(), nu.sum()

        def phi(cc):
            return (cc * Kc + eps * Mm * Mn * (cc * math.log(cc) - cc + 1)
                    + eta * Mm * (cc * Mn * math.log(cc * Mn) - cc * Mn + 1)
                    + eta * Mn * (cc * Mm * math.log(cc * Mm) - cc * Mm + 1))
        assert abs(phi(c) - ub) < 1e-12
        assert phi(c * 1.01) > phi(c) and phi(c * 0.99) > phi(c)


def test_scaling_single_stage_is_plain_sinkhorn():
    """One stage without a tolerance is Algorithm 1 itself."""
    x, mu, y, nu = _small_problem()
    b1, g1, cnt = oracle.uot_sinkhorn_scaling(x, mu, y, nu, [0.05], 1.0, 37, 0.0)
    b2, g2 = oracle.uot_sinkhorn(x, mu, y, nu, 0.05, 1.0, 37)
    assert cnt == [37]
    assert np.array_equal(b1, b2) and np.array_equal(g1, g2)


@pytest.mark.parametrize("init", ["zero", "cstar"])
def test_scaling_reaches_the_fixed_point_of_the_last_temperature(init):
    """The dual is strictly concave, so every start and every temperature path ends at the same
    fixed point of the last temperature: the scaled solve agrees with a long plain solve, the
    stopping rule holds at every stage end, and the marginal identity of the fixed point holds."""
    x, mu, y, nu = _small_problem(n=70, m=60, d=2)
    eta, tol = 1.0, 1e-10
    stages = [1.0, 0.05, 0.01]
    b, g, counts = oracle.uot_sinkhorn_scaling(x, mu, y, nu, stages, eta, 5000, tol, init=init)
    assert all(c < 5000 for c in counts)
    bref, gref = oracle.uot_sinkhorn(x, mu, y, nu, stages[-1], eta, 5000)
    assert rel(b, bref) < 1e-8 and rel(g, gref) < 1e-8
    # one more sweep moves nothing by more than the tolerance
    b2, g2 = oracle.uot_halfsteps(x, mu, y, nu, stages[-1], eta, 2, b, g)
    assert max(np.max(np.abs(b2 - b)), np.max(np.abs(g2 - g))) <= tol * stages[-1]
    P, Q = oracle.uot_marginals(x, mu, y, nu, stages[-1], b, g)
    assert rel(P, mu * np.exp(-b / eta)) < 1e-8


def test_scaling_cstar_start_is_the_log_of_eq_561():
    """With zero sweeps the c* start leaves gamma = eps_0 log c* (eq. (561)) and beta = 0."""
    x, mu, y, nu = _small_problem()
    b, g, counts = oracle.uot_sinkhorn_scaling(x, mu, y, nu, [0.2], 1.5, 0, 0.0, init="cstar")
    c, _ = oracle.uot_cstar(x, mu, y, nu, 0.2, 1.5)
    assert counts == [0] and np.all(b == 0) and np.allclose(g, 0.2 * math.log(c), rtol=0, atol=1e-15)


def test_sinkhorn_divergence_self_is_zero():
    x, mu, _, _ = _small_problem()
    sd, _ = oracle.sinkhorn_divergence(x, mu, x, mu, 0.05, 1.0, 200)
    assert abs(sd) < 1e-13


def test_sinkhorn_divergence_mass_term():
    """eq. (586): with identical supports the three UOT terms are functions of the masses only
    through the extra (1/(2 lam))(mu(X)-nu(X))^2 term plus the UOT values; check the decomposition
    reported alongside the value."""
    x, mu, y, nu = _small_problem()
    eps = 0.05
    sd, (uxy, uxx, uyy) = oracle.sinkhorn_divergence(x, mu, y, nu, eps, 1.0, 300)
    assert abs(sd - (uxy - 0.5 * uxx - 0.5 * uyy + 0.5 * eps * (mu.sum() - nu.sum()) ** 2)) < 1e-14
    assert sd > 0


def _dirac_uot(A, B, eps, eta):
    """UOT of eq. (W4) between A delta_z and B delta_z (zero cost): the plan is one number p >= 0
    and the objective eps (p log(p/(AB)) - p + AB) + eta (p log(p/A) - p + A) + eta (p log(p/B)
    - p + B) is minimised where eps log(p/(AB)) + eta log(p/A) + eta log(p/B) = 0, i.e.
    p = (AB)^((eps + eta)/(eps + 2 eta))."""
    p = (A * B) ** ((eps + eta) / (eps + 2 * eta))
    return (eps * (p * math.log(p / (A * B)) - p + A * B)
            + eta * (p * math.log(p / A) - p + A) + eta * (p * math.log(p / B) - p + B))


@pytest.mark.parametrize("A,B", [(0.7, 1.9), (1.0, 1.0), (2.5, 0.4)])
def test_sinkhorn_divergence_of_diracs_closed_form(A, B):
    """eq. (586) for two Diracs at one location: every UOT term has the closed form above, so the
    divergence, its mass term (1/(2 lambda))(mu(X) - nu(X))^2 included, is fixed without the
    Sinkhorn iteration or the dual.  Several coincident points of the same total mass give the same
    value."""
    eps, eta = 0.5, 1.0
    z = np.array([[0.03, -0.02]])
    ref = (_dirac_uot(A, B, eps, eta) - 0.5 * _dirac_uot(A, A, eps, eta)
           - 0.5 * _dirac_uot(B, B, eps, eta) + 0.5 * eps * (A - B) ** 2)
    sd, (uxy, uxx, uyy) = oracle.sinkhorn_divergence(z, [A], z, [B], eps, eta, 200)
    assert abs(uxy - _dirac_uot(A, B, eps, eta)) < 1e-13
    assert abs(uxx - _dirac_uot(A, A, eps, eta)) < 1e-13
    assert abs(sd - ref) < 1e-13
    zs = np.tile(z, (3, 1))
    sd3, _ = oracle.sinkhorn_divergence(zs, [A / 4, A / 2, A / 4], np.tile(z, (2, 1)),
                                        [B / 3, 2 * B / 3], eps, eta, 200)
    assert abs(sd3 - ref) < 1e-13


@pytest.mark.parametrize("r", [1, 2])
def test_uot_envelope_gradient_vs_central_differences(r):
    """Gradients of the converged UOT value with respect to positions and weights (envelope
    theorem on the dual) against central differences of the value itself."""
    x, mu, y, nu = _small_problem(n=10, m=8)
    eps, eta = 0.05, 1.0
    sweeps = 1500

    def value(xx, mm, yy, nn):
        b, g = oracle.uot_sinkhorn(xx, mm, yy, nn, eps, eta, sweeps, r=r)
        return oracle.uot_dual(xx, mm, yy, nn, eps, eta, b, g, r=r)

    b, g = oracle.uot_sinkhorn(x, mu, y, nu, eps, eta, sweeps, r=r)
    dx, dmu, dy, dnu = oracle.uot_grad(x, mu, y, nu, eps, eta, b, g, r=r)
    h = 1e-5
    for i, k in ((0, 0), (3, 1), (9, 0)):
        xp, xm = x.copy(), x.copy()
        xp[i, k] += h
        xm[i, k] -= h
        fd = (value(xp, mu, y, nu) - value(xm, mu, y, nu)) / (2 * h)
        assert abs(fd - dx[i, k]) < 1e-7 * (1 + abs(fd))
    for i in (0, 5):
        mp_, mm_ = mu.copy(), mu.copy()
        mp_[i] += h
        mm_[i] -= h
        fd = (value(x, mp_, y, nu) - value(x, mm_, y, nu)) / (2 * h)
        assert abs(fd - dmu[i]) < 1e-7 * (1 + abs(fd))
    for j, k in ((2, 1),):
        yp, ym = y.copy(), y.copy()
        yp[j, k] += h
        ym[j, k] -= h
        fd = (value(x, mu, yp, nu) - value(x, mu, ym, nu)) / (2 * h)
        assert abs(fd - dy[j, k]) < 1e-7 * (1 + abs(fd))
    np_, nm_ = nu.copy(), nu.copy()
    np_[4] += h
    nm_[4] -= h
    fd = (value(x, mu, y, np_) - value(x, mu, y, nm_)) / (2 * h)
    assert abs(fd - dnu[4]) < 1e-7 * (1 + abs(fd))


def test_divergence_tends_to_half_energy_mmd():
    """Corollary 477: for probability measures, sd_{1;eta;lambda} tends to the energy distance as
    lambda -> 0 (eps -> inf) after eta -> inf.  With eq. (1205) for MMD^2 (signed, k = -|.|) the
    limit is MMD^2 / 2: the plan tends to P x P~, so each UOT term tends to <P x P~, d>.  The ratio
    approaches 1 as eps grows at large eta."""
    rng = np.random.default_rng(1450)
    n = 120
    x, y = rng.uniform(0, 1, (n, 1)), rng.uniform(0, 1, (n, 1))
    a = b = np.full(n, 1.0 / n)
    half = 0.5 * oracle.mmd2(x, a, y, b, "energy", 1.0)[0]
    errs = []
    for eps in (10.0, 100.0, 1000.0):
        sd, _ = oracle.sinkhorn_divergence(x, a, y, b, eps, 1e4, 300, r=1)
        errs.append(abs(sd / half - 1.0))
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-3


# --------------------------------------------------------------------------- MMD

@pytest.mark.parametrize("kind", ["gauss", "laplace", "energy", "imq"])
def test_mmd_self_is_zero(kind):
    x, mu, _, _ = _small_problem()
    v, _ = oracle.mmd2(x, mu, x, mu, kind, 0.25)
    assert abs(v) < 1e-14


@pytest.mark.parametrize("kind", ["gauss", "laplace", "imq"])
def test_mmd_elementary_bound(kind):
    """0 <= MMD^2 <= sup|k| (mu(X)^2 + nu(X)^2) for nonnegative p.d. kernels (Remark on the
    elementary bound; valid for Gauss, Laplace and IMQ, sup k = 1 resp. 1/c)."""
    x, mu, y, nu = _small_problem()
    v, _ = oracle.mmd2(x, mu, y, nu, kind, 0.25)
    sup = 1.0 / 0.25 if kind == "imq" else 1.0
    assert 0 <= v <= sup * (mu.sum() ** 2 + nu.sum() ** 2)


def test_mmd_energy_1d_cramer_identity():
    """1-D energy distance equals Cramer's distance (Section 'Prominent kernels'): for the signed
    measure c = mu - nu with CDF F and total C, sum_ij c_i c_j (-|z_i - z_j|) = -2 int F (C - F)."""
    rng = np.random.default_rng(31)
    x = rng.uniform(-0.25, 0.25, 400)
    y = rng.normal(0.05, 0.08, 300)
    mu = rng.uniform(0.5, 1.5, 400)
    nu = rng.uniform(0.5, 1.5, 300)
    mu, nu = mu / mu.sum(), 1.5 * nu / nu.sum()
    z = np.concatenate([x, y])
    c = np.concatenate([mu, -nu])
    o = np.argsort(z)
    zs, cs = z[o], c[o]
    F = np.cumsum(cs)[:-1]
    ref = -2.0 * np.sum(F * (c.sum() - F) * np.diff(zs))
    v, _ = oracle.mmd2(x, mu, y, nu, "energy", 1.0)
    assert abs(v - ref) < 1e-12 * max(1.0, abs(ref))


@pytest.mark.parametrize("kind", ["gauss", "laplace", "energy", "imq"])
def test_mmd_grad_vs_central_differences(kind):
    x, mu, y, nu = _small_problem(n=12, m=9, d=3)
    dx, dmu, dy, dnu = oracle.mmd2_grad(x, mu, y, nu, kind, 0.1)
    h = 1e-6
    for i, k in ((0, 0), (4, 2), (11, 1)):
        xp, xm = x.copy(), x.copy()
        xp[i, k] += h
        xm[i, k] -= h
        fd = (oracle.mmd2(xp, mu, y, nu, kind, 0.1)[0] - oracle.mmd2(xm, mu, y, nu, kind, 0.1)[0]) / (2 * h)
        assert abs(fd - dx[i, k]) < 1e-7 * (1 + abs(fd))
    for i in (1, 7):
        mp_, mm_ = mu.copy(), mu.copy()
        mp_[i] += h
        mm_[i] -= h
        fd = (oracle.mmd2(x, mp_, y, nu, kind, 0.1)[0] - oracle.mmd2(x, mm_, y, nu, kind, 0.1)[0]) / (2 * h)
        assert abs(fd - dmu[i]) < 1e-7 * (1 + abs(fd))
    yp, ym = y.copy(), y.copy()
    yp[3, 1] += h
    ym[3, 1] -= h
    fd = (oracle.mmd2(x, mu, yp, nu, kind, 0.1)[0] - oracle.mmd2(x, mu, ym, nu, kind, 0.1)[0]) / (2 * h)
    assert abs(fd - dy[3, 1]) < 1e-7 * (1 + abs(fd))
    np_, nm_ = nu.copy(), nu.copy()
    np_[2] += h
    nm_[2] -= h
    fd = (oracle.mmd2(x, mu, y, np_, kind, 0.1)[0] - oracle.mmd2(x, mu, y, nm_, kind, 0.1)[0]) / (2 * h)
    assert abs(fd - dnu[2]) < 1e-7 * (1 + abs(fd))


# --------------------------------------------------------------------------- workloads

def test_d1_workload_matches_paper_table_parameters():
    """uot_d1_n2k is the paper's Table tab:Sinkhorn3 parameter set (r=2, lambda=20, eta=1) in the
    temperature convention eps = 1/lambda."""
    g = json.load(open(os.path.join(GOLDEN, "paper_parameters.json")))["table_sinkhorn3"]
    c = synth.CONFIGS["uot_d1_n2k"]
    assert abs(c["eps"] - 1.0 / g["lambda_paper"]) < 1e-15 and c["rho"] == g["eta"]


def test_generators_are_seeded_and_in_domain():
    a = synth.make("uot_d3_n1M", n=5000)
    b = synth.make("uot_d3_n1M", n=5000)
    assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["b"], b["b"])
    for c in ("uot_d1_n2k", "uot_d2_n100k", "uot_d3_n1M"):
        w = synth.make(c, n=3000)
        assert w["x"].dtype == np.float32 and w["x"].min() >= -0.25 and w["x"].max() < 0.25
        assert w["y"].min() >= -0.25 and w["y"].max() < 0.25
        assert abs(w["a"].sum() - w["mass_a"]) < 1e-4 and abs(w["b"].sum() - w["mass_b"]) < 1e-4


def test_row_gradients_match_full_gradients():
    """The sampled-row gradient functions agree with the full ones (same definitions, row subset)."""
    x, mu, y, nu = _small_problem(n=15, m=11, d=2)
    rows = np.array([0, 4, 14])
    for r in (1, 2):
        b, g = oracle.uot_sinkhorn(x, mu, y, nu, 0.05, 1.0, 50, r=r)
        dx, dmu, _, _ = oracle.uot_grad(x, mu, y, nu, 0.05, 1.0, b, g, r=r)
        rx, rm = oracle.uot_grad_rows(x, mu, rows, y, nu, 0.05, 1.0, b, g, r=r)
        assert np.allclose(rx, dx[rows], rtol=1e-12, atol=1e-15)
        assert np.allclose(rm, dmu[rows], rtol=1e-12, atol=1e-15)
    for kind in ("gauss", "energy"):
        dx, dmu, _, _ = oracle.mmd2_grad(x, mu, y, nu, kind, 0.1)
        rx, rm = oracle.mmd2_grad_rows(x, mu, rows, y, nu, kind, 0.1)
        assert np.allclose(rx, dx[rows], rtol=1e-12, atol=1e-15)
        assert np.allclose(rm, dmu[rows], rtol=1e-12, atol=1e-15)


def test_golden_divergence_differences_match_the_envelope_gradient():
    """The stored central differences of the converged divergence (written by
    tests/golden/make_divergence_fd.py from the oracle alone) agree with the oracle's envelope
    gradient at the same entries (Theorem "dualization": the gradient of the dual value at the
    maximiser), to the O(h^2) truncation of the differences; the file matches its workload."""
    g = json.load(open(os.path.join(GOLDEN, "divergence_fd_d2_n2000.json")))
    c = synth.CONFIGS[g["workload"]]
    assert (g["eps"], g["rho"]) == (c["eps"], c["rho"]) and len(g["rows"]) == 64
    assert len(g["weight_rows"]) == 16 and g["h"] == c["fd_h"]
    assert rel(g["envelope_dx"], g["fd_dx"]) < 1e-4
    assert rel(g["envelope_da"], g["fd_da"]) < 1e-4
