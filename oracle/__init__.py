"""FP64 CPU oracle (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg may import this
package.  It wraps ``oracle.c`` (plain C, OpenMP) through ctypes and shares no code with the GPU
library.  Arrays are promoted to float64 before the call, so float32 inputs are used exactly.

Notation follows the paper: ``eps`` is the temperature (the paper's 1/lambda), ``eta`` the marginal
penalty, ``beta``/``gamma`` the dual potentials, r the cost exponent (r=2: Gibbs kernel
exp(-|x-y|^2/eps); r=1: exp(-|x-y|/eps)).  Kernel kinds: 0 Gauss exp(-r^2/ell2), 1 Laplace
exp(-r/ell), 2 energy -r, 3 IMQ 1/sqrt(r^2 + c^2).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
KINDS = {"gauss": 0, "laplace": 1, "energy": 2, "imq": 3}
_lib = None


def build(force=True):
    """Compile oracle.c into liboracle.so with gcc (OpenMP, -O2, strict IEEE: no fast-math)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                           "-Wall", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        I = ctypes.c_int
        D = ctypes.c_double
        sig = {
            "orc_kernel": (D, [I, D, D]),
            "orc_direct_sum": (None, [P, I64, P, I64, I, P, I, D, P]),
            "orc_direct_sum_rows": (None, [P, P, I64, P, I64, I, P, I, D, P]),
            "orc_direct_sum_grad": (None, [P, I64, P, I64, I, P, I, D, P]),
            "orc_uot_sinkhorn_halfsteps": (None, [P, P, I64, P, P, I64, I, I, D, D, I64, P, P]),
            "orc_uot_sinkhorn": (None, [P, P, I64, P, P, I64, I, I, D, D, I64, P, P]),
            "orc_uot_beta_rows": (None, [P, P, I64, P, P, P, I64, I, I, D, D, P]),
            "orc_uot_dual": (D, [P, P, I64, P, P, I64, I, I, D, D, P, P]),
            "orc_uot_primal": (D, [P, P, I64, P, P, I64, I, I, D, D, P, P]),
            "orc_uot_marginals": (None, [P, P, I64, P, P, I64, I, I, D, P, P, P, P]),
            "orc_uot_cstar": (D, [P, P, I64, P, P, I64, I, I, D, D, P]),
            "orc_sinkhorn_divergence": (D, [P, P, I64, P, P, I64, I, I, D, D, I64, P]),
            "orc_uot_grad": (None, [P, P, I64, P, P, I64, I, I, D, D, P, P, P, P, P, P]),
            "orc_mmd2": (D, [P, P, I64, P, P, I64, I, I, D, P]),
            "orc_mmd2_grad": (None, [P, P, I64, P, P, I64, I, I, D, P, P, P, P]),
            "orc_uot_grad_rows": (None, [P, P, P, I64, P, P, I64, I, I, D, D, P, P, P, P]),
            "orc_mmd2_grad_rows": (None, [P, P, I64, P, I64, P, P, I64, I, I, D, P, P]),
            "orc_num_threads": (I, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def _pts(x):
    x = _f64(x)
    if x.ndim == 1:
        x = x.reshape(-1, 1)
    return np.ascontiguousarray(x), x.shape[0], x.shape[1]


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _kind(kind):
    return KINDS[kind] if isinstance(kind, str) else int(kind)


def num_threads():
    return lib().orc_num_threads()


def kernel(kind, lam_k, r):
    return lib().orc_kernel(_kind(kind), float(lam_k), float(r))


def direct_sum(x, y, alpha, kind, lam_k):
    """s_i = sum_j K(|x_i - y_j|) alpha_j (eq. fast_sum, evaluated directly)."""
    x, n, d = _pts(x)
    y, m, d2 = _pts(y)
    assert d == d2
    al = _f64(alpha)
    out = np.empty(n)
    lib().orc_direct_sum(_p(x), n, _p(y), m, d, _p(al), _kind(kind), float(lam_k), _p(out))
    return out


def direct_sum_rows(x, rows, y, alpha, kind, lam_k):
    x, n, d = _pts(x)
    y, m, _ = _pts(y)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    al = _f64(alpha)
    out = np.empty(len(rows))
    lib().orc_direct_sum_rows(_p(x), _p(rows), len(rows), _p(y), m, d, _p(al), _kind(kind),
                              float(lam_k), _p(out))
    return out


def direct_sum_grad(x, y, alpha, kind, lam_k):
    x, n, d = _pts(x)
    y, m, _ = _pts(y)
    al = _f64(alpha)
    out = np.empty((n, d))
    lib().orc_direct_sum_grad(_p(x), n, _p(y), m, d, _p(al), _kind(kind), float(lam_k), _p(out))
    return out


def uot_sinkhorn(x, mu, y, nu, eps, eta, sweeps, r=2):
    """Algorithm 1, `sweeps` full sweeps (beta then gamma) from gamma = 0.  Returns (beta, gamma)."""
    x, n, d = _pts(x)
    y, m, _ = _pts(y)
    mu, nu = _f64(mu), _f64(nu)
    beta, gamma = np.empty(n), np.empty(m)
    lib().orc_uot_sinkhorn(_p(x), _p(mu), n, _p(y), _p(nu), m, d, int(r), float(eps), float(eta),
                           int(sweeps), _p(beta), _p(gamma))
    return beta, gamma


def uot_halfsteps(x, mu, y, nu, eps, eta, nhalf, beta, gamma, r=2):
    """Continue Algorithm 1 for `nhalf` half-steps from the given (beta, gamma); returns copies."""
    x, n, d = _pts(x)
    y, m, _ = _pts(y)
    mu, nu = _f64(mu), _f64(nu)
    beta, gamma = _f64(beta).copy(), _f64(gamma).copy()
    lib().orc_uot_sinkhorn_halfsteps(_p(x), _p(mu), n, _p(y), _p(nu), m, d, int(r), float(eps),
                                     float(eta), int(nhalf), _p(beta), _p(gamma))
    return beta, gamma


def uot_beta_rows(x, rows, y, nu, gamma, eps, eta, r=2):
    x, n, d = _pts(x)
    y, m, _ = _pts(y)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    nu, gamma = _f64(nu), _f64(gamma)
    out = np.empty(len(rows))
    lib().orc_uot_beta_rows(_p(x), _p(rows), len(rows), _p(y), _p(nu), _p(gamma), m, d, int(r),
                            float(eps), float(eta), _p(out))
    return out


def uot_dual(x, mu, y, nu, eps, eta, beta, gamma, r=2):
    x, n, d = _pts(x)
    y, m, _ = _pts(y)
    mu, nu, beta, gamma = _f64(mu), _f64(nu), _f64(beta), _f64(gamma)
    return lib().orc_uot_dual(_p(x), _p(mu), n, _p(y), _p(nu), m, d, int(r), float(eps),
                              float(eta), _p(beta), _p(gamma))


def uot_primal(x, mu, y, nu, eps, eta, beta, gamma, r=2):
    x, n, d = _pts(x)
    y, m, _ = _pts(y)
    mu, nu, beta, gamma = _f64(mu), _f64(nu), _f64(beta), _f64(gamma)
    return lib().orc_uot_primal(_p(x), _p(mu), n, _p(y), _p(nu), m, d, int(r), float(eps),
                                float(eta), _p(beta), _p(gamma))


def uot_marginals(x, mu, y, nu, eps, beta, gamma, r=2):
    x, n, d = _pts(x)
    y, m, _ = _pts(y)
    mu, nu, beta, gamma = _f64(mu), _f64(nu), _f64(beta), _f64(gamma)
    P, Q = np.empty(n), np.empty(m)
    lib().orc_uot_marginals(_p(x), _p(mu), n, _p(y), _p(nu), m, d, int(r), float(eps), _p(beta),
                            _p(gamma), _p(P), _p(Q))
    return P, Q


def uot_cstar(x, mu, y, nu, eps, eta, r=2):
    """Returns (c*, objective at c* mu x nu) of eq. (561)."""
    x, n, d = _pts(x)
    y, m, _ = _pts(y)
    mu, nu = _f64(mu), _f64(nu)
    ub = ctypes.c_double(0.0)
    c = lib().orc_uot_cstar(_p(x), _p(mu), n, _p(y), _p(nu), m, d, int(r), float(eps), float(eta),
                            ctypes.byref(ub))
    return c, ub.value


def uot_sinkhorn_scaling(x, mu, y, nu, eps_stages, eta, max_sweeps, tol, init="zero", r=2,
                         beta0=None, gamma0=None):
    """lambda-scaling (Section "lambda-scaling"): Algorithm 1 solved for a sequence of
    temperatures eps_stages (increasing lambda = 1/eps), each stage warm-started from the
    potentials of the previous one.  A stage ends after the first full sweep (beta then gamma) that
    changes no potential by more than tol * eps (the potentials enter the kernel sums as
    e^{potential/eps}), or after `max_sweeps` sweeps.
    init: "zero" (gamma = 0), "cstar" (the remark on initialisation, read as e^{gamma/eps} = c*
    with c* of eq. (561) at the first temperature: gamma = eps_0 log c*), or "warm" (beta0,
    gamma0).  Returns (beta, gamma, sweeps per stage)."""
    xs, n, _ = _pts(x)
    ys, m, _ = _pts(y)
    beta, gamma = np.zeros(n), np.zeros(m)
    if init == "cstar":
        c, _ = uot_cstar(x, mu, y, nu, eps_stages[0], eta, r=r)
        gamma[:] = eps_stages[0] * np.log(c)
    elif init == "warm":
        beta, gamma = _f64(beta0).copy(), _f64(gamma0).copy()
    counts = []
    for eps in eps_stages:
        k = 0
        while k < max_sweeps:
            nb, ng = uot_halfsteps(x, mu, y, nu, eps, eta, 2, beta, gamma, r=r)
            k += 1
            delta = max(np.max(np.abs(nb - beta), initial=0.0), np.max(np.abs(ng - gamma), initial=0.0))
            beta, gamma = nb, ng
            if delta <= tol * eps:
                break
        counts.append(k)
    return beta, gamma, counts


def sinkhorn_divergence(x, mu, y, nu, eps, eta, sweeps, r=2):
    """eq. (586); returns (sd, (UOT(mu,nu), UOT(mu,mu), UOT(nu,nu)))."""
    x, n, d = _pts(x)
    y, m, _ = _pts(y)
    mu, nu = _f64(mu), _f64(nu)
    t = np.empty(3)
    v = lib().orc_sinkhorn_divergence(_p(x), _p(mu), n, _p(y), _p(nu), m, d, int(r), float(eps),
                                      float(eta), int(sweeps), _p(t))
    return v, tuple(t)


def uot_grad(x, mu, y, nu, eps, eta, beta, gamma, r=2):
    """Envelope gradients of the dual value: (dx, dmu, dy, dnu)."""
    x, n, d = _pts(x)
    y, m, _ = _pts(y)
    mu, nu, beta, gamma = _f64(mu), _f64(nu), _f64(beta), _f64(gamma)
    dx, dy = np.empty((n, d)), np.empty((m, d))
    dmu, dnu = np.empty(n), np.empty(m)
    lib().orc_uot_grad(_p(x), _p(mu), n, _p(y), _p(nu), m, d, int(r), float(eps), float(eta),
                       _p(beta), _p(gamma), _p(dx), _p(dmu), _p(dy), _p(dnu))
    return dx, dmu, dy, dnu


def uot_grad_rows(x, mu, rows, y, nu, eps, eta, beta, gamma, r=2):
    """Envelope gradient (dx, dmu) of the dual for selected rows of x (first slot)."""
    x, n, d = _pts(x)
    y, m, _ = _pts(y)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    mu, nu, beta, gamma = _f64(mu), _f64(nu), _f64(beta), _f64(gamma)
    dx, dmu = np.empty((len(rows), d)), np.empty(len(rows))
    lib().orc_uot_grad_rows(_p(x), _p(mu), _p(rows), len(rows), _p(y), _p(nu), m, d, int(r),
                            float(eps), float(eta), _p(beta), _p(gamma), _p(dx), _p(dmu))
    return dx, dmu


def mmd2_grad_rows(x, mu, rows, y, nu, kind, lam_k):
    """Gradient rows (dx, dmu) of eq. (1205) for selected rows of x."""
    x, n, d = _pts(x)
    y, m, _ = _pts(y)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    mu, nu = _f64(mu), _f64(nu)
    dx, dmu = np.empty((len(rows), d)), np.empty(len(rows))
    lib().orc_mmd2_grad_rows(_p(x), _p(mu), n, _p(rows), len(rows), _p(y), _p(nu), m, d,
                             _kind(kind), float(lam_k), _p(dx), _p(dmu))
    return dx, dmu


def mmd2(x, mu, y, nu, kind, lam_k):
    """Signed MMD^2 of eq. (1205); returns (value, (Kxx, Kxy, Kyy) double sums)."""
    x, n, d = _pts(x)
    y, m, _ = _pts(y)
    mu, nu = _f64(mu), _f64(nu)
    t = np.empty(3)
    v = lib().orc_mmd2(_p(x), _p(mu), n, _p(y), _p(nu), m, d, _kind(kind), float(lam_k), _p(t))
    return v, tuple(t)


def mmd2_grad(x, mu, y, nu, kind, lam_k):
    x, n, d = _pts(x)
    y, m, _ = _pts(y)
    mu, nu = _f64(mu), _f64(nu)
    dx, dy = np.empty((n, d)), np.empty((m, d))
    dmu, dnu = np.empty(n), np.empty(m)
    lib().orc_mmd2_grad(_p(x), _p(mu), n, _p(y), _p(nu), m, d, _kind(kind), float(lam_k), _p(dx),
                        _p(dmu), _p(dy), _p(dnu))
    return dx, dmu, dy, dnu
