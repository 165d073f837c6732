"""fastuot for MI355X: fast radial-kernel summation, unbalanced Sinkhorn and MMD on gfx950.

A thin ctypes binding over ``libfastuot.so`` (the C-ABI of ``include/fastuot.h``).  The functions
have the C entry points' names and only marshal arguments: every step of the computation runs in
the library's HIP kernels.  Tensors must be HIP (``torch.cuda``) tensors; work is enqueued on
torch's current stream.  There is no CPU fallback: importing raises if the library is not built.

Parameter convention (temperature form): the Gibbs kernel of the cost |x-y|^r is
exp(-|x-y|^r / lam), i.e. ``lam`` is the reciprocal of the paper's lambda; ``rho`` is the paper's
marginal penalty eta.  Kernels: "gauss" exp(-r^2/lam), "laplace" exp(-r/lam), "energy" -r,
"imq" 1/sqrt(r^2 + lam^2).
"""
import ctypes
import os

import numpy as np

import torch

__all__ = [
    "fastsum_apply", "Plan", "uot_sinkhorn", "uot_sinkhorn_grad", "uot_upper_bound",
    "uot_sinkhorn_scaling", "sinkhorn_divergence",
    "sinkhorn_divergence_grad", "mmd", "mmd_grad", "SinkhornDivergence", "MMD2",
    "FastsumError", "KERNELS", "library_path", "EXPORTED", "fs_profile_enable",
    "fs_profile_select", "fs_profile_query", "fs_profile_reset",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "libfastuot.so")
KERNELS = {"gauss": 0, "laplace": 1, "energy": 2, "imq": 3}
FLAG_WARM_START = 0x1
FLAG_FORCE_VALU = 0x2
FLAG_DETERMINISTIC = 0x4
EXPORTED = ("fs_last_error", "fs_version", "fs_release_cache", "fs_profile_enable",
            "fs_profile_select",
            "fs_profile_query", "fs_profile_reset", "fastsum_apply", "fs_plan_create",
            "fs_plan_apply", "fs_plan_apply_noalloc", "fs_plan_multiplier", "fs_plan_destroy", "uot_sinkhorn", "uot_upper_bound",
            "uot_sinkhorn_scaling", "uot_sinkhorn_grad", "sinkhorn_divergence",
            "sinkhorn_divergence_grad", "mmd", "mmd_grad")
INITS = {"zero": 0, "cstar": 1, "warm": 2}


class FastsumError(RuntimeError):
    """A non-OK status from the library (the message is fs_last_error())."""


class fs_params(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int), ("grid", ctypes.c_int), ("window", ctypes.c_int),
                ("oversampling", ctypes.c_int), ("smoothness", ctypes.c_int),
                ("flags", ctypes.c_uint), ("lambda_", ctypes.c_double),
                ("nearfield_radius", ctypes.c_double), ("bandwidth", ctypes.c_int)]


def library_path():
    return _LIBPATH


def _load():
    if not os.path.exists(_LIBPATH):
        raise ImportError(
            "libfastuot.so is not built (expected at %s); run paper_2306_13618_amd/build.py "
            "or __graft_entry__.build()" % _LIBPATH)
    L = ctypes.CDLL(_LIBPATH)
    P, I64, I, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    PP = ctypes.POINTER(fs_params)
    sig = {
        "fs_last_error": (ctypes.c_char_p, []),
        "fs_version": (I, []),
        "fs_release_cache": (None, []),
        "fs_profile_enable": (I, [I]),
        "fs_profile_select": (I, [ctypes.c_char_p, I]),
        "fs_profile_query": (I, [ctypes.c_char_p, ctypes.POINTER(D), ctypes.POINTER(I64)]),
        "fs_profile_reset": (None, []),
        "fastsum_apply": (I, [P, I64, P, I64, I, P, P, PP, P]),
        "fs_plan_create": (I, [P, I64, P, I64, I, PP, P, ctypes.POINTER(P)]),
        "fs_plan_apply": (I, [P, P, P, I, P]),
        "fs_plan_apply_noalloc": (I, [P, P, P, I, P]),
        "fs_plan_multiplier": (I, [P, P, P, I64, ctypes.POINTER(D), ctypes.POINTER(I), P]),
        "fs_plan_destroy": (None, [P]),
        "uot_sinkhorn": (I, [P, P, I64, P, P, I64, I, PP, D, I, P, P, P, P]),
        "uot_upper_bound": (I, [P, P, I64, P, P, I64, I, PP, D, P, P, P]),
        "uot_sinkhorn_scaling": (I, [P, P, I64, P, P, I64, I, PP, P, I, D, I, D, I, P, P, P, P,
                                     P]),
        "uot_sinkhorn_grad": (I, [P, P, I64, P, P, I64, I, PP, D, P, P, D, P, P, P, P, P]),
        "sinkhorn_divergence": (I, [P, P, I64, P, P, I64, I, PP, D, I, P, P, P, P, P, P, P]),
        "sinkhorn_divergence_grad": (I, [P, P, I64, P, P, I64, I, PP, D, P, P, P, P, D, P, P, P,
                                         P, P]),
        "mmd": (I, [P, P, I64, P, P, I64, I, PP, P, P, P]),
        "mmd_grad": (I, [P, P, I64, P, P, I64, I, PP, D, P, P, P, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


_lib = _load()


def _check(status):
    if status != 0:
        raise FastsumError("fastuot status %d: %s" % (status, _lib.fs_last_error().decode()))


def _params(kernel="gauss", lam=1.0, grid=0, window=0, oversampling=0, smoothness=0,
            nearfield_radius=0.0, flags=0, bandwidth=0):
    p = fs_params()
    p.bandwidth = int(bandwidth)
    p.kernel = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    p.grid = int(grid)
    p.window = int(window)
    p.oversampling = int(oversampling)
    p.smoothness = int(smoothness)
    p.flags = int(flags)
    p.lambda_ = float(lam)
    p.nearfield_radius = float(nearfield_radius)
    return p


def _dev(t, dtype=torch.float32, name="tensor"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a HIP (torch.cuda) tensor" % name)
    if t.dtype != dtype:
        t = t.to(dtype)
    return t.contiguous()


def _pts(t, name):
    t = _dev(t, name=name)
    if t.dim() == 1:
        t = t.reshape(-1, 1)
    if t.dim() != 2:
        raise ValueError("%s must be (count, d)" % name)
    return t


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _opt(out):
    return _ptr(out) if out is not None else ctypes.c_void_p(0)


def fs_release_cache():
    """Release the library's cached device memory (workspace blocks and the multipliers kept from
    recent plans)."""
    _lib.fs_release_cache()


def fs_profile_enable(enable=True):
    """Record HIP events around the library's passes (spread, fold, fft, gather, ...)."""
    _check(_lib.fs_profile_enable(int(bool(enable))))


def fs_profile_select(name=None, period=1):
    """Record only the passes called `name` (None: all), every `period`-th of them."""
    _check(_lib.fs_profile_select(name.encode() if name else None, int(period)))


def fs_profile_query(name):
    """(total milliseconds, launch count) of one pass since the last reset."""
    ms, cnt = ctypes.c_double(0.0), ctypes.c_int64(0)
    _check(_lib.fs_profile_query(name.encode(), ctypes.byref(ms), ctypes.byref(cnt)))
    return ms.value, cnt.value


def fs_profile_reset():
    _lib.fs_profile_reset()


def fastsum_apply(x, y, v, kernel="gauss", lam=1.0, grid=0, window=0, oversampling=0,
                  smoothness=0, nearfield_radius=0.0, flags=0, bandwidth=0):
    """out_i = sum_j K(x_i - y_j) v_j (eq. fast_sum); grid=0 selects direct summation."""
    x, y = _pts(x, "x"), _pts(y, "y")
    v = _dev(v, name="v").reshape(-1)
    out = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
    p = _params(kernel, lam, grid, window, oversampling, smoothness, nearfield_radius, flags,
                bandwidth)
    _check(_lib.fastsum_apply(_ptr(x), x.shape[0], _ptr(y), y.shape[0], x.shape[1], _ptr(v),
                              _ptr(out), ctypes.byref(p), _stream(x.device)))
    return out


class Plan:
    """fs_plan_create / fs_plan_apply / fs_plan_destroy."""

    def __init__(self, x, y, kernel="gauss", lam=1.0, grid=0, window=0, oversampling=0,
                 smoothness=0, nearfield_radius=0.0, flags=0, bandwidth=0):
        x, y = _pts(x, "x"), _pts(y, "y")
        self.n, self.m, self.d, self.device = x.shape[0], y.shape[0], x.shape[1], x.device
        p = _params(kernel, lam, grid, window, oversampling, smoothness, nearfield_radius, flags,
                bandwidth)
        h = ctypes.c_void_p(0)
        _check(_lib.fs_plan_create(_ptr(x), self.n, _ptr(y), self.m, self.d, ctypes.byref(p),
                                   _stream(x.device), ctypes.byref(h)))
        self._h = h

    def apply(self, v, transpose=False):
        v = _dev(v, name="v").reshape(-1)
        out = torch.empty(self.m if transpose else self.n, dtype=torch.float32, device=self.device)
        _check(_lib.fs_plan_apply(self._h, _ptr(v), _ptr(out), int(bool(transpose)),
                                  _stream(self.device)))
        return out

    def apply_noalloc(self, v, out, transpose=False):
        """fs_plan_apply_noalloc: the same product into the caller's `out`, with the library's
        temporaries in its static device scratch (no allocation by the library)."""
        v = _dev(v, name="v").reshape(-1)
        nt = self.m if transpose else self.n
        if not isinstance(out, torch.Tensor) or not out.is_cuda or out.dtype != torch.float32 \
                or not out.is_contiguous() or out.numel() != nt:
            raise ValueError("out must be a contiguous float32 HIP tensor of %d elements" % nt)
        _check(_lib.fs_plan_apply_noalloc(self._h, _ptr(v), _ptr(out), int(bool(transpose)),
                                          _stream(self.device)))
        return out

    def multiplier(self):
        """fs_plan_multiplier: (M_k as a float32 array of shape (N/2+1,)*d indexed [k_d..k_1],
        phihat(k) for k = 0..N/2, torus period in data units, N)."""
        P, N = ctypes.c_double(0.0), ctypes.c_int(0)
        # first call: the sizes only (no array written)
        _check(_lib.fs_plan_multiplier(self._h, None, None, 1 << 62, ctypes.byref(P),
                                       ctypes.byref(N), _stream(self.device)))
        H = N.value // 2 + 1
        mult = np.empty((H,) * self.d, dtype=np.float32)
        phat = np.empty(H, dtype=np.float64)
        _check(_lib.fs_plan_multiplier(self._h, mult.ctypes.data_as(ctypes.c_void_p),
                                       phat.ctypes.data_as(ctypes.c_void_p), mult.size,
                                       ctypes.byref(P), ctypes.byref(N), _stream(self.device)))
        return mult, phat, P.value, N.value

    def close(self):
        if getattr(self, "_h", None):
            _lib.fs_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


def uot_sinkhorn(x, a, y, b, lam, rho, iters, kernel="gauss", grid=0, window=0, oversampling=0,
                 smoothness=0, nearfield_radius=0.0, flags=0, bandwidth=0, f0=None, g0=None):
    """Algorithm 2: `iters` sweeps; returns (f, g, dual objective).  f0/g0 warm-start."""
    x, y = _pts(x, "x"), _pts(y, "y")
    a, b = _dev(a, name="a").reshape(-1), _dev(b, name="b").reshape(-1)
    n, m = x.shape[0], y.shape[0]
    f = torch.empty(n, dtype=torch.float64, device=x.device)
    g = torch.empty(m, dtype=torch.float64, device=x.device)
    if f0 is not None or g0 is not None:
        f.copy_(f0 if f0 is not None else torch.zeros_like(f))
        g.copy_(g0 if g0 is not None else torch.zeros_like(g))
        flags |= FLAG_WARM_START
    p = _params(kernel, lam, grid, window, oversampling, smoothness, nearfield_radius, flags,
                bandwidth)
    obj = ctypes.c_double(0.0)
    _check(_lib.uot_sinkhorn(_ptr(x), _ptr(a), n, _ptr(y), _ptr(b), m, x.shape[1],
                             ctypes.byref(p), float(rho), int(iters), _ptr(f), _ptr(g),
                             ctypes.byref(obj), _stream(x.device)))
    return f, g, obj.value


def uot_upper_bound(x, a, y, b, lam, rho, kernel="gauss", grid=0, window=0, oversampling=0,
                    smoothness=0, nearfield_radius=0.0, bandwidth=0):
    """(c*, objective at c* mu x nu) of eq. (561); the objective bounds UOT from above.  For the
    r = 1 cost ("laplace") the grid settings drive one energy-kernel sum."""
    x, y = _pts(x, "x"), _pts(y, "y")
    a, b = _dev(a, name="a").reshape(-1), _dev(b, name="b").reshape(-1)
    p = _params(kernel, lam, grid, window, oversampling, smoothness, nearfield_radius, 0,
                bandwidth)
    c, ub = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _check(_lib.uot_upper_bound(_ptr(x), _ptr(a), x.shape[0], _ptr(y), _ptr(b), y.shape[0],
                                x.shape[1], ctypes.byref(p), float(rho), ctypes.byref(c),
                                ctypes.byref(ub), _stream(x.device)))
    return c.value, ub.value


def uot_sinkhorn_scaling(x, a, y, b, eps_stages, rho, max_sweeps, tol, init="zero", f0=None,
                         g0=None, kernel="gauss", grid=0, window=0, oversampling=0, smoothness=0,
                         nearfield_radius=0.0, flags=0, bandwidth=0):
    """lambda-scaling over the temperatures eps_stages; returns (f, g, sweeps per stage,
    objective).  init: "zero", "cstar" or "warm" (f0, g0)."""
    x, y = _pts(x, "x"), _pts(y, "y")
    a, b = _dev(a, name="a").reshape(-1), _dev(b, name="b").reshape(-1)
    n, m = x.shape[0], y.shape[0]
    f = torch.zeros(n, dtype=torch.float64, device=x.device)
    g = torch.zeros(m, dtype=torch.float64, device=x.device)
    if init == "warm":
        f.copy_(f0 if f0 is not None else torch.zeros_like(f))
        g.copy_(g0 if g0 is not None else torch.zeros_like(g))
    stages = (ctypes.c_double * len(eps_stages))(*[float(e) for e in eps_stages])
    counts = (ctypes.c_int * len(eps_stages))()
    p = _params(kernel, eps_stages[0], grid, window, oversampling, smoothness, nearfield_radius,
                flags, bandwidth)
    obj = ctypes.c_double(0.0)
    _check(_lib.uot_sinkhorn_scaling(_ptr(x), _ptr(a), n, _ptr(y), _ptr(b), m, x.shape[1],
                                     ctypes.byref(p), ctypes.cast(stages, ctypes.c_void_p),
                                     len(eps_stages), float(rho), int(max_sweeps), float(tol),
                                     INITS[init], _ptr(f), _ptr(g),
                                     ctypes.cast(counts, ctypes.c_void_p), ctypes.byref(obj),
                                     _stream(x.device)))
    return f, g, list(counts), obj.value


def uot_sinkhorn_grad(x, a, y, b, lam, rho, f, g, kernel="gauss", grid=0, window=0,
                      oversampling=0, smoothness=0, nearfield_radius=0.0, flags=0, bandwidth=0,
                      scale=1.0):
    """Envelope gradients (dx, da, dy, db) of the UOT value at the potentials (f, g)."""
    x, y = _pts(x, "x"), _pts(y, "y")
    a, b = _dev(a, name="a").reshape(-1), _dev(b, name="b").reshape(-1)
    f, g = _dev(f, torch.float64, "f"), _dev(g, torch.float64, "g")
    dx, dy = torch.empty_like(x), torch.empty_like(y)
    da, db = torch.empty_like(a), torch.empty_like(b)
    p = _params(kernel, lam, grid, window, oversampling, smoothness, nearfield_radius, flags,
                bandwidth)
    _check(_lib.uot_sinkhorn_grad(_ptr(x), _ptr(a), x.shape[0], _ptr(y), _ptr(b), y.shape[0],
                                  x.shape[1], ctypes.byref(p), float(rho), _ptr(f), _ptr(g),
                                  float(scale), _ptr(dx), _ptr(da), _ptr(dy), _ptr(db),
                                  _stream(x.device)))
    return dx, da, dy, db


def sinkhorn_divergence(x, a, y, b, lam, rho, iters, kernel="gauss", grid=0, window=0,
                        oversampling=0, smoothness=0, nearfield_radius=0.0, flags=0,
                        bandwidth=0, return_potentials=False):
    """eq. (586).  Returns the value (and the three UOT values), optionally the potentials."""
    x, y = _pts(x, "x"), _pts(y, "y")
    a, b = _dev(a, name="a").reshape(-1), _dev(b, name="b").reshape(-1)
    n, m = x.shape[0], y.shape[0]
    pots = [torch.empty(k, dtype=torch.float64, device=x.device) for k in (n, m, n, m)]
    p = _params(kernel, lam, grid, window, oversampling, smoothness, nearfield_radius, flags,
                bandwidth)
    val = ctypes.c_double(0.0)
    terms = (ctypes.c_double * 3)()
    _check(_lib.sinkhorn_divergence(_ptr(x), _ptr(a), n, _ptr(y), _ptr(b), m, x.shape[1],
                                    ctypes.byref(p), float(rho), int(iters), _ptr(pots[0]),
                                    _ptr(pots[1]), _ptr(pots[2]), _ptr(pots[3]),
                                    ctypes.byref(val), terms, _stream(x.device)))
    out = (val.value, tuple(terms))
    return out + (tuple(pots),) if return_potentials else out


def sinkhorn_divergence_grad(x, a, y, b, lam, rho, pots, kernel="gauss", grid=0, window=0,
                             oversampling=0, smoothness=0, nearfield_radius=0.0, flags=0,
                             bandwidth=0, scale=1.0):
    x, y = _pts(x, "x"), _pts(y, "y")
    a, b = _dev(a, name="a").reshape(-1), _dev(b, name="b").reshape(-1)
    pots = [_dev(t, torch.float64, "potential") for t in pots]
    dx, dy = torch.empty_like(x), torch.empty_like(y)
    da, db = torch.empty_like(a), torch.empty_like(b)
    p = _params(kernel, lam, grid, window, oversampling, smoothness, nearfield_radius, flags,
                bandwidth)
    _check(_lib.sinkhorn_divergence_grad(_ptr(x), _ptr(a), x.shape[0], _ptr(y), _ptr(b),
                                         y.shape[0], x.shape[1], ctypes.byref(p), float(rho),
                                         _ptr(pots[0]), _ptr(pots[1]), _ptr(pots[2]),
                                         _ptr(pots[3]), float(scale), _ptr(dx), _ptr(da),
                                         _ptr(dy), _ptr(db), _stream(x.device)))
    return dx, da, dy, db


def mmd(x, a, y, b, kernel="gauss", lam=1.0, grid=0, window=0, oversampling=0, smoothness=0,
        nearfield_radius=0.0, flags=0, bandwidth=0, terms=False):
    """Signed MMD^2 of eq. (1205); with terms=True also (sum aaK, sum abK, sum bbK)."""
    x, y = _pts(x, "x"), _pts(y, "y")
    a, b = _dev(a, name="a").reshape(-1), _dev(b, name="b").reshape(-1)
    p = _params(kernel, lam, grid, window, oversampling, smoothness, nearfield_radius, flags,
                bandwidth)
    val = ctypes.c_double(0.0)
    t3 = (ctypes.c_double * 3)()
    _check(_lib.mmd(_ptr(x), _ptr(a), x.shape[0], _ptr(y), _ptr(b), y.shape[0], x.shape[1],
                    ctypes.byref(p), ctypes.byref(val), t3 if terms else None,
                    _stream(x.device)))
    return (val.value, tuple(t3)) if terms else val.value


def mmd_grad(x, a, y, b, kernel="gauss", lam=1.0, grid=0, window=0, oversampling=0,
             smoothness=0, nearfield_radius=0.0, flags=0, bandwidth=0, scale=1.0):
    x, y = _pts(x, "x"), _pts(y, "y")
    a, b = _dev(a, name="a").reshape(-1), _dev(b, name="b").reshape(-1)
    dx, dy = torch.empty_like(x), torch.empty_like(y)
    da, db = torch.empty_like(a), torch.empty_like(b)
    p = _params(kernel, lam, grid, window, oversampling, smoothness, nearfield_radius, flags,
                bandwidth)
    _check(_lib.mmd_grad(_ptr(x), _ptr(a), x.shape[0], _ptr(y), _ptr(b), y.shape[0], x.shape[1],
                         ctypes.byref(p), float(scale), _ptr(dx), _ptr(da), _ptr(dy), _ptr(db),
                         _stream(x.device)))
    return dx, da, dy, db


class SinkhornDivergence(torch.autograd.Function):
    """S(a, b) of eq. (586) with the hand-written envelope backward (positions and weights)."""

    @staticmethod
    def forward(ctx, x, a, y, b, lam, rho, iters, opts):
        opts = dict(opts or {})
        val, _, pots = sinkhorn_divergence(x, a, y, b, lam, rho, iters, return_potentials=True,
                                           **opts)
        ctx.save_for_backward(x, a, y, b, *pots)
        ctx.cfg = (lam, rho, opts)
        return torch.tensor(val, dtype=torch.float64, device=x.device)

    @staticmethod
    def backward(ctx, gout):
        x, a, y, b, *pots = ctx.saved_tensors
        lam, rho, opts = ctx.cfg
        dx, da, dy, db = sinkhorn_divergence_grad(x, a, y, b, lam, rho, pots,
                                                  scale=float(gout.item()), **opts)
        return dx.view_as(x), da.view_as(a), dy.view_as(y), db.view_as(b), None, None, None, None


class MMD2(torch.autograd.Function):
    """Signed MMD^2 of eq. (1205) with the hand-written backward (positions and weights)."""

    @staticmethod
    def forward(ctx, x, a, y, b, opts):
        opts = dict(opts or {})
        val = mmd(x, a, y, b, **opts)
        ctx.save_for_backward(x, a, y, b)
        ctx.opts = opts
        return torch.tensor(val, dtype=torch.float64, device=x.device)

    @staticmethod
    def backward(ctx, gout):
        x, a, y, b = ctx.saved_tensors
        dx, da, dy, db = mmd_grad(x, a, y, b, scale=float(gout.item()), **ctx.opts)
        return dx.view_as(x), da.view_as(a), dy.view_as(y), db.view_as(b), None
