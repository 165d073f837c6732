"""GPU parity at the workloads' full sizes, on sampled outputs the FP64 oracle computes one by one,
and the gradient check against central differences of the oracle's converged divergence."""
import json
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2306_13618_amd as fu  # noqa: E402

DEV = torch.device("cuda:0")
TOL = 1e-5


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def relmax(got, ref):
    got, ref = np.asarray(got, float), np.asarray(ref, float)
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def last_halfstep_error(w, f, g, eps, rho, r=2, k=96):
    """The final gamma is the gamma half-step of the final beta: recompute it in FP64 for sampled
    rows (Algorithm 1's update) and compare."""
    rows = synth.sample_rows(w["m"], k, seed=3)
    ref = oracle.uot_beta_rows(w["y"], rows, w["x"], w["a"], f, eps, rho, r=r)
    return relmax(g[rows], ref)


@pytest.mark.parametrize("cfg,grid,window", [("uot_d3_n1M", 64, 6), ("uot_d2_n100k", 128, 6)])
def test_uot_full_size(cfg, grid, window):
    w = synth.make(cfg)
    print("case", cfg, w["n"], "points", w["iters"], "sweeps", flush=True)
    f, g, obj = fu.uot_sinkhorn(T(w["x"]), T(w["a"]), T(w["y"]), T(w["b"]), w["eps"], w["rho"],
                                w["iters"], kernel="gauss", grid=grid, window=window)
    f, g = f.cpu().numpy(), g.cpu().numpy()
    assert np.isfinite(obj) and np.all(np.isfinite(f)) and np.all(np.isfinite(g))
    assert last_halfstep_error(w, f, g, w["eps"], w["rho"]) < TOL


def test_uot_laplace_d3_n4M_full_size():
    """The 4M Laplace workload at full size (n = m = 4M, grid 256^3, bandwidth 192, smoothness 6,
    r = 1, near field, 50 sweeps): the final gamma against an FP64 gamma half-step of the final
    beta on sampled rows."""
    w = synth.make("laplace_d3_n4M")
    print("case laplace_d3_n4M", w["n"], "points", w["iters"], "sweeps", flush=True)
    f, g, obj = fu.uot_sinkhorn(T(w["x"]), T(w["a"]), T(w["y"]), T(w["b"]), w["eps"], w["rho"],
                                w["iters"], kernel="laplace", grid=w["grid"], window=w["window"],
                                bandwidth=w["bandwidth"], smoothness=w["smoothness"])
    f, g = f.cpu().numpy(), g.cpu().numpy()
    assert np.isfinite(obj) and np.all(np.isfinite(f)) and np.all(np.isfinite(g))
    err = last_halfstep_error(w, f, g, w["eps"], w["rho"], r=1, k=48)
    print("sampled last-half-step error %.2e" % err)
    assert err < TOL


def test_d3_n1M_fastsum_gauss_and_energy_full_size():
    w = synth.make("uot_d3_n1M")
    x, y = T(w["x"]), T(w["y"])
    rows = synth.sample_rows(w["n"], 96, seed=4)
    v = w["b"]
    got = fu.fastsum_apply(x, y, T(v), kernel="gauss", lam=w["mmd_lambda"], grid=64,
                           window=6).cpu().numpy()
    ref = oracle.direct_sum_rows(w["x"], rows, w["y"], v, "gauss", w["mmd_lambda"])
    assert relmax(got[rows], ref) < TOL
    got = fu.fastsum_apply(x, y, T(v), kernel="energy", grid=256, window=6,
                           nearfield_radius=w["nearfield_radius"]).cpu().numpy()
    ref = oracle.direct_sum_rows(w["x"], rows, w["y"], v, "energy", 1.0)
    assert relmax(got[rows], ref) < TOL


def test_d3_n1M_mmd_full_size_properties():
    """MMD(mu, mu) = 0 at full size; the two-measure value is finite and the three double sums are
    consistent with the sampled kernel sums."""
    w = synth.make("uot_d3_n1M")
    x, a, y, b = T(w["x"]), T(w["a"]), T(w["y"]), T(w["b"])
    for kind, opts in (("gauss", {"lam": w["mmd_lambda"], "grid": 64}),
                       ("energy", {"grid": 256, "nearfield_radius": w["nearfield_radius"]})):
        v0, t0 = fu.mmd(x, a, x, a, kernel=kind, window=6, terms=True, **opts)
        assert abs(v0) < 1e-6 * abs(t0[0]), kind
        v, t3 = fu.mmd(x, a, y, b, kernel=kind, window=6, terms=True, **opts)
        assert np.isfinite(v) and abs(v - (t3[0] - 2 * t3[1] + t3[2])) < 1e-12 * max(map(abs, t3))


def test_d32_n200k_mfma_full_size():
    w = synth.make("gauss_d32_n200k")
    rows = synth.sample_rows(w["n"], 64, seed=5)
    v = w["b"] / w["b"].max()
    got = fu.fastsum_apply(T(w["x"]), T(w["y"]), T(v), kernel="gauss", lam=w["eps"],
                           grid=0).cpu().numpy()
    ref = oracle.direct_sum_rows(w["x"], rows, w["y"], v, "gauss", w["eps"])
    assert relmax(got[rows], ref) < TOL


def test_d2_n200k_divergence_gradient_full_size_against_oracle_envelope():
    """Gradient of S at n=m=200k (fast path) against the FP64 direct envelope gradient at the GPU's
    potentials, on 64 sampled rows."""
    w = synth.make("divergence_d2_n200k")
    opts = {"grid": w["grid"], "window": w["window"]}
    x, a, y, b = T(w["x"]), T(w["a"]), T(w["y"]), T(w["b"])
    val, _, pots = fu.sinkhorn_divergence(x, a, y, b, w["eps"], w["rho"], 300,
                                          return_potentials=True, **opts)
    dx, da, _, _ = fu.sinkhorn_divergence_grad(x, a, y, b, w["eps"], w["rho"], pots, **opts)
    fab, gab, faa, _ = (p.cpu().numpy() for p in pots)
    rows = synth.sample_rows(w["n"], 64, seed=6)
    g1x, g1a = oracle.uot_grad_rows(w["x"], w["a"], rows, w["y"], w["b"], w["eps"], w["rho"],
                                    fab, gab)
    g2x, g2a = oracle.uot_grad_rows(w["x"], w["a"], rows, w["x"], w["a"], w["eps"], w["rho"],
                                    faa, faa)
    Ma, Mb = float(np.sum(w["a"], dtype=np.float64)), float(np.sum(w["b"], dtype=np.float64))
    refx = g1x - g2x
    refa = g1a - g2a + w["eps"] * (Ma - Mb)
    ex = relmax(dx.cpu().numpy()[rows], refx)
    ea = relmax(da.cpu().numpy()[rows], refa)
    print("divergence gradient errors: dx %.2e da %.2e" % (ex, ea))
    assert ex < 1e-4 and ea < 1e-4


def test_d2_n200k_mmd_gradient_full_size():
    w = synth.make("divergence_d2_n200k")
    x, a, y, b = T(w["x"]), T(w["a"]), T(w["y"]), T(w["b"])
    dx, da, _, _ = fu.mmd_grad(x, a, y, b, kernel="gauss", lam=w["mmd_lambda"], grid=w["grid"],
                               window=w["window"])
    rows = synth.sample_rows(w["n"], 48, seed=7)
    rx, ra = oracle.mmd2_grad_rows(w["x"], w["a"], rows, w["y"], w["b"], "gauss", w["mmd_lambda"])
    assert relmax(dx.cpu().numpy()[rows], rx) < 1e-4
    assert relmax(da.cpu().numpy()[rows], ra) < 1e-4


def test_d2_gradient_against_central_differences():
    """dS/dx and dS/da from the GPU (fast path, converged potentials) against central differences
    (h = 1e-3 in positions, 1e-3 of the mean weight in weights) of the oracle's converged FP64
    divergence, at a reduced size of the same workload."""
    w = synth.make("divergence_d2_n200k", n=320, m=300)
    eps, rho, sweeps = w["eps"], w["rho"], 700
    opts = {"grid": 128, "window": 6}
    x = T(w["x"]).requires_grad_()
    a = T(w["a"]).requires_grad_()
    s = fu.SinkhornDivergence.apply(x, a, T(w["y"]), T(w["b"]), eps, rho, sweeps, opts)
    s.backward()
    gx, ga = x.grad.cpu().numpy(), a.grad.cpu().numpy()
    rng = np.random.default_rng(11)
    coords = [(int(i), int(c)) for i, c in zip(rng.integers(0, 320, 12), rng.integers(0, 2, 12))]
    widx = [int(i) for i in rng.integers(0, 320, 6)]
    xs, as_ = w["x"].astype(np.float64), w["a"].astype(np.float64)

    def S(xx, aa):
        return oracle.sinkhorn_divergence(xx, aa, w["y"], w["b"], eps, rho, sweeps)[0]

    h = 1e-3
    fd, got = [], []
    for i, c in coords:
        xp, xm = xs.copy(), xs.copy()
        xp[i, c] += h
        xm[i, c] -= h
        fd.append((S(xp, as_) - S(xm, as_)) / (2 * h))
        got.append(gx[i, c])
    ha = 1e-3 * as_.mean()
    fda, gota = [], []
    for i in widx:
        ap, am = as_.copy(), as_.copy()
        ap[i] += ha
        am[i] -= ha
        fda.append((S(xs, ap) - S(xs, am)) / (2 * ha))
        gota.append(ga[i])
    ex, ea = relmax(got, fd), relmax(gota, fda)
    print("FD check: dx %.2e  da %.2e" % (ex, ea))
    assert ex < 1e-4 and ea < 1e-4


def test_d2_gradient_against_golden_central_differences_64_coordinates():
    """dS/dx on 64 random position coordinates and dS/da on 16 random weights of the Sinkhorn
    divergence (eq. (586)) at n = 2000, m = 1800 of the d = 2 mixture workload (eps = 0.01,
    rho = 0.5), from the GPU (fast path, SinkhornDivergence backward) against central differences
    (h = 1e-3) of the oracle's converged FP64 divergence, stored in tests/golden by the committed
    script beside it.  Error normalised by the largest |gradient| of the sample."""
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                    "divergence_fd_d2_n2000.json")))
    w = synth.make(g["workload"], n=g["n"], m=g["m"])
    x = T(w["x"]).requires_grad_()
    a = T(w["a"]).requires_grad_()
    s = fu.SinkhornDivergence.apply(x, a, T(w["y"]), T(w["b"]), g["eps"], g["rho"], g["sweeps"],
                                    {"grid": 128, "window": 6})
    s.backward()
    gx = x.grad.cpu().numpy()[np.array(g["rows"]), np.array(g["comps"])]
    ga = a.grad.cpu().numpy()[np.array(g["weight_rows"])]
    ex, ea = relmax(gx, g["fd_dx"]), relmax(ga, g["fd_da"])
    print("golden FD check (64 positions, 16 weights): dx %.2e  da %.2e" % (ex, ea))
    assert ex < 1e-4 and ea < 1e-4
