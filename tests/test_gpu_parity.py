"""GPU parity: the HIP path (through the C-ABI) against the FP64 CPU oracle on the same seeded
inputs.  Tolerance: relative error <= 1e-5 for every FP32 kernel sum and for the Sinkhorn
potentials and objective (the stated accuracy of the FP32 fast summation); sizes span several
tiles and end in ragged tails."""
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


def relinf(got, ref):
    got, ref = np.asarray(got, float), np.asarray(ref, float)
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def rel2(got, ref):
    got, ref = np.asarray(got, float), np.asarray(ref, float)
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def clouds(d, n, m, seed, spread=0.03):
    rng = np.random.default_rng([4242, d, n, m, seed])
    x = rng.uniform(-0.25, 0.25, (n, d)).astype(np.float32)
    base = x[rng.integers(0, n, m)]
    y = np.clip(base + rng.normal(0, spread, (m, d)), -0.25, synth.HI).astype(np.float32)
    v = rng.uniform(0.5, 1.5, m).astype(np.float32)
    return x, y, v


# --------------------------------------------------------------------------- direct sums

@pytest.mark.parametrize("kind,lam", [("gauss", 0.02), ("laplace", 0.05), ("energy", 1.0),
                                      ("imq", 0.3)])
@pytest.mark.parametrize("d", [1, 2, 3])
def test_direct_sum(kind, lam, d):
    x, y, v = clouds(d, 1537, 1201, 1)
    got = fu.fastsum_apply(T(x), T(y), T(v), kernel=kind, lam=lam, grid=0).cpu().numpy()
    ref = oracle.direct_sum(x, y, v, kind, lam)
    assert relinf(got, ref) < TOL


# --------------------------------------------------------------------------- NFFT fast sums

@pytest.mark.parametrize("d,grid,window,lam", [(1, 64, 6, 0.02), (2, 64, 6, 0.02),
                                               (2, 128, 4, 0.02), (3, 128, 6, 0.02),
                                               (3, 64, 6, 0.02), (3, 64, 4, 0.02),
                                               (3, 128, 5, 0.005)])
def test_fastsum_gauss(d, grid, window, lam):
    x, y, v = clouds(d, 3001, 2777, 2)
    got = fu.fastsum_apply(T(x), T(y), T(v), kernel="gauss", lam=lam, grid=grid,
                           window=window).cpu().numpy()
    ref = oracle.direct_sum(x, y, v, "gauss", lam)
    assert relinf(got, ref) < TOL


@pytest.mark.parametrize("kind,lam,d,grid", [("laplace", 0.01, 1, 256), ("laplace", 0.01, 2, 256),
                                             ("laplace", 0.01, 3, 128), ("energy", 1.0, 1, 256),
                                             ("energy", 1.0, 2, 256), ("energy", 1.0, 3, 256),
                                             ("imq", 1.0, 1, 128), ("imq", 0.5, 2, 128),
                                             ("imq", 0.05, 2, 256), ("imq", 0.02, 3, 256)])
def test_fastsum_nearfield_kernels(kind, lam, d, grid):
    x, y, v = clouds(d, 2003, 1999, 3)
    got = fu.fastsum_apply(T(x), T(y), T(v), kernel=kind, lam=lam, grid=grid,
                           window=6).cpu().numpy()
    ref = oracle.direct_sum(x, y, v, kind, lam)
    assert relinf(got, ref) < TOL


@pytest.mark.parametrize("kind,d,smooth,radius", [("energy", 3, 4, 0.0), ("laplace", 3, 6, 0.0),
                                                  ("energy", 3, 12, 0.0), ("energy", 3, 8, 1 / 16),
                                                  ("laplace", 2, 12, 0.0), ("energy", 1, 6, 0.0)])
def test_fastsum_nearfield_smoothness_and_radius(kind, d, smooth, radius):
    """Inner polynomials of 4..12 coefficients and an explicit near-field radius."""
    x, y, v = clouds(d, 2500, 2300, 8)
    lam = 0.01 if kind == "laplace" else 1.0
    got = fu.fastsum_apply(T(x), T(y), T(v), kernel=kind, lam=lam, grid=256, window=6,
                           smoothness=smooth, nearfield_radius=radius).cpu().numpy()
    ref = oracle.direct_sum(x, y, v, kind, lam)
    assert relinf(got, ref) < TOL


@pytest.mark.parametrize("cfg,kind,n,radius", [("uot_d3_n1M", "energy", 200_000, 1 / 16),
                                               ("uot_d3_n1M", "laplace", 300_000, 0.0),
                                               ("uot_d2_n100k", "energy", 150_000, 0.02)])
def test_fastsum_nearfield_dense_sampled(cfg, kind, n, radius):
    """Dense clouds (several cells per radius, uniform and clustered): sampled rows against the
    oracle's direct sums."""
    w = synth.make(cfg, n=n, m=n - 1234)
    lam = 0.01 if kind == "laplace" else 1.0
    got = fu.fastsum_apply(T(w["x"]), T(w["y"]), T(w["b"]), kernel=kind, lam=lam, grid=256,
                           window=6, nearfield_radius=radius).cpu().numpy()
    rows = synth.sample_rows(n, 64, seed=9)
    ref = oracle.direct_sum_rows(w["x"], rows, w["y"], w["b"], kind, lam)
    assert relinf(got[rows], ref) < TOL


def dense_and_sparse(n, m, seed, frac=0.8):
    """A fraction `frac` of the points in a small cube (many per grid cell), the rest spread over
    the whole box (a few per brick): full, partial and single-node matrix-core groups."""
    rng = np.random.default_rng([777, n, m, seed])

    def pts(k):
        kd = int(frac * k)
        p = np.concatenate([rng.uniform(-0.05, 0.05, (kd, 3)),
                            rng.uniform(-0.25, 0.25, (k - kd, 3))])
        return rng.permutation(p).astype(np.float32)
    return pts(n), pts(m), rng.uniform(0.5, 1.5, m).astype(np.float32)


@pytest.mark.parametrize("window,lam", [(6, 0.02), (5, 0.02), (4, 0.02)])
def test_fastsum_gauss_matrix_core_groups(window, lam):
    """3-D gather on the matrix cores (groups of up to 16 nodes per brick of 4 cells) against the
    oracle on sampled rows and against the lane-per-node kernels on every row."""
    x, y, v = dense_and_sparse(50_000, 47_001, window)
    args = dict(kernel="gauss", lam=lam, grid=64, window=window)
    got = fu.fastsum_apply(T(x), T(y), T(v), **args).cpu().numpy()
    valu = fu.fastsum_apply(T(x), T(y), T(v), flags=fu.FLAG_FORCE_VALU, **args).cpu().numpy()
    rows = synth.sample_rows(len(x), 200, seed=window)
    ref = oracle.direct_sum_rows(x, rows, y, v, "gauss", lam)
    assert relinf(got[rows], ref) < TOL
    assert relinf(got, valu) < 2e-6
    assert np.any(got != valu)  # the two paths differ in rounding: the matrix cores ran


@pytest.mark.parametrize("kind,lam", [("laplace", 0.01), ("energy", 1.0), ("imq", 0.05)])
def test_fastsum_nearfield_matrix_core_groups(kind, lam):
    """Near-field kernels with the 3-D matrix-core spread and gather (dense clusters) against the
    oracle on sampled rows and against the lane-per-node kernels on every row."""
    x, y, v = dense_and_sparse(40_000, 37_003, 11, frac=0.95)
    args = dict(kernel=kind, lam=lam, grid=128, window=6)
    got = fu.fastsum_apply(T(x), T(y), T(v), **args).cpu().numpy()
    valu = fu.fastsum_apply(T(x), T(y), T(v), flags=fu.FLAG_FORCE_VALU, **args).cpu().numpy()
    rows = synth.sample_rows(len(x), 200, seed=12)
    ref = oracle.direct_sum_rows(x, rows, y, v, kind, lam)
    assert relinf(got[rows], ref) < TOL
    assert relinf(got, valu) < 2e-6
    assert np.any(got != valu)  # the two paths differ in rounding: the matrix cores ran


@pytest.mark.parametrize("window", [2, 3])
def test_fastsum_matrix_core_small_windows(window):
    """Windows of 4 and 6 points (two matrix rows of z offsets, partly empty operand columns): the
    matrix-core spread and gather against the lane-per-node kernels on every row, and against the
    oracle's direct sums on sampled rows, where a window this short leaves its own approximation
    error: the matrix-core path may not be further from the oracle than the lane-per-node one
    (beyond the split operands' rounding)."""
    x, y, v = dense_and_sparse(30_000, 28_001, 40 + window)
    args = dict(kernel="gauss", lam=0.05, grid=64, window=window)
    got = fu.fastsum_apply(T(x), T(y), T(v), **args).cpu().numpy()
    valu = fu.fastsum_apply(T(x), T(y), T(v), flags=fu.FLAG_FORCE_VALU, **args).cpu().numpy()
    assert relinf(got, valu) < 2e-6
    assert np.any(got != valu)
    rows = synth.sample_rows(len(x), 200, seed=60 + window)
    ref = oracle.direct_sum_rows(x, rows, y, v, "gauss", 0.05)
    e_mc, e_valu = relinf(got[rows], ref), relinf(valu[rows], ref)
    print("window %d: matrix cores %.2e, lane-per-node %.2e from the oracle" % (window, e_mc, e_valu))
    assert e_mc <= e_valu + 2e-6


@pytest.mark.parametrize("n,m", [(64, 48), (17, 1), (1, 300)])
def test_fastsum_matrix_core_tiny_clusters(n, m):
    """A few points in one cluster (a handful of groups, one block per tile, blocks of the minimum
    size) against the oracle."""
    rng = np.random.default_rng([50, n, m])
    x = rng.uniform(-0.002, 0.002, (n, 3)).astype(np.float32)
    y = rng.uniform(-0.002, 0.002, (m, 3)).astype(np.float32)
    v = rng.uniform(0.5, 1.5, m).astype(np.float32)
    got = fu.fastsum_apply(T(x), T(y), T(v), kernel="gauss", lam=0.02, grid=64,
                           window=6).cpu().numpy()
    ref = oracle.direct_sum(x, y, v, "gauss", 0.02)
    assert relinf(got, ref) < TOL


@pytest.mark.parametrize("kind,lam,bandwidth", [("gauss", 0.05, 16), ("gauss", 0.05, 24),
                                                ("gauss", 0.05, 40), ("laplace", 0.05, 24),
                                                ("energy", 1.0, 40)])
def test_fastsum_bandwidth_on_64_grid(kind, lam, bandwidth):
    """3-D sums with bandwidth N on a 64^3 grid (the plane-major spectrum and the one-pass y-z
    transform) against the same band-limited sums on a 128^3 grid (three strided passes): both
    evaluate the same Fourier sum over |k| <= N/2 (and the same near field, whose radius follows
    N), up to window errors far below FP32 rounding."""
    x, y, v = clouds(3, 3001, 2777, 5)
    args = dict(kernel=kind, lam=lam, window=6, bandwidth=bandwidth)
    a = fu.fastsum_apply(T(x), T(y), T(v), grid=64, **args).cpu().numpy()
    b = fu.fastsum_apply(T(x), T(y), T(v), grid=128, **args).cpu().numpy()
    assert relinf(a, b) < 2e-6


@pytest.mark.parametrize("d,grid,bandwidth,lam", [(1, 64, 0, 0.02), (2, 128, 0, 0.01),
                                                  (3, 64, 0, 0.02), (3, 256, 192, 0.004)])
def test_plan_multiplier_against_the_gaussian_fourier_series(d, grid, bandwidth, lam):
    """Unit pin of b_k (eq. (ansatz_NFFT)): for the Gaussian exp(-|x|^2/lam) the plan's multiplier
    M_k, with its window deconvolution divided out, equals the Fourier coefficients of the
    periodised kernel sampled on the N-grid, prod_i sum_l sqrt(pi lam') exp(-pi^2 lam' (k_i +
    l N)^2) with lam' = lam / P^2 in torus units (Poisson summation).  The window transform the
    plan divides by is itself checked against the Kaiser-Bessel transform
    I0(m sqrt(b^2 - (2 pi k / G)^2)) / (G phi(0)), phi(0) = sinh(b m) / (pi m), b = pi (2 - N/G)."""
    from scipy.special import i0
    rng = np.random.default_rng([55, d, grid])
    x = rng.uniform(-0.25, 0.25, (500, d)).astype(np.float32)
    pl = fu.Plan(T(x), T(x), kernel="gauss", lam=lam, grid=grid, window=6, bandwidth=bandwidth)
    mult, phat, P, N = pl.multiplier()
    pl.close()
    assert N == (bandwidth or grid // 2)
    m, G = 6, grid
    b = np.pi * (2.0 - N / G)
    k = np.arange(N // 2 + 1)
    ref_phat = i0(m * np.sqrt(b * b - (2 * np.pi * k / G) ** 2)) / G / (np.sinh(b * m) / (np.pi * m))
    assert np.max(np.abs(phat - ref_phat) / ref_phat) < 1e-12
    lp = lam / P ** 2
    beta = sum(np.sqrt(np.pi * lp) * np.exp(-np.pi ** 2 * lp * (k + l * N) ** 2) for l in (-2, -1, 0, 1, 2))
    dec = 1.0 / (G * G * phat ** 2) * np.where(k == N // 2, 0.5, 1.0)
    ref, decd = np.ones((1,) * 0), np.ones((1,) * 0)
    for i in range(d):  # first coordinate fastest: the last array axis
        shape = [1] * d
        shape[d - 1 - i] = len(k)
        ref = ref * beta.reshape(shape)
        decd = decd * dec.reshape(shape)
    # b_k recovered from the float32 multiplier; compared on the scale of the largest coefficient
    # (the deconvolution amplifies the FP64 rounding floor of b_k near the band corner, ~1e-17)
    bk = mult.astype(np.float64) / decd
    err = np.max(np.abs(bk - ref)) / np.max(np.abs(ref))
    print("b_k vs Gaussian Fourier series: d=%d G=%d N=%d P=%.4f: %.2e" % (d, G, N, P, err))
    assert err < 1e-6


@pytest.mark.parametrize("d,grid,window,kind,lam", [(3, 64, 8, "gauss", 0.02),
                                                     (3, 64, 7, "gauss", 0.005),
                                                     (3, 64, 8, "laplace", 0.05),
                                                     (2, 128, 8, "laplace", 0.05),
                                                     (2, 128, 7, "energy", 1.0),
                                                     (1, 64, 8, "gauss", 0.02)])
def test_fastsum_wide_windows(d, grid, window, kind, lam):
    """Windows of 14 and 16 points (cutoffs 7 and 8: too wide for the matrix-core groups, so the
    lane-per-node spread and gather run with their widest boxes), with and without the near field,
    against the oracle."""
    x, y, v = clouds(d, 3000, 2777, 14)
    got = fu.fastsum_apply(T(x), T(y), T(v), kernel=kind, lam=lam, grid=grid,
                           window=window).cpu().numpy()
    assert relinf(got, oracle.direct_sum(x, y, v, kind, lam)) < TOL


def test_fastsum_3d_grid512_tile_keys():
    """A 512^3 grid: its 2^27 cells exceed the binning's cell-key space, so nodes are sorted by
    tile only and every pass takes the chunk path (lane-per-node spread and gather, the fold over
    the tiles with a chunk nearby after a clearing pass, the strided FFT passes at their largest
    size).  Both directions of one plan against the oracle."""
    x, y, v = clouds(3, 5000, 4001, 12)
    w = np.random.default_rng(13).uniform(0.5, 1.5, len(x)).astype(np.float32)
    pl = fu.Plan(T(x), T(y), kernel="gauss", lam=0.002, grid=512, window=6)
    got = pl.apply(T(v)).cpu().numpy()
    got_t = pl.apply(T(w), transpose=True).cpu().numpy()
    pl.close()
    assert relinf(got, oracle.direct_sum(x, y, v, "gauss", 0.002)) < TOL
    assert relinf(got_t, oracle.direct_sum(y, x, w, "gauss", 0.002)) < TOL


def test_plan_multiplier_reuse():
    """Plans that differ in kernel, lambda, grid, window, bandwidth or dimension, then the same
    plans again in reverse order: the multipliers M_k come from the library's cache of recent
    plans (four entries, least recently used first) for the last ones and are recomputed for the
    first ones after their eviction, and again after fs_release_cache.  The window tables are
    cached per (window, bandwidth, grid, moment-form operands): the second and third plans share
    the first one's window and grid but not its bandwidth or dimension, so a table taken from the
    wrong entry would change their window shape.  Every result against the oracle, and the later
    runs against the first."""
    x3, y3, v3 = clouds(3, 3001, 2777, 2)
    x2, y2, v2 = clouds(2, 3001, 2777, 2)
    cases = [
        ((x3, y3, v3), dict(kernel="gauss", lam=0.02, grid=64, window=6)),
        ((x3, y3, v3), dict(kernel="gauss", lam=0.02, grid=64, window=6, bandwidth=40)),
        ((x2, y2, v2), dict(kernel="gauss", lam=0.02, grid=64, window=6)),
        ((x3, y3, v3), dict(kernel="gauss", lam=0.02, grid=64, window=4)),
        ((x3, y3, v3), dict(kernel="gauss", lam=0.02, grid=128, window=6)),
        ((x3, y3, v3), dict(kernel="laplace", lam=0.01, grid=128, window=6)),
        ((x3, y3, v3), dict(kernel="gauss", lam=0.005, grid=128, window=5)),
    ]
    first = []
    for (x, y, v), args in cases:
        got = fu.fastsum_apply(T(x), T(y), T(v), **args).cpu().numpy()
        ref = oracle.direct_sum(x, y, v, args["kernel"], args["lam"])
        assert relinf(got, ref) < TOL, args
        first.append(got)
    for i in reversed(range(len(cases))):
        (x, y, v), args = cases[i]
        got = fu.fastsum_apply(T(x), T(y), T(v), **args).cpu().numpy()
        assert relinf(got, first[i]) < 2e-6, args
    # an emptied cache: the multipliers are computed again
    fu.fs_release_cache()
    (x, y, v), args = cases[-1]
    got = fu.fastsum_apply(T(x), T(y), T(v), **args).cpu().numpy()
    assert relinf(got, first[-1]) < 2e-6


@pytest.mark.parametrize("n,m,sweeps", [(8000, 7001, 10), (24000, 22001, 50)])
def test_uot_matrix_core_groups(n, m, sweeps):
    """A Sinkhorn solve whose kernel sums take the headline's kernels (3-D matrix-core spread with
    the weights formed inside, matrix-core gather with the potential update applied inside; dense
    clusters, grid 64^3, window 6, eps = 0.02, rho = 1) against the oracle's iterates, up to the
    headline's 50 sweeps (Algorithm 2).  Reports the dual residual of Table
    Accuracy_analysis2, |b~ - b|/|b| + |g~ - g|/|g|."""
    x, y, _ = dense_and_sparse(n, m, 21, frac=0.95)
    rng = np.random.default_rng(22)
    a = rng.uniform(0.5, 1.5, len(x)).astype(np.float32)
    b = rng.uniform(0.5, 1.5, len(y)).astype(np.float32)
    a, b = a / a.sum(), (1.2 * b / b.sum()).astype(np.float32)
    eps, rho = 0.02, 1.0
    print("case matrix-core UOT n=%d m=%d sweeps=%d" % (n, m, sweeps), flush=True)
    f, g, obj = fu.uot_sinkhorn(T(x), T(a), T(y), T(b), eps, rho, sweeps, kernel="gauss",
                                grid=64, window=6)
    beta, gamma = oracle.uot_sinkhorn(x, a, y, b, eps, rho, sweeps)
    D = oracle.uot_dual(x, a, y, b, eps, rho, beta, gamma)
    f, g = f.cpu().numpy(), g.cpu().numpy()
    print("dual residual %.2e (relinf f %.2e g %.2e, objective %.2e)" % (
        rel2(f, beta) + rel2(g, gamma), relinf(f, beta), relinf(g, gamma), abs(obj - D) / abs(D)))
    assert relinf(f, beta) < TOL
    assert relinf(g, gamma) < TOL
    assert abs(obj - D) < TOL * abs(D)
    fv, _, _ = fu.uot_sinkhorn(T(x), T(a), T(y), T(b), eps, rho, sweeps, kernel="gauss",
                               grid=64, window=6, flags=fu.FLAG_FORCE_VALU)
    assert np.any(fv.cpu().numpy() != f)  # the matrix cores ran


def dense_and_sparse_2d(n, m, seed, frac=0.8):
    """2-D: a fraction `frac` of the points in a small square (many per grid cell), the rest
    spread over the whole box: full, partial and single-node matrix-core groups."""
    rng = np.random.default_rng([778, n, m, seed])

    def pts(k):
        kd = int(frac * k)
        p = np.concatenate([rng.uniform(-0.03, 0.03, (kd, 2)),
                            rng.uniform(-0.25, 0.25, (k - kd, 2))])
        return rng.permutation(p).astype(np.float32)
    return pts(n), pts(m), rng.uniform(0.5, 1.5, m).astype(np.float32)


@pytest.mark.parametrize("kind,lam,grid,window", [("gauss", 0.01, 128, 6), ("gauss", 0.01, 128, 4),
                                                  ("gauss", 0.05, 64, 5), ("gauss", 0.05, 16, 3),
                                                  ("laplace", 0.01, 256, 6),
                                                  ("energy", 1.0, 256, 6)])
def test_fastsum_2d_matrix_core_groups(kind, lam, grid, window):
    """2-D spread and gather on the matrix cores (tiles of 32 or 16 cells, window widths 6..12)
    against the oracle on sampled rows and against the lane-per-node kernels on every row."""
    x, y, v = dense_and_sparse_2d(40_000, 37_001, grid + window)
    args = dict(kernel=kind, lam=lam, grid=grid, window=window)
    got = fu.fastsum_apply(T(x), T(y), T(v), **args).cpu().numpy()
    valu = fu.fastsum_apply(T(x), T(y), T(v), flags=fu.FLAG_FORCE_VALU, **args).cpu().numpy()
    rows = synth.sample_rows(len(x), 200, seed=grid)
    ref = oracle.direct_sum_rows(x, rows, y, v, kind, lam)
    if window >= 5:  # the narrow windows carry the NFFT error of their width
        assert relinf(got[rows], ref) < TOL
    assert relinf(got, valu) < 2e-6
    assert np.any(got != valu)  # the two paths differ in rounding: the matrix cores ran


def test_uot_2d_matrix_core_groups():
    """A 2-D Sinkhorn solve whose kernel sums take the matrix-core spread and gather (dense
    clusters, grid 128^2) against the oracle's iterates."""
    x, y, _ = dense_and_sparse_2d(8000, 7001, 23, frac=0.95)
    rng = np.random.default_rng(24)
    a = rng.uniform(0.5, 1.5, len(x)).astype(np.float32)
    b = rng.uniform(0.5, 1.5, len(y)).astype(np.float32)
    a, b = a / a.sum(), (1.3 * b / b.sum()).astype(np.float32)
    eps, rho, sweeps = 0.01, 0.5, 10
    f, g, obj = fu.uot_sinkhorn(T(x), T(a), T(y), T(b), eps, rho, sweeps, kernel="gauss",
                                grid=128, window=6)
    beta, gamma = oracle.uot_sinkhorn(x, a, y, b, eps, rho, sweeps)
    D = oracle.uot_dual(x, a, y, b, eps, rho, beta, gamma)
    assert relinf(f.cpu().numpy(), beta) < TOL
    assert relinf(g.cpu().numpy(), gamma) < TOL
    assert abs(obj - D) < TOL * abs(D)
    fv, _, _ = fu.uot_sinkhorn(T(x), T(a), T(y), T(b), eps, rho, sweeps, kernel="gauss",
                               grid=128, window=6, flags=fu.FLAG_FORCE_VALU)
    assert np.any(fv.cpu().numpy() != f.cpu().numpy())  # the matrix cores ran


@pytest.mark.parametrize("kind,lam,grid", [("gauss", 0.02, 64), ("energy", 1.0, 128)])
def test_mmd_matrix_core_groups(kind, lam, grid):
    """MMD^2 of dense 3-D clouds (matrix-core spread and gather) against the oracle."""
    x, y, _ = dense_and_sparse(9000, 8501, 31, frac=0.95)
    rng = np.random.default_rng(32)
    a = rng.uniform(0.5, 1.5, len(x)).astype(np.float32)
    b = rng.uniform(0.5, 1.5, len(y)).astype(np.float32)
    a, b = (a / a.sum()).astype(np.float32), (b / b.sum()).astype(np.float32)
    ref, terms = oracle.mmd2(x, a, y, b, kind, lam)
    val, t3 = fu.mmd(T(x), T(a), T(y), T(b), kernel=kind, lam=lam, grid=grid, window=6,
                     terms=True)
    for k in range(3):
        assert abs(t3[k] - terms[k]) < TOL * abs(terms[k])
    assert abs(val - ref) < TOL * max(abs(t) for t in terms)
    _, tv = fu.mmd(T(x), T(a), T(y), T(b), kernel=kind, lam=lam, grid=grid, window=6,
                   terms=True, flags=fu.FLAG_FORCE_VALU)
    assert any(tv[k] != t3[k] for k in range(3))  # the matrix cores ran


def test_fastsum_signed_weights_and_wide_gaussian():
    # a Gaussian wider than the data: the plan switches to the boundary-regularised torus
    x, y, v = clouds(2, 1500, 1300, 4)
    v = v - 1.0
    got = fu.fastsum_apply(T(x), T(y), T(v), kernel="gauss", lam=0.25, grid=128,
                           window=6).cpu().numpy()
    ref = oracle.direct_sum(x, y, v, "gauss", 0.25)
    assert relinf(got, ref) < TOL


def test_plan_adjoint_and_transpose():
    x, y, v = clouds(3, 2500, 1800, 5)
    u = np.random.default_rng(5).normal(size=2500).astype(np.float32)
    pl = fu.Plan(T(x), T(y), kernel="gauss", lam=0.02, grid=64, window=6)
    kv = pl.apply(T(v)).cpu().numpy().astype(float)
    ktu = pl.apply(T(u), transpose=True).cpu().numpy().astype(float)
    assert relinf(kv, oracle.direct_sum(x, y, v, "gauss", 0.02)) < TOL
    assert relinf(ktu, oracle.direct_sum(y, x, u, "gauss", 0.02)) < TOL
    lhs, rhs = u.astype(float) @ kv, ktu @ v.astype(float)
    assert abs(lhs - rhs) < 1e-5 * (np.abs(u) @ np.abs(kv))


def test_fastsum_edge_cases():
    x, y, v = clouds(2, 40, 30, 6)
    # no sources: zero output
    out = fu.fastsum_apply(T(x), T(y[:0]), T(v[:0]), kernel="gauss", lam=0.05, grid=64)
    assert float(out.abs().max()) == 0.0
    # no targets
    out = fu.fastsum_apply(T(x[:0]), T(y), T(v), kernel="gauss", lam=0.05, grid=64)
    assert out.numel() == 0
    # a single source and target
    got = fu.fastsum_apply(T(x[:1]), T(y[:1]), T(v[:1]), kernel="gauss", lam=0.05, grid=64)
    ref = oracle.direct_sum(x[:1], y[:1], v[:1], "gauss", 0.05)
    assert relinf(got.cpu().numpy(), ref) < TOL
    # all points at one location (degenerate bounding box)
    xs = np.zeros((50, 3), np.float32) + 0.1
    got = fu.fastsum_apply(T(xs), T(xs), T(np.ones(50, np.float32)), kernel="gauss", lam=0.05,
                           grid=32).cpu().numpy()
    assert np.allclose(got, 50.0, rtol=TOL)
    # a 3-D set binned into matrix-core groups with an empty or a one-point partner set (both
    # sets are binned around one synchronisation, the empty one with no node kernels)
    x3, y3, v3 = dense_and_sparse(20_000, 18_001, 41, frac=0.95)
    kw = dict(kernel="gauss", lam=0.02, grid=64, window=6)
    out = fu.fastsum_apply(T(x3), T(y3[:0]), T(v3[:0]), **kw)
    assert out.numel() == len(x3) and float(out.abs().max()) == 0.0
    out = fu.fastsum_apply(T(x3[:0]), T(y3), T(v3), **kw)
    assert out.numel() == 0
    rows = synth.sample_rows(len(x3), 64, seed=3)
    got = fu.fastsum_apply(T(x3), T(y3[:1]), T(v3[:1]), **kw).cpu().numpy()
    assert relinf(got[rows], oracle.direct_sum_rows(x3, rows, y3[:1], v3[:1], "gauss", 0.02)) < TOL
    got = fu.fastsum_apply(T(x3[:1]), T(y3), T(v3), **kw).cpu().numpy()
    assert relinf(got, oracle.direct_sum(x3[:1], y3, v3, "gauss", 0.02)) < TOL


@pytest.mark.parametrize("case", ["gauss_d3_matrix_cores", "laplace_d3_near_field",
                                  "gauss_d2_matrix_cores", "energy_d1"])
def test_deterministic_mode_is_bitwise_reproducible(case):
    """FS_FLAG_DETERMINISTIC: nodes sharing a cell keep their input order (stable radix-sorted
    ranks instead of the atomic counters), the near field adds no partial sums through atomics,
    so two runs on the same inputs agree bit for bit, with another workload run in between; the
    results stay within the tolerance of the oracle."""
    flags = fu.FLAG_DETERMINISTIC
    if case == "gauss_d3_matrix_cores":
        x, y, _ = dense_and_sparse(20_000, 18_001, 31, frac=0.95)
        kw = dict(kernel="gauss", grid=64, window=6)
        eps, rho, r = 0.02, 1.0, 2
    elif case == "laplace_d3_near_field":
        w = synth.make("laplace_d3_n4M", n=30_000, m=28_000)
        x, y = w["x"], w["y"]
        kw = dict(kernel="laplace", grid=128, window=6)
        eps, rho, r = 0.01, 1.0, 1
    elif case == "gauss_d2_matrix_cores":
        x, y, _ = dense_and_sparse_2d(30_000, 27_003, 32, frac=0.95)
        kw = dict(kernel="gauss", grid=128, window=6)
        eps, rho, r = 0.01, 0.5, 2
    else:
        rng = np.random.default_rng(33)
        x = rng.uniform(-0.25, 0.25, (4000, 1)).astype(np.float32)
        y = rng.uniform(-0.25, 0.25, (3500, 1)).astype(np.float32)
        kw = dict(kernel="energy", grid=256, window=6)
    rng = np.random.default_rng(34)
    a = rng.uniform(0.5, 1.5, len(x)).astype(np.float32)
    b = rng.uniform(0.5, 1.5, len(y)).astype(np.float32)
    a, b = (a / a.sum()).astype(np.float32), (1.2 * b / b.sum()).astype(np.float32)
    other = clouds(3, 50_000, 40_000, 5)

    def run():
        out = fu.fastsum_apply(T(x), T(y), T(b), lam=1.0 if kw["kernel"] == "energy" else 0.05,
                               flags=flags, **kw)
        if kw["kernel"] == "energy":
            return [out]
        f, g, obj = fu.uot_sinkhorn(T(x), T(a), T(y), T(b), eps, rho, 5, flags=flags, **kw)
        return [out, f, g, torch.tensor([obj], dtype=torch.float64)]

    first = [t.cpu() for t in run()]
    fu.fastsum_apply(T(other[0]), T(other[1]), T(other[2]), kernel="laplace", lam=0.01, grid=128,
                     window=6)
    second = [t.cpu() for t in run()]
    for p, q in zip(first, second):
        assert torch.equal(p, q)
    lam = 1.0 if kw["kernel"] == "energy" else 0.05
    rows = synth.sample_rows(len(x), 64, seed=7)
    ref = oracle.direct_sum_rows(x, rows, y, b, kw["kernel"], lam)
    assert relinf(first[0].numpy()[rows], ref) < TOL
    if kw["kernel"] != "energy":
        beta, gamma = oracle.uot_sinkhorn(x, a, y, b, eps, rho, 5, r=r)
        assert relinf(first[1].numpy(), beta) < TOL and relinf(first[2].numpy(), gamma) < TOL


def test_failure_paths_report_and_recover(monkeypatch):
    """Failure handling, forced from the host: (1) zero source weights make every Sinkhorn kernel
    sum zero, so the update's count of non-positive sums reports FS_ENUMERIC (fast fused path,
    fast path with the near field, direct path), also from the side-by-side terms of a divergence;
    (2) the workspace limit of the failure-injection hook refuses an allocation inside the plan
    build, reported as FS_ENOMEM.  After each failure the library still computes correct sums."""
    w = synth.make("uot_d3_n1M", n=20_000, m=18_000)
    x, a, y = T(w["x"]), T(w["a"]), T(w["y"])
    zero = torch.zeros(18_000, dtype=torch.float32, device=DEV)
    for kw in (dict(kernel="gauss", grid=64, window=6), dict(kernel="laplace", grid=128, window=6),
               dict(kernel="gauss", grid=0)):
        lam = 0.02 if kw["kernel"] == "gauss" else 0.01
        with pytest.raises(fu.FastsumError, match="status -5"):
            fu.uot_sinkhorn(x, a, y, zero, lam, 1.0, 3, **kw)
    # the divergence's terms run in three threads: the failing (b, b) term reports from its own
    # thread, and the call returns only after all three have ended
    with pytest.raises(fu.FastsumError, match="status -5"):
        fu.sinkhorn_divergence(x, a, y, zero, 0.02, 1.0, 3, kernel="gauss", grid=64, window=6)
    monkeypatch.setenv("FASTUOT_WORKSPACE_LIMIT", str(1 << 20))
    with pytest.raises(fu.FastsumError, match="status -3.*FASTUOT_WORKSPACE_LIMIT"):
        fu.fastsum_apply(x, y, T(w["b"]), kernel="gauss", lam=0.02, grid=64, window=6)
    monkeypatch.delenv("FASTUOT_WORKSPACE_LIMIT")
    got = fu.fastsum_apply(x, y, T(w["b"]), kernel="gauss", lam=0.02, grid=64,
                           window=6).cpu().numpy()
    rows = synth.sample_rows(20_000, 64, seed=8)
    assert relinf(got[rows], oracle.direct_sum_rows(w["x"], rows, w["y"], w["b"], "gauss",
                                                    0.02)) < TOL


def test_bad_arguments_raise():
    x, y, v = clouds(2, 40, 30, 7)
    with pytest.raises(fu.FastsumError):
        fu.fastsum_apply(T(x), T(y), T(v), kernel="gauss", lam=0.05, grid=100)  # not 2^k
    with pytest.raises(fu.FastsumError):
        fu.fastsum_apply(T(x), T(y), T(v), kernel="gauss", lam=-1.0, grid=64)
    bad = x.copy()
    bad[3, 1] = np.nan
    with pytest.raises(fu.FastsumError):
        fu.fastsum_apply(T(bad), T(y), T(v), kernel="gauss", lam=0.05, grid=64)
    x4 = np.zeros((10, 4), np.float32)
    with pytest.raises(fu.FastsumError):
        fu.fastsum_apply(T(x4), T(x4), T(np.ones(10, np.float32)), kernel="gauss", lam=0.05,
                         grid=64)


# --------------------------------------------------------------------------- MFMA direct path

@pytest.mark.parametrize("n,m", [(1000, 777), (64, 33)])
def test_mfma_gram_gauss_d32(n, m):
    w = synth.make("gauss_d32_n200k", n=n, m=m)
    v = w["b"] / w["b"].max()
    got = fu.fastsum_apply(T(w["x"]), T(w["y"]), T(v), kernel="gauss", lam=1.0,
                           grid=0).cpu().numpy()
    ref = oracle.direct_sum(w["x"], w["y"], v, "gauss", 1.0)
    assert relinf(got, ref) < TOL
    valu = fu.fastsum_apply(T(w["x"]), T(w["y"]), T(v), kernel="gauss", lam=1.0, grid=0,
                            flags=fu.FLAG_FORCE_VALU).cpu().numpy()
    assert relinf(valu, ref) < TOL


@pytest.mark.parametrize("d,n,m,lam", [(16, 2100, 1900, 0.5), (64, 1500, 3333, 2.0),
                                       (128, 700, 650, 4.0), (32, 40, 5000, 1.0)])
def test_mfma_gram_gauss_other_dims(d, n, m, lam):
    rng = np.random.default_rng([77, d, n, m])
    x = (rng.normal(size=(n, d)) / np.sqrt(d)).astype(np.float32)
    y = (rng.normal(0.1, 1.0, size=(m, d)) / np.sqrt(d)).astype(np.float32)
    v = rng.uniform(0.5, 1.5, m).astype(np.float32)
    got = fu.fastsum_apply(T(x), T(y), T(v), kernel="gauss", lam=lam, grid=0).cpu().numpy()
    ref = oracle.direct_sum(x, y, v, "gauss", lam)
    assert relinf(got, ref) < TOL
    # the transposed roles through a plan
    u = rng.uniform(0.5, 1.5, n).astype(np.float32)
    pl = fu.Plan(T(x), T(y), kernel="gauss", lam=lam, grid=0)
    assert relinf(pl.apply(T(u), transpose=True).cpu().numpy(),
                  oracle.direct_sum(y, x, u, "gauss", lam)) < TOL


@pytest.mark.parametrize("lam", [0.1, 0.05, 0.02])
def test_direct_d32_small_lambda(lam):
    """Narrow Gaussians at d = 32: the matrix-core exponent's error grows with
    (R_x + R_y)^2 / lambda, so the library takes the FP32 VALU kernel where that arithmetic would
    miss 1e-5.  Kernel sums and a short Sinkhorn solve (eps = lambda) against the oracle."""
    w = synth.make("gauss_d32_n200k", n=1500, m=1300)
    v = w["b"] / w["b"].max()
    got = fu.fastsum_apply(T(w["x"]), T(w["y"]), T(v), kernel="gauss", lam=lam,
                           grid=0).cpu().numpy()
    ref = oracle.direct_sum(w["x"], w["y"], v, "gauss", lam)
    assert relinf(got, ref) < TOL
    f, g, obj = fu.uot_sinkhorn(T(w["x"]), T(w["a"]), T(w["y"]), T(w["b"]), lam, w["rho"], 5,
                                kernel="gauss", grid=0)
    beta, gamma = oracle.uot_sinkhorn(w["x"], w["a"], w["y"], w["b"], lam, w["rho"], 5)
    assert relinf(f.cpu().numpy(), beta) < TOL
    assert relinf(g.cpu().numpy(), gamma) < TOL


@pytest.mark.parametrize("d,kind", [(2, "gauss"), (3, "laplace"), (20, "gauss")])
def test_uot_direct_rows_far_from_every_source(d, kind):
    """Direct Sinkhorn at a temperature where every kernel value of some rows underflows FP32
    (two clusters 0.6 apart, eps = 0.002 for the Gaussian): the log-domain direct sums keep those
    rows, and the potentials match the oracle's log-sum-exp iteration."""
    rng = np.random.default_rng([17, d])
    n, m = 700, 600
    x = rng.normal(0, 0.02, (n, d))
    x[: n // 5] += 0.6 / np.sqrt(d)
    y = rng.normal(0, 0.02, (m, d))
    x, y = x.astype(np.float32), y.astype(np.float32)
    a = rng.uniform(0.5, 1.5, n).astype(np.float32)
    b = rng.uniform(0.5, 1.5, m).astype(np.float32)
    a, b = (a / a.sum()).astype(np.float32), (1.2 * b / b.sum()).astype(np.float32)
    eps, rho, r = (0.002, 1.0, 2) if kind == "gauss" else (0.004, 1.0, 1)
    f, g, obj = fu.uot_sinkhorn(T(x), T(a), T(y), T(b), eps, rho, 8, kernel=kind, grid=0)
    beta, gamma = oracle.uot_sinkhorn(x, a, y, b, eps, rho, 8, r=r)
    assert relinf(f.cpu().numpy(), beta) < TOL
    assert relinf(g.cpu().numpy(), gamma) < TOL
    D = oracle.uot_dual(x, a, y, b, eps, rho, beta, gamma, r=r)
    assert abs(obj - D) <= TOL * abs(D)


def _structured_d32(kind, n, m, seed):
    rng = np.random.default_rng([91, n, m, seed])
    d = 32
    if kind == "clustered":
        c = rng.normal(size=(8, d)) / np.sqrt(d)
        x = c[rng.integers(0, 8, n)] + 0.05 * rng.normal(size=(n, d)) / np.sqrt(d)
        y = c[rng.integers(0, 8, m)] + 0.05 * rng.normal(size=(m, d)) / np.sqrt(d)
    else:  # far from the origin: the common centre removes the offset
        x = 0.3 * rng.normal(size=(n, d)) / np.sqrt(d) + 3.0
        y = 0.3 * rng.normal(size=(m, d)) / np.sqrt(d) + 3.0
    return (x.astype(np.float32), y.astype(np.float32),
            rng.uniform(0.5, 1.5, m).astype(np.float32))


@pytest.mark.parametrize("kind,lam", [("clustered", 0.5), ("clustered", 0.25),
                                      ("shifted", 0.2), ("shifted", 0.05)])
def test_mfma_gram_structured_clouds(kind, lam):
    """Clustered clouds (near pairs whose exponent cancels large norm terms) and clouds far from
    the origin, at widths where the matrix-core path is taken: within 1e-5 of the oracle, and the
    matrix cores ran (the result differs in rounding from the VALU kernel's)."""
    x, y, v = _structured_d32(kind, 1700, 1400, int(100 * lam))
    got = fu.fastsum_apply(T(x), T(y), T(v), kernel="gauss", lam=lam, grid=0).cpu().numpy()
    valu = fu.fastsum_apply(T(x), T(y), T(v), kernel="gauss", lam=lam, grid=0,
                            flags=fu.FLAG_FORCE_VALU).cpu().numpy()
    ref = oracle.direct_sum(x, y, v, "gauss", lam)
    assert relinf(got, ref) < TOL
    assert relinf(valu, ref) < TOL
    assert np.any(got != valu)


def test_plan_apply_on_two_streams():
    """fs_plan_apply is stream-ordered and returns without waiting: two plans (a d = 32
    matrix-core direct plan and a 3-D NFFT plan) applied alternately on two streams, with new
    inputs each time and no synchronisation in between; every result against the oracle."""
    w32 = synth.make("gauss_d32_n200k", n=1500, m=1300)
    x3, y3, _ = clouds(3, 6000, 5000, 9)
    p32 = fu.Plan(T(w32["x"]), T(w32["y"]), kernel="gauss", lam=1.0, grid=0)
    p3 = fu.Plan(T(x3), T(y3), kernel="gauss", lam=0.02, grid=64, window=6)
    rng = np.random.default_rng(123)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    ins, outs = [], []
    for it in range(4):
        v32 = rng.uniform(0.5, 1.5, len(w32["y"])).astype(np.float32)
        v3 = rng.uniform(0.5, 1.5, len(y3)).astype(np.float32)
        t32, t3 = T(v32), T(v3)
        torch.cuda.synchronize()
        with torch.cuda.stream(s1):
            o32 = p32.apply(t32)
        with torch.cuda.stream(s2):
            o3 = p3.apply(t3)
        ins.append((v32, v3, t32, t3))
        outs.append((o32, o3))
    torch.cuda.synchronize()
    rows = synth.sample_rows(len(x3), 150, seed=3)
    for (v32, v3, _, _), (o32, o3) in zip(ins, outs):
        assert relinf(o32.cpu().numpy(), oracle.direct_sum(w32["x"], w32["y"], v32, "gauss", 1.0)) < TOL
        assert relinf(o3.cpu().numpy()[rows],
                      oracle.direct_sum_rows(x3, rows, y3, v3, "gauss", 0.02)) < TOL
    p32.close()
    p3.close()


def test_uot_mfma_d32():
    """The d = 32 Sinkhorn on the MFMA path (Gibbs kernel exp(-|x-y|^2/eps)) against the oracle."""
    w = synth.make("gauss_d32_n200k", n=1500, m=1300)
    f, g, obj = fu.uot_sinkhorn(T(w["x"]), T(w["a"]), T(w["y"]), T(w["b"]), w["eps"], w["rho"],
                                10, kernel="gauss", grid=0)
    beta, gamma = oracle.uot_sinkhorn(w["x"], w["a"], w["y"], w["b"], w["eps"], w["rho"], 10)
    assert relinf(f.cpu().numpy(), beta) < TOL
    assert relinf(g.cpu().numpy(), gamma) < TOL


# --------------------------------------------------------------------------- Sinkhorn

_cache = {}


def oracle_uot(key, x, a, y, b, eps, rho, sweeps, r=2):
    if key not in _cache:
        beta, gamma = oracle.uot_sinkhorn(x, a, y, b, eps, rho, sweeps, r=r)
        D = oracle.uot_dual(x, a, y, b, eps, rho, beta, gamma, r=r)
        _cache[key] = (beta, gamma, D)
    return _cache[key]


@pytest.mark.parametrize("grid", [0, 64])
def test_uot_d1_n2k(grid):
    """The 1-D workload in full: d=1, n=m=2000, 200 sweeps, eps=0.05, rho=1 (the paper's lambda=20,
    eta=1)."""
    w = synth.make("uot_d1_n2k")
    beta, gamma, D = oracle_uot("uot_d1_n2k", w["x"], w["a"], w["y"], w["b"], w["eps"], w["rho"],
                                w["iters"])
    f, g, obj = fu.uot_sinkhorn(T(w["x"]), T(w["a"]), T(w["y"]), T(w["b"]), w["eps"], w["rho"],
                                w["iters"], kernel="gauss", grid=grid, window=6)
    f, g = f.cpu().numpy(), g.cpu().numpy()
    assert rel2(f, beta) < TOL and rel2(g, gamma) < TOL
    assert abs(obj - D) < TOL * abs(D)


@pytest.mark.parametrize("cfg,n,sweeps,grid,window", [("uot_d2_n100k", 3000, 30, 128, 6),
                                                      ("uot_d3_n1M", 2500, 20, 64, 6),
                                                      ("uot_d3_n1M", 2500, 20, 64, 4)])
def test_uot_reduced(cfg, n, sweeps, grid, window):
    w = synth.make(cfg, n=n, m=n - 217)
    beta, gamma, D = oracle_uot((cfg, n, sweeps), w["x"], w["a"], w["y"], w["b"], w["eps"],
                                w["rho"], sweeps)
    f, g, obj = fu.uot_sinkhorn(T(w["x"]), T(w["a"]), T(w["y"]), T(w["b"]), w["eps"], w["rho"],
                                sweeps, kernel="gauss", grid=grid, window=window)
    f, g = f.cpu().numpy(), g.cpu().numpy()
    assert rel2(f, beta) < TOL and rel2(g, gamma) < TOL
    assert abs(obj - D) < TOL * abs(D)


def test_uot_laplace_4M_plan_reduced():
    """The 4M Laplace workload's plan (grid 256^3, bandwidth N = 192, i.e. a non-integer
    oversampling 4/3, smoothness 8, window 6, default near-field radius p/N; r = 1 Gibbs kernel
    exp(-|x-y|/eps), eps = 0.01) at reduced n: 10 sweeps against the oracle's iterates, with the
    dual residual of Table Accuracy_analysis2.  At this sparse size most of every sum comes from
    the smooth part, whose regularisation error with smoothness 6 (4.5e-6 of the largest sum)
    drove the potentials to 2e-5 after 10 sweeps; smoothness 8 gives 3e-7 and 1.5e-6."""
    w = synth.make("laplace_d3_n4M", n=2000, m=1800)
    sweeps = 10
    beta, gamma, D = oracle_uot("laplace_d3_n4M-small", w["x"], w["a"], w["y"], w["b"], w["eps"],
                                w["rho"], sweeps, r=1)
    f, g, obj = fu.uot_sinkhorn(T(w["x"]), T(w["a"]), T(w["y"]), T(w["b"]), w["eps"], w["rho"],
                                sweeps, kernel="laplace", grid=w["grid"], window=w["window"],
                                bandwidth=w["bandwidth"], smoothness=w["smoothness"])
    f, g = f.cpu().numpy(), g.cpu().numpy()
    print("dual residual %.2e" % (rel2(f, beta) + rel2(g, gamma)))
    assert relinf(f, beta) < TOL and relinf(g, gamma) < TOL
    assert abs(obj - D) < TOL * abs(D)


@pytest.mark.parametrize("grid", [128, 256])
def test_uot_laplace_rows_far_from_the_mass(grid):
    """r = 1 Gibbs kernel on the 2-D mixture clouds (eps = 0.01, rho = 0.5): many targets lie far
    from every source (sums down to 1e-5 of the largest), where the update takes the direct
    re-evaluation; 40 sweeps against the oracle's iterates."""
    w = synth.make("divergence_d2_n200k", n=1200, m=1000)
    eps, rho, sweeps = w["eps"], w["rho"], 40
    beta, gamma, D = oracle_uot("mixture-laplace-1200", w["x"], w["a"], w["y"], w["b"], eps, rho,
                                sweeps, r=1)
    f, g, obj = fu.uot_sinkhorn(T(w["x"]), T(w["a"]), T(w["y"]), T(w["b"]), eps, rho, sweeps,
                                kernel="laplace", grid=grid, window=6)
    f, g = f.cpu().numpy(), g.cpu().numpy()
    assert relinf(f, beta) < TOL and relinf(g, gamma) < TOL
    assert abs(obj - D) < TOL * abs(D)


def test_uot_laplace_gibbs_kernel():
    """r = 1: Gibbs kernel exp(-|x-y|/eps) through the near-field-corrected fast sum."""
    w = synth.make("laplace_d3_n4M", n=2000, m=1800)
    sweeps = 10
    beta, gamma, D = oracle_uot("laplace_d3_n4M-small", w["x"], w["a"], w["y"], w["b"], w["eps"],
                                w["rho"], sweeps, r=1)
    for grid in (0, 128):
        f, g, obj = fu.uot_sinkhorn(T(w["x"]), T(w["a"]), T(w["y"]), T(w["b"]), w["eps"],
                                    w["rho"], sweeps, kernel="laplace", grid=grid, window=6)
        f, g = f.cpu().numpy(), g.cpu().numpy()
        assert rel2(f, beta) < TOL and rel2(g, gamma) < TOL, grid
        assert abs(obj - D) < TOL * abs(D), grid


@pytest.mark.parametrize("kind,grid", [("gauss", 0), ("laplace", 0), ("laplace", 256),
                                       ("gauss", 128)])
def test_uot_upper_bound(kind, grid):
    """c* of eq. (561) and the objective at c* mu x nu against the oracle (r = 2 from moments,
    r = 1 through an energy-kernel sum)."""
    w = synth.make("divergence_d2_n200k", n=2000, m=1700)
    r = 2 if kind == "gauss" else 1
    c, ub = fu.uot_upper_bound(T(w["x"]), T(w["a"]), T(w["y"]), T(w["b"]), w["eps"], w["rho"],
                               kernel=kind, grid=grid, window=6)
    cref, ubref = oracle.uot_cstar(w["x"], w["a"], w["y"], w["b"], w["eps"], w["rho"], r=r)
    assert abs(c - cref) < 1e-6 * abs(cref)
    assert abs(ub - ubref) < 1e-6 * abs(ubref)
    # it bounds the solved problem's value from above
    _, _, obj = fu.uot_sinkhorn(T(w["x"]), T(w["a"]), T(w["y"]), T(w["b"]), w["eps"], w["rho"],
                                200, kernel=kind, grid=0)
    assert obj <= ub


@pytest.mark.parametrize("grid,init", [(0, "zero"), (0, "cstar"), (128, "zero"), (128, "cstar")])
def test_uot_scaling_against_oracle(grid, init):
    """lambda-scaling: temperatures 1, 0.05, 0.01 with warm starts and the per-sweep stopping rule.
    The sweep counts agree with the oracle's under the same rule (the FP32 kernel sums put a noise
    floor under the measured change, so a stage may run a few sweeps longer); the potentials
    agree with the oracle's iterate after the same number of sweeps per stage."""
    w = synth.make("divergence_d2_n200k", n=900, m=800)
    stages, rho, tol = [1.0, 0.05, 0.01], 1.0, 1e-6
    f, g, counts, obj = fu.uot_sinkhorn_scaling(T(w["x"]), T(w["a"]), T(w["y"]), T(w["b"]), stages,
                                                rho, 3000, tol, init=init, grid=grid, window=6)
    _, _, cref = oracle.uot_sinkhorn_scaling(w["x"], w["a"], w["y"], w["b"], stages, rho, 3000,
                                             tol, init=init)
    print("sweeps per stage: GPU", counts, "oracle", cref)
    assert all(abs(c1 - c2) <= max(2, c2 // 10) for c1, c2 in zip(counts, cref))
    # the oracle's iterate after the GPU's sweep counts, stage by stage
    bref, gref, _ = oracle.uot_sinkhorn_scaling(w["x"], w["a"], w["y"], w["b"], stages[:1], rho,
                                                counts[0], 0.0, init=init)
    for eps, c in zip(stages[1:], counts[1:]):
        bref, gref, _ = oracle.uot_sinkhorn_scaling(w["x"], w["a"], w["y"], w["b"], [eps], rho, c,
                                                    0.0, init="warm", beta0=bref, gamma0=gref)
    assert relinf(f.cpu().numpy(), bref) < 1e-5 and relinf(g.cpu().numpy(), gref) < 1e-5
    dref = oracle.uot_dual(w["x"], w["a"], w["y"], w["b"], stages[-1], rho, bref, gref)
    assert abs(obj - dref) < 1e-6 * abs(dref)


def test_uot_scaling_single_stage_is_uot_sinkhorn():
    w = synth.make("divergence_d2_n200k", n=700, m=650)
    args = (T(w["x"]), T(w["a"]), T(w["y"]), T(w["b"]))
    f1, g1, c1, o1 = fu.uot_sinkhorn_scaling(*args, [0.05], 1.0, 25, 0.0, grid=0)
    f2, g2, o2 = fu.uot_sinkhorn(*args, 0.05, 1.0, 25, grid=0)
    assert c1 == [25]
    assert relinf(f1.cpu().numpy(), f2.cpu().numpy()) < 1e-12
    assert relinf(g1.cpu().numpy(), g2.cpu().numpy()) < 1e-12 and abs(o1 - o2) < 1e-12 * abs(o2)


@pytest.mark.parametrize("d", [2, 3])
def test_tolerance_stop_is_the_fixed_sweep_solve(d):
    """A solve that stops on its tolerance after k sweeps ends in the state of the solve of exactly
    k sweeps, bit for bit in deterministic mode.  On fused half-steps (matrix-core clusters) the
    change of a sweep is read back one sweep late and the sweep queued meanwhile is undone, so
    this pins the stop sweep, the restored potentials and the objective."""
    flags = fu.FLAG_DETERMINISTIC
    if d == 2:
        x, y, _ = dense_and_sparse_2d(30_000, 27_003, 51, frac=0.95)
        kw = dict(kernel="gauss", grid=128, window=6)
        eps, rho = 0.01, 0.5
    else:
        x, y, _ = dense_and_sparse(20_000, 18_001, 52, frac=0.95)
        kw = dict(kernel="gauss", grid=64, window=6)
        eps, rho = 0.02, 1.0
    rng = np.random.default_rng(53)
    a = rng.uniform(0.5, 1.5, len(x)).astype(np.float32)
    b = rng.uniform(0.5, 1.5, len(y)).astype(np.float32)
    a, b = (a / a.sum()).astype(np.float32), (1.2 * b / b.sum()).astype(np.float32)
    args = (T(x), T(a), T(y), T(b))
    f1, g1, counts, o1 = fu.uot_sinkhorn_scaling(*args, [eps], rho, 400, 1e-3, flags=flags, **kw)
    k = counts[0]
    assert 2 < k < 400  # stopped by the tolerance, with sweeps queued ahead of the check
    f2, g2, o2 = fu.uot_sinkhorn(*args, eps, rho, k, flags=flags, **kw)
    assert torch.equal(f1, f2) and torch.equal(g1, g2) and o1 == o2


def test_uot_warm_start_continues_the_iteration():
    w = synth.make("uot_d1_n2k", n=700, m=650)
    x, a, y, b = (T(w[k]) for k in ("x", "a", "y", "b"))
    f1, g1, _ = fu.uot_sinkhorn(x, a, y, b, w["eps"], w["rho"], 7, grid=64)
    f2, g2, o2 = fu.uot_sinkhorn(x, a, y, b, w["eps"], w["rho"], 5, grid=64, f0=f1, g0=g1)
    beta, gamma = oracle.uot_sinkhorn(w["x"], w["a"], w["y"], w["b"], w["eps"], w["rho"], 12)
    assert rel2(f2.cpu().numpy(), beta) < TOL and rel2(g2.cpu().numpy(), gamma) < TOL


def test_uot_objective_without_sweeps():
    w = synth.make("uot_d1_n2k", n=300, m=280)
    _, _, obj = fu.uot_sinkhorn(T(w["x"]), T(w["a"]), T(w["y"]), T(w["b"]), w["eps"], w["rho"], 0)
    D = oracle.uot_dual(w["x"], w["a"], w["y"], w["b"], w["eps"], w["rho"], np.zeros(300),
                        np.zeros(280))
    assert abs(obj - D) < TOL * abs(D)


def test_sinkhorn_divergence():
    w = synth.make("divergence_d2_n200k", n=900, m=800)
    sweeps = 60
    sd, terms = oracle.sinkhorn_divergence(w["x"], w["a"], w["y"], w["b"], w["eps"], w["rho"],
                                           sweeps)
    for grid in (0, 128):
        val, t3 = fu.sinkhorn_divergence(T(w["x"]), T(w["a"]), T(w["y"]), T(w["b"]), w["eps"],
                                         w["rho"], sweeps, grid=grid, window=6)
        for k in range(3):
            assert abs(t3[k] - terms[k]) < TOL * abs(terms[k])
        assert abs(val - sd) < 1e-4 * abs(sd) + 1e-5 * max(abs(t) for t in terms)


# --------------------------------------------------------------------------- MMD

@pytest.mark.parametrize("eps,eta", [(1.0, 1.0), (1.0, 100.0), (10.0, 1e4)])
def test_divergence_energy_limit_experiment(eps, eta):
    """The setup of the Corollary 477 experiment (1-D uniform probability measures, r = 1 cost):
    GPU sd_{1;eta;lambda} and energy MMD^2 against the oracle.  The FP32 kernel sums resolve the
    UOT terms to ~1e-7 of their size, so sd (a difference of terms) is judged against the largest
    term."""
    rng = np.random.default_rng([1450, 7])
    n = 1500
    x = rng.uniform(0, 1, (n, 1)).astype(np.float32)
    y = rng.uniform(0, 1, (n, 1)).astype(np.float32)
    a = np.full(n, 1.0 / n, np.float32)
    sd, terms = fu.sinkhorn_divergence(T(x), T(a), T(y), T(a), eps, eta, 300, kernel="laplace",
                                       grid=256, window=6)
    sdr, tr = oracle.sinkhorn_divergence(x, a, y, a, eps, eta, 300, r=1)
    scale = max(abs(t) for t in tr)
    print("sd GPU %.9g oracle %.9g (terms up to %.3g): error %.2e of the largest term, %.2e of sd"
          % (sd, sdr, scale, abs(sd - sdr) / scale, abs(sd - sdr) / abs(sdr)))
    # the terms' FP32 floor (measured 2e-7 to 8e-7 of the largest term for eps = 1 ... 10) bounds
    # the error of sd, which is ~1e-3 of the terms here.  By eq. (995) a half-step adds
    # eta / (1 + eta lambda) times the sums' relative rounding to a potential and passes earlier
    # errors on scaled by eta / (eta + eps), so the rounding reaches the potentials up to eta times
    # over; at eta = 1e4 the run-to-run spread of this error reached 2.2e-6 of the largest term.
    bar = 2e-6 if eta <= 100.0 else 5e-6
    assert abs(sd - sdr) < bar * scale
    m2 = fu.mmd(T(x), T(a), T(y), T(a), kernel="energy", grid=256, window=6)
    m2r, mt = oracle.mmd2(x, a, y, a, "energy", 1.0)
    assert abs(m2 - m2r) < TOL * max(abs(t) for t in mt)


@pytest.mark.parametrize("eps,eta,shift", [(0.1, 1.0, 0.3), (1.0, 1.0, 0.3), (1.0, 100.0, 0.3),
                                           (10.0, 100.0, 0.3), (0.1, 1.0, 0.1)])
def test_divergence_relative_to_itself(eps, eta, shift):
    """sd_{1;eta;lambda} of eq. (586) judged against its own size: 1-D uniform probability
    measures on [0, 1) and [shift, 1 + shift) (r = 1 cost), where the divergence is a resolvable
    fraction of its UOT terms.  The FP32 kernel sums leave an error of about 1e-7 of the largest
    term in each, so sd is resolved to 1e-5 of itself while |sd| >= 1e-2 of the largest term.
    eta stays at most 100: by eq. (995) a half-step scales perturbations of the other potential by
    eta / (eta + eps) and adds eta / (1 + eta lambda) times the sums' relative rounding, so the
    rounding can move the potentials by up to eta times itself (at eta = 1e4 the run-to-run spread
    reached 1e-5 of sd; that regime is covered against the largest term by
    test_divergence_energy_limit_experiment)."""
    rng = np.random.default_rng([1450, 11, int(100 * shift)])
    n = 1500
    x = rng.uniform(0, 1, (n, 1)).astype(np.float32)
    y = (shift + rng.uniform(0, 1, (n, 1))).astype(np.float32)
    a = np.full(n, 1.0 / n, np.float32)
    sd, terms = fu.sinkhorn_divergence(T(x), T(a), T(y), T(a), eps, eta, 300, kernel="laplace",
                                       grid=256, window=6)
    sdr, tr = oracle.sinkhorn_divergence(x, a, y, a, eps, eta, 300, r=1)
    ratio = abs(sdr) / max(abs(t) for t in tr)
    print("sd GPU %.10g oracle %.10g: rel err %.2e, |sd| / largest term %.2e" % (
        sd, sdr, abs(sd - sdr) / abs(sdr), ratio))
    assert ratio >= 1e-2
    assert abs(sd - sdr) < TOL * abs(sdr)


@pytest.mark.parametrize("kind,lam,grid", [("gauss", 0.02, 0), ("gauss", 0.02, 64),
                                           ("laplace", 0.05, 128), ("energy", 1.0, 256),
                                           ("energy", 1.0, 0), ("imq", 0.1, 128), ("imq", 0.1, 0)])
@pytest.mark.parametrize("d", [2, 3])
def test_mmd(kind, lam, grid, d):
    w = synth.make("uot_d3_n1M" if d == 3 else "uot_d2_n100k", n=1800, m=1500)
    x, y = w["x"][:, :d], w["y"][:, :d]
    ref, terms = oracle.mmd2(x, w["a"], y, w["b"], kind, lam)
    val, t3 = fu.mmd(T(x), T(w["a"]), T(y), T(w["b"]), kernel=kind, lam=lam, grid=grid, window=6,
                     terms=True)
    for k in range(3):
        assert abs(t3[k] - terms[k]) < TOL * abs(terms[k])
    scale = max(abs(t) for t in terms)
    assert abs(val - ref) < TOL * scale
    val1 = fu.mmd(T(x), T(w["a"]), T(y), T(w["b"]), kernel=kind, lam=lam, grid=grid, window=6)
    assert abs(val1 - ref) < TOL * scale


@pytest.mark.parametrize("kind,lam,grid", [("gauss", 0.25, 64), ("laplace", 0.5, 128),
                                           ("imq", 1.0, 128), ("energy", 1.0, 128)])
@pytest.mark.parametrize("n", [100, 1000, 10000])
def test_mmd_accuracy_experiment(kind, lam, grid, n):
    """The MMD accuracy experiment (Table Accuracy_analysis3: d = 2, points and weights uniform on
    [0, 1], l = 1/2, c = 1; probability vectors and unnormalised weights), GPU against the FP64
    oracle.  The FP32 bar is relative to the largest of the three double sums; the paper's residual
    relative to MMD^2 itself is printed (it grows where MMD^2 is small against the sums)."""
    rng = np.random.default_rng([1365, n])
    x = rng.uniform(0, 1, (n, 2)).astype(np.float32)
    y = rng.uniform(0, 1, (n, 2)).astype(np.float32)
    for norm in (True, False):
        a = rng.uniform(0, 1, n)
        b = rng.uniform(0, 1, n)
        if norm:
            a, b = a / a.sum(), b / b.sum()
        a, b = a.astype(np.float32), b.astype(np.float32)
        ref, terms = oracle.mmd2(x, a, y, b, kind, lam)
        val = fu.mmd(T(x), T(a), T(y), T(b), kernel=kind, lam=lam, grid=grid, window=6)
        scale = max(abs(t) for t in terms)
        print("%s n=%d %s: residual %.2e (vs largest term %.2e)"
              % (kind, n, "probability" if norm else "unbalanced", abs(val - ref) / abs(ref),
                 abs(val - ref) / scale))
        assert abs(val - ref) < TOL * scale


def test_mmd_self_is_zero():
    w = synth.make("uot_d3_n1M", n=2000)
    x, a = T(w["x"]), T(w["a"])
    val, t3 = fu.mmd(x, a, x, a, kernel="gauss", lam=0.02, grid=64, terms=True)
    assert abs(val) < 1e-6 * abs(t3[0])


# --------------------------------------------------------------------------- gradients

@pytest.mark.parametrize("kind,grid,tol", [("gauss", 0, 1e-4), ("gauss", 64, 1e-4),
                                           ("laplace", 0, 1e-4), ("laplace", 256, 1e-4),
                                           ("laplace", 128, 1e-4)])
def test_uot_grad_against_oracle_envelope(kind, grid, tol):
    """Backward kernels: the GPU envelope gradient at given potentials equals the oracle's direct
    FP64 gradient at the same potentials.  With the r = 1 (Laplace Gibbs) kernel at eps = 0.01 on
    these mixture clouds, about half the rows have kernel sums below 1e-2 of the largest (targets
    far from every source) while the plan keeps their mass; there the fast sum's absolute error
    floor would be a large relative error, so those rows are re-evaluated directly."""
    w = synth.make("divergence_d2_n200k", n=1200, m=1000)
    r = 2 if kind == "gauss" else 1
    beta, gamma = oracle.uot_sinkhorn(w["x"], w["a"], w["y"], w["b"], w["eps"], w["rho"], 40, r=r)
    ref = oracle.uot_grad(w["x"], w["a"], w["y"], w["b"], w["eps"], w["rho"], beta, gamma, r=r)
    got = fu.uot_sinkhorn_grad(T(w["x"]), T(w["a"]), T(w["y"]), T(w["b"]), w["eps"], w["rho"],
                               T(beta), T(gamma), kernel=kind, grid=grid, window=6)
    errs = [relinf(gv.cpu().numpy(), rv) for gv, rv in zip(got, ref)]
    print("uot grad rel errors (dx, da, dy, db):", errs)
    assert max(errs) < tol


@pytest.mark.parametrize("kind,lam,grid,cfg", [("gauss", 0.02, 0, "uot_d2_n100k"),
                                               ("gauss", 0.02, 64, "uot_d2_n100k"),
                                               ("energy", 1.0, 256, "uot_d2_n100k"),
                                               ("energy", 1.0, 256, "uot_d3_n1M"),
                                               ("laplace", 0.05, 128, "uot_d3_n1M"),
                                               ("imq", 0.1, 128, "uot_d2_n100k"),
                                               ("imq", 0.05, 256, "uot_d3_n1M")])
def test_mmd_grad_against_oracle(kind, lam, grid, cfg):
    w = synth.make(cfg, n=1100, m=900)
    ref = oracle.mmd2_grad(w["x"], w["a"], w["y"], w["b"], kind, lam)
    got = fu.mmd_grad(T(w["x"]), T(w["a"]), T(w["y"]), T(w["b"]), kernel=kind, lam=lam, grid=grid,
                      window=6)
    errs = [relinf(gv.cpu().numpy(), rv) for gv, rv in zip(got, ref)]
    print("mmd grad rel errors (dx, da, dy, db):", errs)
    assert max(errs) < 1e-4


def test_autograd_functions():
    """The autograd Functions: SinkhornDivergence's backward of 2.5 S (the scale reaches the
    gradient call) against the FP64 oracle's envelope gradient (Theorem "dualization") at the
    forward's potentials, on every row; MMD2's against the oracle's gradient."""
    w = synth.make("divergence_d2_n200k", n=500, m=450)
    x = T(w["x"]).requires_grad_()
    a = T(w["a"]).requires_grad_()
    y, b = T(w["y"]), T(w["b"])
    s = fu.SinkhornDivergence.apply(x, a, y, b, w["eps"], w["rho"], 300, {"grid": 64})
    (2.5 * s).backward()
    _, _, pots = fu.sinkhorn_divergence(x.detach(), a.detach(), y, b, w["eps"], w["rho"], 300,
                                        return_potentials=True, grid=64)
    fab, gab, faa, _ = (p.cpu().numpy() for p in pots)
    rows = np.arange(len(w["x"]))
    g1x, g1a = oracle.uot_grad_rows(w["x"], w["a"], rows, w["y"], w["b"], w["eps"], w["rho"],
                                    fab, gab)
    g2x, g2a = oracle.uot_grad_rows(w["x"], w["a"], rows, w["x"], w["a"], w["eps"], w["rho"],
                                    faa, faa)
    Ma, Mb = float(np.sum(w["a"], dtype=np.float64)), float(np.sum(w["b"], dtype=np.float64))
    refx = 2.5 * (g1x - g2x)
    refa = 2.5 * (g1a - g2a + w["eps"] * (Ma - Mb))
    ex = relinf(x.grad.cpu().numpy(), refx)
    ea = relinf(a.grad.cpu().numpy(), refa)
    print("autograd divergence gradient: dx %.2e da %.2e" % (ex, ea))
    assert ex < 1e-4 and ea < 1e-4
    x2 = T(w["x"]).requires_grad_()
    m2 = fu.MMD2.apply(x2, a.detach(), y, b, {"kernel": "gauss", "lam": 0.01, "grid": 64})
    m2.backward()
    ref = oracle.mmd2_grad(w["x"], w["a"], w["y"], w["b"], "gauss", 0.01)[0]
    assert relinf(x2.grad.cpu().numpy(), ref) < 1e-4

