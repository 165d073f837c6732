"""Seeded synthetic point clouds and weights for the fast radial-kernel summation workloads.

This module only draws random numbers and holds the workload recipes.  It contains none of the
method's arithmetic, and it is the one piece shared by the CPU oracle, the tests and the benchmark.

Every array is drawn in float64 from ``numpy.random.default_rng([2306, 13618, k, rep])`` (k: the
workload's index) and cast to float32 once, so the GPU path and the oracle see bit-identical inputs (the oracle promotes the
float32 values back to float64).

Workloads (all coordinates inside the cube [-1/4, 1/4)^d, weights drawn U(0.5, 1.5) and rescaled to
the stated total masses; the paper's own synthetic setup draws uniform points and uniform weights,
Section "Empirical measures"):

* ``uot_d1_n2k``: d=1, n=m=2000; x ~ U[-1/4,1/4), y ~ N(0.05, 0.08^2) clipped; masses 1.0 / 1.5;
  Gibbs kernel exp(-|x-y|^2/eps), eps=0.05, rho=1 (the paper's lambda=20, eta=1); 200 sweeps.
* ``uot_d2_n100k``: d=2, n=m=100k; x from an 8-component, y from a 12-component Gaussian mixture
  (means U[-0.15,0.15]^2, sigma=0.02, equal component weights), clipped; masses 1.0 / 1.3;
  eps=0.01, rho=0.5; grid 128^2, window cutoff 6; 100 sweeps.
* ``uot_d3_n1M``: d=3, n=m=1M; x ~ U[-1/4,1/4)^3, y = clip(x + N(0, 0.03^2 I)); masses 1.0 / 1.2;
  UOT eps=0.02, rho=1, 50 sweeps; MMD with the energy kernel (near-field radius 1/16) and with the
  Gaussian lambda=0.02; grid 64^3, window cutoff 6.
* ``divergence_d2_n200k``: d=2, n=m=200k, clouds as uot_d2_n100k; Sinkhorn divergence (eps=0.01,
  rho=0.5) and Gaussian MMD (lambda=0.01), forward and backward.
* ``laplace_d3_n4M``: d=3, n=m=4M, clouds as uot_d3_n1M; Laplace Gibbs kernel exp(-|x-y|/eps),
  eps=0.01, near field; grid 256^3 with bandwidth 192 and smoothness 8; rho=1, 50 sweeps;
  masses 1.0 / 1.2.
* ``gauss_d32_n200k``: d=32, n=m=200k; x ~ N(0, I)/sqrt(32), y ~ N(0.1, I)/sqrt(32) (not clipped);
  Gaussian lambda=1; masses 1.0 / 1.2; direct summation.
"""
import numpy as np

SEED_ROOT = (2306, 13618)
CFG_INDEX = {"uot_d1_n2k": 0, "uot_d2_n100k": 1, "uot_d3_n1M": 2, "divergence_d2_n200k": 3,
             "laplace_d3_n4M": 4, "gauss_d32_n200k": 5}

# The largest float32 strictly below 1/4: "clipped to [-1/4, 1/4)".
HI = float(np.nextafter(np.float32(0.25), np.float32(0.0)))
LO = -0.25

CONFIGS = {
    "uot_d1_n2k": dict(d=1, n=2000, mass_a=1.0, mass_b=1.5, kernel="gauss", eps=0.05, rho=1.0,
                 iters=200, grid=64, window=6, points="uot_d1_n2k"),
    "uot_d2_n100k": dict(d=2, n=100_000, mass_a=1.0, mass_b=1.3, kernel="gauss", eps=0.01, rho=0.5,
                 iters=100, grid=128, window=6, points="mixture"),
    "uot_d3_n1M": dict(d=3, n=1_000_000, mass_a=1.0, mass_b=1.2, kernel="gauss", eps=0.02, rho=1.0,
                 iters=50, grid=64, window=6, points="perturbed", mmd_lambda=0.02,
                 nearfield_radius=1.0 / 16),
    "divergence_d2_n200k": dict(d=2, n=200_000, mass_a=1.0, mass_b=1.3, kernel="gauss", eps=0.01,
                                rho=0.5, iters=2000, grid=128, window=6, points="mixture",
                                mmd_lambda=0.01, fd_h=1e-3, fd_coords=64),
    "laplace_d3_n4M": dict(d=3, n=4_000_000, mass_a=1.0, mass_b=1.2, kernel="laplace", eps=0.01,
                  rho=1.0, iters=50, grid=256, window=6, points="perturbed", bandwidth=192,
                  smoothness=8),
    "gauss_d32_n200k": dict(d=32, n=200_000, mass_a=1.0, mass_b=1.2, kernel="gauss", eps=1.0,
                            rho=1.0, iters=50, grid=0, window=0, points="gauss32"),
}


def rng_for(cfg, rep=0):
    return np.random.default_rng([SEED_ROOT[0], SEED_ROOT[1], CFG_INDEX[cfg], rep])


def _weights(rng, n, mass):
    w = rng.uniform(0.5, 1.5, n)
    return w * (mass / w.sum())


def _mixture(rng, n, d, k):
    means = rng.uniform(-0.15, 0.15, (k, d))
    comp = rng.integers(0, k, n)
    pts = means[comp] + rng.normal(0.0, 0.02, (n, d))
    return np.clip(pts, LO, HI)


def make(cfg, rep=0, n=None, m=None):
    """Return a dict with float32 arrays x (n,d), a (n,), y (m,d), b (m,) and the config's scalars.

    ``n``/``m`` override the point counts (same recipe, same seed stream) for reduced-size runs.
    """
    c = dict(CONFIGS[cfg])
    d = c["d"]
    n = c["n"] if n is None else int(n)
    m = n if m is None else int(m)
    rng = rng_for(cfg, rep)
    kind = c["points"]
    if kind == "uot_d1_n2k":
        x = rng.uniform(LO, 0.25, (n, d))
        y = np.clip(rng.normal(0.05, 0.08, (m, d)), LO, HI)
    elif kind == "mixture":
        x = _mixture(rng, n, d, 8)
        y = _mixture(rng, m, d, 12)
    elif kind == "perturbed":
        x = rng.uniform(LO, 0.25, (n, d))
        base = x if m == n else rng.uniform(LO, 0.25, (m, d))
        y = np.clip(base + rng.normal(0.0, 0.03, (m, d)), LO, HI)
    elif kind == "gauss32":
        x = rng.normal(0.0, 1.0, (n, d)) / np.sqrt(d)
        y = rng.normal(0.1, 1.0, (m, d)) / np.sqrt(d)
    else:
        raise ValueError(kind)
    a = _weights(rng, n, c["mass_a"])
    b = _weights(rng, m, c["mass_b"])
    c.update(n=n, m=m,
             x=np.ascontiguousarray(x, dtype=np.float32),
             y=np.ascontiguousarray(y, dtype=np.float32),
             a=np.ascontiguousarray(a, dtype=np.float32),
             b=np.ascontiguousarray(b, dtype=np.float32))
    return c


def sample_rows(n, k, seed=0):
    """Seeded sorted sample of k distinct row indices out of n (for sampled full-size checks)."""
    rng = np.random.default_rng([SEED_ROOT[0], SEED_ROOT[1], 99, seed])
    k = min(k, n)
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)
