"""Writes divergence_fd_d2_n2000.json: central differences of the converged FP64 Sinkhorn
divergence (eq. (586)) with respect to 64 random position coordinates and 16 random weights, on a
reduced size (n = 2000, m = 1800) of the d = 2 Gaussian-mixture divergence workload (eps = 0.01,
rho = 0.5), together with the oracle's envelope gradient at the same entries.

Only the FP64 CPU oracle is called.  The perturbed terms are UOT(mu, nu) and UOT(mu, mu); the
third term UOT(nu, nu) does not depend on x or a.  Each UOT value is the dual of Theorem
"dualization" after SWEEPS sweeps of Algorithm 1 from gamma = 0 (converged: the divergence changes
by less than 1e-15 relative between 600 and 1200 sweeps).

Run from the repository root:  python tests/golden/make_divergence_fd.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "divergence_fd_d2_n2000.json")
N, M, SWEEPS, H = 2000, 1800, 600, 1e-3
NCOORD, NWEIGHT = 64, 16


def uot(x, a, y, b, eps, rho):
    beta, gamma = oracle.uot_sinkhorn(x, a, y, b, eps, rho, SWEEPS)
    return oracle.uot_dual(x, a, y, b, eps, rho, beta, gamma), beta, gamma


def divergence(x, a, y, b, eps, rho, uyy):
    uxy = uot(x, a, y, b, eps, rho)[0]
    uxx = uot(x, a, x, a, eps, rho)[0]
    return uxy - 0.5 * uxx - 0.5 * uyy + 0.5 * eps * (a.sum() - b.sum()) ** 2


def main():
    w = synth.make("divergence_d2_n200k", n=N, m=M)
    eps, rho = w["eps"], w["rho"]
    x, a = w["x"].astype(np.float64), w["a"].astype(np.float64)
    y, b = w["y"].astype(np.float64), w["b"].astype(np.float64)
    rng = np.random.default_rng([2306, 13618, 64])
    rows = rng.choice(N, NCOORD, replace=False)
    comps = rng.integers(0, 2, NCOORD)
    widx = rng.choice(N, NWEIGHT, replace=False)
    uyy = uot(y, b, y, b, eps, rho)[0]
    # envelope gradient at the converged potentials (first slot of UOT(mu, nu), both slots of
    # UOT(mu, mu), and the mass term)
    _, fab, gab = uot(x, a, y, b, eps, rho)
    _, faa, _ = uot(x, a, x, a, eps, rho)
    g1x, g1a = oracle.uot_grad_rows(x, a, rows, y, b, eps, rho, fab, gab)
    g2x, g2a = oracle.uot_grad_rows(x, a, rows, x, a, eps, rho, faa, faa)
    env_dx = (g1x - g2x)[np.arange(NCOORD), comps]
    h1x, h1a = oracle.uot_grad_rows(x, a, widx, y, b, eps, rho, fab, gab)
    h2x, h2a = oracle.uot_grad_rows(x, a, widx, x, a, eps, rho, faa, faa)
    env_da = h1a - h2a + eps * (a.sum() - b.sum())
    t0 = time.time()
    fd_dx = []
    for k, (i, c) in enumerate(zip(rows, comps)):
        xp, xm = x.copy(), x.copy()
        xp[i, c] += H
        xm[i, c] -= H
        fd_dx.append((divergence(xp, a, y, b, eps, rho, uyy)
                      - divergence(xm, a, y, b, eps, rho, uyy)) / (2 * H))
        print("position %d/%d: fd %.10e envelope %.10e (%.0f s)" % (
            k + 1, NCOORD, fd_dx[-1], env_dx[k], time.time() - t0), flush=True)
    ha = H * a.mean()
    fd_da = []
    for k, i in enumerate(widx):
        ap, am = a.copy(), a.copy()
        ap[i] += ha
        am[i] -= ha
        fd_da.append((divergence(x, ap, y, b, eps, rho, uyy)
                      - divergence(x, am, y, b, eps, rho, uyy)) / (2 * ha))
        print("weight %d/%d: fd %.10e envelope %.10e" % (k + 1, NWEIGHT, fd_da[-1], env_da[k]),
              flush=True)
    rec = {
        "what": "central differences of the converged FP64 Sinkhorn divergence, eq. (586)",
        "workload": "divergence_d2_n200k", "n": N, "m": M, "eps": eps, "rho": rho,
        "sweeps": SWEEPS, "h": H, "h_weight": ha,
        "rows": [int(i) for i in rows], "comps": [int(c) for c in comps],
        "fd_dx": [float(v) for v in fd_dx], "envelope_dx": [float(v) for v in env_dx],
        "weight_rows": [int(i) for i in widx],
        "fd_da": [float(v) for v in fd_da], "envelope_da": [float(v) for v in env_da],
    }
    with open(OUT, "w") as fh:
        json.dump(rec, fh, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
