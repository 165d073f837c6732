"""Benchmark: unbalanced Sinkhorn sweeps/s with NFFT fast summation on one MI355X.

Headline workload: d=3, n=m=1M, x ~ U[-1/4,1/4)^3, y = clip(x + N(0,0.03^2)), weights U(0.5,1.5)
with masses 1.0 / 1.2, Gibbs kernel exp(-|x-y|^2/eps), eps=0.02, rho=1, 50 sweeps per solve, FFT
grid 64^3, Kaiser-Bessel window cutoff 6.  One timed step is one full uot_sinkhorn call (plan:
scaling, binning, kernel coefficients; 50 sweeps; objective) with the inputs resident in HBM.
value = sweeps per second.

Also reported (extra keys of the same JSON line):
  * GPU direct-summation sweeps/s on the same inputs and the speedup of the fast path;
  * the sampled full-size error of the last half-step against the FP64 oracle (and the sampled
    errors of the other workloads), computed in the CPU-baseline leg together with its timing;
  * the dominant kernel's (the spread's) roofline, its average duration taken from HIP events
    around every 5th of its launches during the timed steps, and per-pass average durations and
    HBM GB/s of spread, FFT and gather from one further, untimed step with events around every
    pass;
  * the secondary metric: forward and forward+backward ms of the Sinkhorn divergence on the
    d=2, n=m=200k Gaussian-mixture workload;
  * the other workloads: 2-D 100k Sinkhorn, MMD at 1M (energy, Gauss, IMQ), the MMD accuracy
    experiment at n=10k, the 4M Laplace Sinkhorn and the d=32 MFMA sum;
  * the FP64 oracle's rate on the host cores (a bounded sample scaled to sweeps/s).
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP16_MFMA_TFLOPS = 2500.0  # MI355X published dense FP16 matrix peak
PEAK_HBM_GBS = 8000.0          # MI355X published HBM3E bandwidth
PEAK_FP32_VALU_TFLOPS = 157.3  # MI355X published FP32 vector peak (256 CUs x 2.4 GHz x 256)
NF_FLOPS_PER_PAIR = 30         # near-field flops per pair inside the radius (see nearfield_row)
SPREAD_SAMPLE = 5              # time every 5th spread launch of the timed steps


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=None, help="override the point count (testing only)")
    ap.add_argument("--no-direct", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--grid", type=int, default=64)
    ap.add_argument("--window", type=int, default=6)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other workloads (2-D Sinkhorn, MMD, 4M Laplace, d=32 MFMA)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 256 MiB device-to-device copy first (counter calibration)")
    return ap.parse_args()


def log(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


def traffic_from_profile(kernel_src):
    """HBM bytes per launch of the spread kernel from the committed rocprofv3 --pmc summary, if it
    was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "spread_pmc_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    digest = hashlib.sha256(open(kernel_src, "rb").read()).hexdigest()
    if rec.get("source_sha256") != digest:
        return None
    return rec.get("bytes_per_launch")


def timed(torch, fn, reps=1):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        out = fn()
    torch.cuda.synchronize()
    return out, (time.perf_counter() - t0) / reps


def nearfield_pairs(xt, ys, radius, k=4096, seed=0):
    """Pairs (target, source) closer than `radius`, estimated from k sampled targets counted
    exactly against every source with a k-d tree on the host (the near field's algorithmic work
    per kernel sum)."""
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(seed)
    idx = rng.choice(len(xt), size=min(k, len(xt)), replace=False)
    tree = cKDTree(ys)
    cnt = tree.query_ball_point(xt[idx], radius, return_length=True)
    return float(np.mean(cnt)) * len(xt)


def nearfield_row(fu, torch, run, pairs, label):
    """Average near-field pass time of `run` (events around every near-field launch of one call)
    and its throughput against the FP32 vector roofline: each pair inside the radius costs
    NF_FLOPS_PER_PAIR flops (3 differences and 3 multiply-adds for r^2, the square root, the inner
    polynomial in r^2 (8 coefficients: 16 flops), the kernel's exponential, the difference and the
    weighted accumulation)."""
    fu.fs_profile_reset()
    fu.fs_profile_select("nearfield", 1)
    fu.fs_profile_enable(True)
    run()
    torch.cuda.synchronize()
    fu.fs_profile_enable(False)
    ms, cnt = fu.fs_profile_query("nearfield")
    fu.fs_profile_reset()
    t = ms / cnt * 1e-3
    tflops = pairs * NF_FLOPS_PER_PAIR / t / 1e12
    log("near field %s: %.2f ms per pass, %.3g pairs, %.3g pairs/s" % (label, 1e3 * t, pairs,
                                                                        pairs / t))
    return {"avg_ms": 1e3 * t, "passes": cnt, "pairs_in_radius": pairs, "pairs_per_s": pairs / t,
            "roofline": {"bound": "alu", "achieved": tflops, "peak": PEAK_FP32_VALU_TFLOPS,
                         "unit": "TFLOP/s", "frac": tflops / PEAK_FP32_VALU_TFLOPS,
                         "work": "%d flops per pair inside the radius; pairs from %s"
                                 % (NF_FLOPS_PER_PAIR,
                                    "4096 sampled targets counted exactly (k-d tree)")}}


def extra_rows(fu, torch, dev, synth, keep):
    """The other workloads of the hot path, timed on the GPU.  Outputs needed for the sampled
    error checks go to `keep`; the checks themselves run in the CPU-baseline leg."""
    rows = {}

    # 2-D Gaussian-mixture Sinkhorn, n=m=100k, grid 128^2, 100 sweeps, fast vs direct
    w = synth.make("uot_d2_n100k")
    x, a, y, b = (torch.from_numpy(w[k]).to(dev) for k in ("x", "a", "y", "b"))
    run = lambda: fu.uot_sinkhorn(x, a, y, b, w["eps"], w["rho"], w["iters"], grid=w["grid"],
                                  window=w["window"])
    timed(torch, run)
    (f, g, _), t = timed(torch, run, 2)
    _, td = timed(torch, lambda: fu.uot_sinkhorn(x, a, y, b, w["eps"], w["rho"], 2, grid=0))
    rows["uot_d2_n100k"] = {"sweeps_per_s": w["iters"] / t, "direct_sweeps_per_s": 2 / td,
                            "speedup_vs_direct": (w["iters"] / t) / (2 / td),
                            "err_sampled_last_halfstep": None}
    keep["uot_d2_n100k"] = ("uot", "uot_d2_n100k", 2, f.cpu().numpy(), g.cpu().numpy())
    log("2-D 100k: %.0f sweeps/s fast, %.1f direct" % (w["iters"] / t, 2 / td))

    # MMD^2 at d=3, n=m=1M: energy kernel (near-field radius 1/16), Gaussian lambda=0.02, and the
    # inverse multiquadric with c = 0.05 (near-field radius 1/16)
    w = synth.make("uot_d3_n1M")
    x, a, y, b = (torch.from_numpy(w[k]).to(dev) for k in ("x", "a", "y", "b"))
    mmd_rows = {}
    for kind, opts in (("energy", {"grid": 256, "nearfield_radius": w["nearfield_radius"]}),
                       ("gauss", {"lam": w["mmd_lambda"], "grid": 64}),
                       ("imq", {"lam": 0.05, "grid": 256, "nearfield_radius": w["nearfield_radius"]})):
        fu.mmd(x, a, y, b, kernel=kind, window=6, **opts)
        v, t = timed(torch, lambda: fu.mmd(x, a, y, b, kernel=kind, window=6, **opts), 2)
        mmd_rows[kind] = {"ms": 1e3 * t, "mmd2": v, **{k: o for k, o in opts.items()}}
        log("MMD %s 1M: %.1f ms" % (kind, 1e3 * t))
    # the energy MMD's near field: one kernel sum on the union of both sets
    z = np.concatenate([w["x"], w["y"]])
    mmd_rows["energy"]["nearfield"] = nearfield_row(
        fu, torch, lambda: fu.mmd(x, a, y, b, kernel="energy", window=6, grid=256,
                                  nearfield_radius=w["nearfield_radius"]),
        nearfield_pairs(z, z, w["nearfield_radius"]), "energy MMD 1M")
    rows["mmd_d3_n1M"] = mmd_rows

    # the MMD accuracy experiment (Table Accuracy_analysis3): d = 2, n = m = 10000 points and
    # weights uniform on [0, 1], l = 1/2, c = 1; probability vectors and unnormalised weights
    rng = np.random.default_rng([1365, 10000])
    xe = rng.uniform(0, 1, (10000, 2)).astype(np.float32)
    ye = rng.uniform(0, 1, (10000, 2)).astype(np.float32)
    acc = {}
    for norm in (True, False):
        ae, be = rng.uniform(0, 1, 10000), rng.uniform(0, 1, 10000)
        if norm:
            ae, be = ae / ae.sum(), be / be.sum()
        ae, be = ae.astype(np.float32), be.astype(np.float32)
        label = "probability" if norm else "unbalanced"
        for kind, lam, grid in (("gauss", 0.25, 64), ("laplace", 0.5, 128), ("imq", 1.0, 128),
                                ("energy", 1.0, 128)):
            T = lambda z: torch.from_numpy(z).to(dev)
            v, t = timed(torch, lambda: fu.mmd(T(xe), T(ae), T(ye), T(be), kernel=kind, lam=lam,
                                               grid=grid, window=6))
            acc["%s_%s" % (kind, label)] = {"mmd2": v, "ms": 1e3 * t, "residual": None}
            keep["acc_%s_%s" % (kind, label)] = ("mmd", xe, ae, ye, be, kind, lam, v)
    rows["mmd_accuracy_d2_n10k"] = acc

    # 4M Laplace Gibbs-kernel Sinkhorn (r = 1) with near field, grid 256^3
    w = synth.make("laplace_d3_n4M")
    x, a, y, b = (torch.from_numpy(w[k]).to(dev) for k in ("x", "a", "y", "b"))
    it = 5
    opts = {"kernel": "laplace", "grid": w["grid"], "window": w["window"],
            "bandwidth": w["bandwidth"], "smoothness": w["smoothness"]}
    fu.uot_sinkhorn(x, a, y, b, w["eps"], w["rho"], 1, **opts)
    (f, g, _), t = timed(torch, lambda: fu.uot_sinkhorn(x, a, y, b, w["eps"], w["rho"], it, **opts))
    rows["uot_laplace_d3_n4M"] = {"sweeps_per_s": it / t, "sweeps_timed": it,
                                  "grid": w["grid"], "bandwidth": w["bandwidth"],
                                  "smoothness": w["smoothness"],
                                  "err_sampled_last_halfstep": None}
    # near field of this plan: default radius smoothness / N in torus units
    pl = fu.Plan(x, y, kernel="laplace", lam=w["eps"], **{k: v for k, v in opts.items()
                                                          if k != "kernel"})
    _, _, period, bw = pl.multiplier()
    pl.close()
    radius = w["smoothness"] / bw * period
    rows["uot_laplace_d3_n4M"]["nearfield"] = nearfield_row(
        fu, torch, lambda: fu.uot_sinkhorn(x, a, y, b, w["eps"], w["rho"], 1, **opts),
        nearfield_pairs(w["x"], w["y"], radius), "4M Laplace")
    rows["uot_laplace_d3_n4M"]["nearfield"]["radius"] = radius
    keep["uot_laplace_d3_n4M"] = ("uot", "laplace_d3_n4M", 1, f.cpu().numpy(), g.cpu().numpy())
    log("4M Laplace: %.1f sweeps/s (%d sweeps incl. plan)" % (it / t, it))

    # lambda-scaling (Section "lambda-scaling": Lambda = {1, 20, 100}, eta = 25, probability
    # measures): the 2-D mixtures normalised to mass 1, temperatures 1, 0.05, 0.01 against a
    # solve at 0.01 alone, both to the same stopping rule (largest change <= 1e-4 eps per sweep)
    w = synth.make("uot_d2_n100k")
    a1, b1 = w["a"] / w["a"].sum(dtype=np.float64), w["b"] / w["b"].sum(dtype=np.float64)
    x, a, y, b = (torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32)).to(dev)
                  for v in (w["x"], a1, w["y"], b1))
    sc = {}
    for label, stages, init in (("scaled_zero_start", [1.0, 0.05, 0.01], "zero"),
                                ("scaled_cstar_start", [1.0, 0.05, 0.01], "cstar"),
                                ("single_temperature", [0.01], "zero")):
        (f, g, counts, obj), t = timed(torch, lambda: fu.uot_sinkhorn_scaling(
            x, a, y, b, stages, 25.0, 6000, 1e-4, init=init, grid=w["grid"], window=w["window"]))
        sc[label] = {"stages": stages, "sweeps": counts, "total_sweeps": sum(counts),
                     "ms": 1e3 * t, "objective": obj}
        log("lambda-scaling %s: sweeps %s, %.1f ms" % (label, counts, 1e3 * t))
    rows["lambda_scaling_d2_n100k"] = sc

    # Corollary 477 experiment: sd_{1;eta;lambda}(P, P~) of 1-D uniform probability measures
    # (n = m = 10000) against half the energy MMD^2 of eq. (1205), for growing temperatures and
    # marginal penalties (300 sweeps per UOT term, grid 256)
    rng = np.random.default_rng([1450, 10000])
    xe = torch.from_numpy(rng.uniform(0, 1, (10000, 1)).astype(np.float32)).to(dev)
    ye = torch.from_numpy(rng.uniform(0, 1, (10000, 1)).astype(np.float32)).to(dev)
    pe = torch.full((10000,), 1e-4, dtype=torch.float32, device=dev)
    half = 0.5 * fu.mmd(xe, pe, ye, pe, kernel="energy", grid=256, window=6)
    conv = {"half_energy_mmd2": half, "sd": {}}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for eps in (1.0, 10.0, 100.0):
        for eta in (1.0, 100.0, 1e4):
            sd, _ = fu.sinkhorn_divergence(xe, pe, ye, pe, eps, eta, 300, kernel="laplace",
                                           grid=256, window=6)
            conv["sd"]["eps=%g,eta=%g" % (eps, eta)] = {"sd": sd, "ratio_to_half_mmd2": sd / half}
    torch.cuda.synchronize()
    conv["ms_all"] = 1e3 * (time.perf_counter() - t0)
    rows["divergence_to_energy_d1_n10k"] = conv
    log("sd -> energy: half MMD^2 %.6g, sd(eps=100, eta=1e4) %.6g, %.0f ms for 9 divergences"
        % (half, conv["sd"]["eps=100,eta=10000"]["sd"], conv["ms_all"]))

    # upper bound of eq. (561) at the headline workload: r = 2 from moments, r = 1 through one
    # energy-kernel sum (grid 256, near-field radius 1/16)
    w = synth.make("uot_d3_n1M")
    x, a, y, b = (torch.from_numpy(w[k]).to(dev) for k in ("x", "a", "y", "b"))
    ub = {}
    for label, opts in (("r2", {"kernel": "gauss"}),
                        ("r1", {"kernel": "laplace", "grid": 256, "window": 6,
                                "nearfield_radius": w["nearfield_radius"]})):
        (c, bound), t = timed(torch, lambda: fu.uot_upper_bound(x, a, y, b, w["eps"], w["rho"],
                                                                **opts))
        ub[label] = {"cstar": c, "bound": bound, "ms": 1e3 * t}
        log("upper bound %s: c* %.6g, bound %.6g, %.2f ms" % (label, c, bound, 1e3 * t))
    rows["upper_bound_d3_n1M"] = ub

    # d = 32 direct Gaussian sum on the matrix-core path (FP16 hi/lo Gram tiles of the centred
    # coordinates, BF16 norm step), n=m=200k
    w = synth.make("gauss_d32_n200k")
    x, y, b = (torch.from_numpy(w[k]).to(dev) for k in ("x", "y", "b"))
    fu.fastsum_apply(x, y, b, kernel="gauss", lam=w["eps"], grid=0)
    out, t = timed(torch, lambda: fu.fastsum_apply(x, y, b, kernel="gauss", lam=w["eps"], grid=0), 3)
    flops = 3 * 2.0 * w["d"] * w["n"] * w["m"]
    rows["mfma_gauss_d32_n200k"] = {
        "ms": 1e3 * t, "err_sampled": None,
        "roofline": {"bound": "mfma", "achieved": flops / t / 1e12, "peak": 2500.0,
                     "unit": "TFLOP/s", "frac": flops / t / 1e12 / 2500.0,
                     "work": "3 FP16 products x 2 x d x n x m (coordinate K steps; the "
                             "norm step not counted)"},
        "pairs_per_s": w["n"] * w["m"] / t}
    keep["mfma_gauss_d32_n200k"] = ("sum", "gauss_d32_n200k", out.cpu().numpy())
    log("d=32 MFMA: %.2f ms" % (1e3 * t))
    return rows


def cpu_baseline_leg(synth, w, f, g, extras, keep):
    """The FP64 oracle on the host cores: its rate on a bounded sample of the headline workload,
    and, from the same leg, the exact values of sampled rows (and of the small MMD experiment)
    against which every GPU result of this run is scored."""
    import oracle
    n, m, eps, rho = w["n"], w["m"], w["eps"], w["rho"]

    def rel(got, ref):
        return float(np.max(np.abs(np.asarray(got) - ref)) / np.max(np.abs(ref)))

    # rate: beta and gamma half-steps for R sampled rows each against all sources
    R = 8192
    rows = synth.sample_rows(n, R, seed=2)
    t1 = time.perf_counter()
    oracle.uot_beta_rows(w["x"], rows, w["y"], w["b"], np.zeros(m), eps, rho)
    oracle.uot_beta_rows(w["y"], rows, w["x"], w["a"], np.zeros(n), eps, rho)
    tcpu = time.perf_counter() - t1
    sweep_s = tcpu * (n / R)
    cpu = {"value": 1.0 / sweep_s, "unit": "sweeps/s", "cores": oracle.num_threads(),
           "kind": "oracle",
           "sample": "FP64 beta and gamma half-steps (Algorithm 1, log-sum-exp) for %d of %d "
                     "rows each against all %d sources, %.1f s, scaled to one full sweep"
                     % (R, n, m, tcpu)}
    log("oracle %.3g sweeps/s on %d threads" % (cpu["value"], cpu["cores"]))

    # headline: the last (gamma) half-step recomputed from the GPU's final beta
    idx = synth.sample_rows(m, 128, seed=1)
    ref = oracle.uot_beta_rows(w["y"], idx, w["x"], w["a"], f, eps, rho)
    err = rel(g[idx], ref)
    log("sampled last-half-step error %.2e (%d rows)" % (err, len(idx)))

    for key, item in keep.items():
        if item[0] == "uot":
            _, cfg, r, fk, gk = item
            wk = synth.make(cfg)
            idx = synth.sample_rows(wk["m"], 64, seed=3)
            refk = oracle.uot_beta_rows(wk["y"], idx, wk["x"], wk["a"], fk, wk["eps"], wk["rho"], r=r)
            extras[key]["err_sampled_last_halfstep"] = rel(gk[idx], refk)
        elif item[0] == "sum":
            _, cfg, out = item
            wk = synth.make(cfg)
            idx = synth.sample_rows(wk["n"], 64, seed=5)
            refk = oracle.direct_sum_rows(wk["x"], idx, wk["y"], wk["b"], "gauss", wk["eps"])
            extras[key]["err_sampled"] = rel(out[idx], refk)
        elif item[0] == "mmd":
            _, xe, ae, ye, be, kind, lam, v = item
            refv, terms = oracle.mmd2(xe, ae, ye, be, kind, lam)
            entry = extras["mmd_accuracy_d2_n10k"][key[4:]]
            entry["residual"] = abs(v - refv) / abs(refv)
            entry["err_vs_largest_term"] = abs(v - refv) / max(abs(t) for t in terms)
    return cpu, err


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the fast-summation path is built and timed on a "
              "single MI355X (sharding across GPUs is not implemented).",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2306_13618_amd as fu
    import synth

    dev = torch.device("cuda:0")
    w = synth.make("uot_d3_n1M", n=args.n)
    n, m, d = w["n"], w["m"], w["d"]
    eps, rho, sweeps = w["eps"], w["rho"], w["iters"]
    x, a, y, b = (torch.from_numpy(w[k]).to(dev) for k in ("x", "a", "y", "b"))
    torch.cuda.synchronize()
    if args.calib_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def step(grid, iters):
        return fu.uot_sinkhorn(x, a, y, b, eps, rho, iters, kernel="gauss", grid=grid,
                               window=args.window)

    log("warmup %d steps (n=m=%d, d=%d, %d sweeps/step, grid %d, window %d)"
        % (args.warmup, n, d, sweeps, args.grid, args.window))
    for _ in range(args.warmup):
        step(args.grid, sweeps)
    torch.cuda.synchronize()
    # timed steps: HIP events around every SPREAD_SAMPLE-th launch of the dominant kernel (the
    # spread) on its stream, few enough that their own cost stays out of the wall time
    fu.fs_profile_reset()
    fu.fs_profile_select("spread", SPREAD_SAMPLE)
    fu.fs_profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        f, g, obj = step(args.grid, sweeps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    fu.fs_profile_enable(False)
    sp_ms, sp_cnt = fu.fs_profile_query("spread")
    # per-pass breakdown from one more (untimed) step with events around every pass
    fu.fs_profile_reset()
    fu.fs_profile_select(None, 1)
    fu.fs_profile_enable(True)
    step(args.grid, sweeps)
    torch.cuda.synchronize()
    fu.fs_profile_enable(False)
    passes = {}
    for name in ("spread", "fold", "fft", "gather", "update"):
        ms, cnt = fu.fs_profile_query(name)
        passes[name] = {"avg_ms": ms / cnt if cnt else None, "launches": cnt}
    fu.fs_profile_reset()
    ms_per_step = 1e3 * elapsed / args.steps
    value = sweeps * args.steps / elapsed
    log("fast %.3f ms/step, %.1f sweeps/s, objective %.9g" % (ms_per_step, value, obj))
    log("passes (avg ms): " + ", ".join("%s %.4f" % (k, v["avg_ms"] or 0) for k, v in passes.items()))

    # ---- roofline of the dominant kernel (spread): algorithmic work per launch
    W = 2 * args.window
    sp = sp_ms / sp_cnt  # sampled over the timed steps
    flops_per_launch = n * 2.0 * W ** d          # one multiply and one add per window point
    achieved_tflops = flops_per_launch / (sp * 1e-3) / 1e12
    # node record, FP32 base weight and FP64 potential (the weights are formed in the spread),
    # grid written
    bytes_per_launch = n * (16 + 4 + 8) + 4 * args.grid ** d
    traffic = traffic_from_profile(os.path.join(ROOT, "paper_2306_13618_amd", "csrc", "nfft.hip"))
    roofline = {"bound": "mfma", "achieved": achieved_tflops, "peak": PEAK_FP16_MFMA_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved_tflops / PEAK_FP16_MFMA_TFLOPS,
                "traffic": traffic,
                "kernel": "k_spread_mom16 (spreading, adjoint NFFT, Chebyshev moments of the "
                          "(y, z) window on the FP16 matrix cores with hi/lo split operands)",
                "work_per_launch": "%d nodes x 2 x %d^%d flops (the window products at FP32 "
                                   "accuracy that the kernel's result equals)" % (n, W, d),
                "timed_launches": sp_cnt}
    window_terms = n * float(W ** d)
    hbm = {}
    G = args.grid
    for name, nbytes in (("spread", bytes_per_launch),
                         ("gather", n * (16 + 8) + 4 * G ** d),  # record, FP64 potential out
                         ("fft", 2 * 4 * G ** d)):
        t = passes[name]["avg_ms"]
        hbm[name] = {"algorithmic_bytes": nbytes,
                     "GBs": nbytes / (t * 1e-3) / 1e9 if t else None,
                     "frac_of_8TBs": (nbytes / (t * 1e-3) / 1e9) / PEAK_HBM_GBS if t else None}

    # ---- GPU direct summation on the same inputs (one sweep)
    direct = None
    if not args.no_direct:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        step(0, 1)
        torch.cuda.synchronize()
        direct = 1.0 / (time.perf_counter() - t0)
        log("direct %.3f s/sweep" % (1.0 / direct))

    # ---- secondary: Sinkhorn divergence forward and forward+backward (d=2, n=m=200k)
    secondary = None
    if not args.no_secondary:
        w3 = synth.make("divergence_d2_n200k")
        x3, a3, y3, b3 = (torch.from_numpy(w3[k]).to(dev) for k in ("x", "a", "y", "b"))
        it3 = 300
        opts = {"grid": w3["grid"], "window": w3["window"]}
        for rep in range(2):  # first repetition warms up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            with torch.no_grad():
                fu.sinkhorn_divergence(x3, a3, y3, b3, w3["eps"], w3["rho"], it3, **opts)
            torch.cuda.synchronize()
            fwd_ms = 1e3 * (time.perf_counter() - t0)
            xg = x3.clone().requires_grad_()
            ag = a3.clone().requires_grad_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s = fu.SinkhornDivergence.apply(xg, ag, y3, b3, w3["eps"], w3["rho"], it3, opts)
            s.backward()
            torch.cuda.synchronize()
            fb_ms = 1e3 * (time.perf_counter() - t0)
        secondary = {"workload": "Sinkhorn divergence, d=2 n=m=200k Gaussian mixtures, eps=0.01 "
                                 "rho=0.5, %d sweeps per UOT term, grid 128^2, window 6" % it3,
                     "fwd_ms": fwd_ms, "fwd_bwd_ms": fb_ms, "bwd_over_fwd": (fb_ms - fwd_ms) / fwd_ms,
                     "value": float(s.item())}
        log("divergence fwd %.1f ms, fwd+bwd %.1f ms" % (fwd_ms, fb_ms))

    keep = {}
    extras = None if args.no_extras else extra_rows(fu, torch, dev, synth, keep)

    # ---- CPU-baseline leg: the FP64 oracle on the host cores (rate and sampled references)
    cpu, err_sampled = None, None
    if not args.no_cpu:
        cpu, err_sampled = cpu_baseline_leg(synth, w, f.cpu().numpy(), g.cpu().numpy(),
                                            extras if extras is not None else {}, keep)

    line = {
        "metric": "UOT Sinkhorn iters/sec fast-sum vs direct, n=1M d=3 at rel err<=1e-5; fwd+bwd ms",
        "value": value, "unit": "sweeps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "UOT Sinkhorn, d=3 n=m=%d uniform / perturbed clouds, Gauss eps=%g "
                               "rho=%g, %d sweeps per step, grid %d^3, window %d"
                               % (n, eps, rho, sweeps, args.grid, args.window),
                   "n": n, "m": m, "d": d, "sweeps_per_step": sweeps, "grid": args.grid,
                   "window": args.window, "update_dtype": "f64"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "direct_sweeps_per_s": direct,
        "speedup_vs_direct": (value / direct) if direct else None,
        "err_sampled_last_halfstep": err_sampled,
        "objective": obj,
        "passes_avg_ms": {k: v["avg_ms"] for k, v in passes.items()},
        "window_terms_per_s_spread": window_terms / (sp * 1e-3),
        "hbm": hbm,
        "secondary": secondary,
        "rows": extras,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
