"""fs_plan_apply_noalloc (the allocation-free variant of fs_plan_apply, temporaries in a static
device array) against fs_plan_apply and the oracle, through the C-ABI: two calls in a row, the
second on a smaller plan, then the direct matrix-core path and a plan beyond the array's limit."""
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


def clouds(n, m, seed):
    rng = np.random.default_rng([5150, n, m, seed])
    x = rng.uniform(-0.25, 0.25, (n, 3)).astype(np.float32)
    y = np.clip(x[rng.integers(0, n, m)] + rng.normal(0, 0.03, (m, 3)), -0.25,
                synth.HI).astype(np.float32)
    return x, y, rng.uniform(0.5, 1.5, m).astype(np.float32), rng.uniform(0.5, 1.5, n).astype(np.float32)


def check_plan(x, y, v, u, kind, lam, **opts):
    pl = fu.Plan(T(x), T(y), kernel=kind, lam=lam, **opts)
    for transpose, vv, xt, ys in ((False, v, x, y), (True, u, y, x)):
        print("case noalloc %s n=%d m=%d transpose=%d" % (kind, len(x), len(y), transpose),
              flush=True)
        ref = pl.apply(T(vv), transpose=transpose)
        out = torch.full((len(xt),), float("nan"), dtype=torch.float32, device=DEV)
        got = pl.apply_noalloc(T(vv), out, transpose=transpose)
        torch.cuda.synchronize()
        got, ref = got.cpu().numpy(), ref.cpu().numpy()
        assert np.all(np.isfinite(got))
        assert relinf(got, ref) < TOL
        rows = synth.sample_rows(len(xt), 64, seed=len(xt))
        assert relinf(got[rows], oracle.direct_sum_rows(xt, rows, ys, vv, kind, lam)) < TOL
    pl.close()


def test_noalloc_fast_path_two_calls_second_smaller():
    x, y, v, u = clouds(60_000, 50_000, 1)
    check_plan(x, y, v, u, "gauss", 0.02, grid=64, window=6)
    x, y, v, u = clouds(3000, 2500, 2)
    check_plan(x, y, v, u, "laplace", 0.01, grid=128, window=6)


def test_noalloc_direct_matrix_core_path():
    w = synth.make("gauss_d32_n200k", n=1500, m=1300)
    check_plan(w["x"], w["y"], w["b"], w["a"], "gauss", 1.0, grid=0)


def test_noalloc_rejects_plans_beyond_the_scratch():
    rng = np.random.default_rng(9)
    n = 2_200_000
    x = rng.uniform(-0.25, 0.25, (n, 1)).astype(np.float32)
    pl = fu.Plan(T(x), T(x), kernel="gauss", lam=0.02, grid=64, window=6)
    out = torch.zeros(n, dtype=torch.float32, device=DEV)
    with pytest.raises(fu.FastsumError, match="scratch"):
        pl.apply_noalloc(T(np.ones(n, np.float32)), out)
    pl.close()
