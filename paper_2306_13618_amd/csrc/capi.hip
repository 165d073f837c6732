// extern "C" entry points of libfastuot (declared in include/fastuot.h).
// Every entry point validates its arguments, runs the work on the caller's stream, converts
// internal failures (fs::Error) into a negative fs_status and records the message.
#include <algorithm>
#include <functional>
#include <mutex>
#include <string>
#include <system_error>
#include <thread>

#include "solver.h"

// Scratch of fs_plan_apply_noalloc: the operator-order weights and sums of the fast path, or the
// partial row sums of the direct matrix-core path.  One copy per GPU, held until the process
// ends.  Host code never passes this name to a kernel: it is a host-side stand-in, and the
// device address of each GPU's copy comes from hipGetSymbolAddress (noalloc_scratch below).
constexpr size_t FS_NOALLOC_SCRATCH_BYTES = size_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[FS_NOALLOC_SCRATCH_BYTES];

namespace fs {
const char *last_error();
int profile_enable(int on);
int profile_select(const char *pass, int period);
int profile_query(const char *pass, double *total_ms, int64_t *count);
void profile_reset();

namespace {

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Device address of the current GPU's copy of `scratch`, looked up once per device (with that
// device current) and kept.
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[MAX_DEVICES] = {};

char *noalloc_scratch() {
    int dev = 0;
    FS_HIP(hipGetDevice(&dev));
    FS_REQUIRE(dev >= 0 && dev < MAX_DEVICES, FS_EUNSUPPORTED, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        FS_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        FS_REQUIRE(ptr != nullptr, FS_EHIP, "no device address for the scratch array");
        g_scratch_dev[dev] = ptr;
    }
    return static_cast<char *>(g_scratch_dev[dev]);
}

// Runs independent pieces of work side by side: pieces[0] on the caller's stream s in this
// thread, pieces[k] (k >= 1) on library stream k - 1 in a thread of its own (the current device
// made current there).  The library streams first wait for the work queued on s so far.  Each
// piece synchronises its own stream before it returns, so all have finished on return; an error
// in a side piece is raised here with its status and message after every piece has ended.
using Piece = std::function<void(hipStream_t)>;

void run_side_by_side(hipStream_t s, const std::vector<Piece> &pieces) {
    const int np = (int)pieces.size();
    FS_REQUIRE(np >= 1 && np <= 1 + LIB_STREAMS, FS_EINVAL, "%d pieces of work", np);
    int dev = 0;
    FS_HIP(hipGetDevice(&dev));
    std::vector<hipStream_t> st(np, s);
    for (int k = 1; k < np; ++k) st[k] = library_stream(k - 1);
    hipEvent_t ready = nullptr;
    FS_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    struct Result {
        int code = FS_OK;
        std::string msg;
    };
    std::vector<Result> res(np);
    auto side = [&](int k) {
        try {
            clear_error();
            FS_HIP(hipSetDevice(dev));
            pieces[k](st[k]);
        } catch (const Error &e) {
            res[k].code = e.code;
            res[k].msg = last_error();
        } catch (const std::bad_alloc &) {
            res[k].code = FS_ENOMEM;
            res[k].msg = "host allocation failed";
        } catch (...) {
            res[k].code = FS_EHIP;
            res[k].msg = "unexpected internal error";
        }
    };
    {
        hipError_t e = hipEventRecord(ready, s);
        for (int k = 1; k < np && e == hipSuccess; ++k) e = hipStreamWaitEvent(st[k], ready, 0);
        if (e != hipSuccess) {
            (void)hipEventDestroy(ready);
            FS_HIP(e);
        }
    }
    // every thread that was started is joined, whatever throws (a thread that cannot be started
    // leaves its piece to this thread)
    std::vector<std::thread> th(np);
    auto join_all = [&] {
        for (auto &t : th)
            if (t.joinable()) t.join();
        (void)hipEventDestroy(ready);
    };
    try {
        for (int k = 1; k < np; ++k) {
            try {
                th[k] = std::thread(side, k);
            } catch (const std::system_error &) {
                side(k);
            }
        }
        pieces[0](s);
    } catch (...) {
        join_all();
        throw;
    }
    join_all();
    for (int k = 1; k < np; ++k)
        if (res[k].code != FS_OK) {
            set_error("%s", res[k].msg.c_str());
            throw Error{res[k].code};
        }
}

void check_params(const fs_params *p) {
    FS_REQUIRE(p != nullptr, FS_EINVAL, "params is NULL");
    FS_REQUIRE(p->grid >= 0, FS_EINVAL, "grid must be >= 0");
    FS_REQUIRE(p->window >= 0 && p->oversampling >= 0 && p->smoothness >= 0, FS_EINVAL,
               "window, oversampling and smoothness must be >= 0");
    FS_REQUIRE(p->nearfield_radius >= 0 && std::isfinite(p->nearfield_radius), FS_EINVAL,
               "nearfield_radius must be finite and >= 0");
}

void check_points(const void *ptr, int64_t count, const char *name) {
    FS_REQUIRE(count >= 0, FS_EINVAL, "%s: negative size", name);
    FS_REQUIRE(count == 0 || ptr != nullptr, FS_EINVAL, "%s is NULL", name);
    FS_REQUIRE(count < (int64_t(1) << 31), FS_EINVAL, "%s: more than 2^31 - 1 points", name);
}

void check_transport(const fs_params *p, double rho) {
    FS_REQUIRE(p->kernel == FS_GAUSS || p->kernel == FS_LAPLACE, FS_EINVAL,
               "transport uses the Gibbs kernel of |x-y|^2 (FS_GAUSS) or |x-y| (FS_LAPLACE)");
    FS_REQUIRE(p->lambda > 0 && std::isfinite(p->lambda), FS_EINVAL, "lambda must be > 0");
    FS_REQUIRE(rho > 0 && std::isfinite(rho), FS_EINVAL, "rho must be > 0");
}

template <class F>
int guarded(F &&f) {
    try {
        clear_error();
        f();
        return FS_OK;
    } catch (const Error &e) {
        return e.code;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return FS_ENOMEM;
    } catch (...) {
        set_error("unexpected internal error");
        return FS_EHIP;
    }
}

// Solve one UOT problem with a fresh operator; potentials returned in caller order.
double solve_uot(const float *x, const float *a, int64_t n, const float *y, const float *b,
                 int64_t m, int d, const fs_params &p, double rho, int iters, bool warm,
                 double *f, double *g, hipStream_t s, double tol = 0.0, int *sweeps = nullptr) {
    auto op = make_op(x, n, y, m, d, p, s);
    DevBuf<float> ao(n + 1), bo(m + 1);
    DevBuf<double> fo(n + 1), go(m + 1);
    op->to_op(0, a, ao.p, s);
    op->to_op(1, b, bo.p, s);
    if (warm) {
        op->to_op64(0, f, fo.p, s);
        op->to_op64(1, g, go.p, s);
    }
    double obj = 0.0;
    sinkhorn_solve(*op, ao.p, bo.p, p.lambda, rho, iters, warm, fo.p, go.p, &obj, s, tol, sweeps);
    if (f) op->from_op64(0, fo.p, f, s);
    if (g) op->from_op64(1, go.p, g, s);
    FS_HIP(hipStreamSynchronize(s));
    return obj;
}

// c* of eq. (561) (Proposition "optimal independent measure", eta_1 = eta_2 = rho, 1/lambda_paper
// = eps) and the objective of eq. (W4) at pi = c* mu x nu, which bounds UOT from above.
void cstar_bound(const float *x, const float *a, int64_t n, const float *y, const float *b,
                 int64_t m, int d, const fs_params &p, double rho, double *cstar, double *bound,
                 hipStream_t s) {
    const int r = (p.kernel == FS_GAUSS) ? 2 : 1;
    double Ma = 0.0, Mb = 0.0;
    const double D = pair_cost_mean(x, a, n, y, b, m, d, r, p, &Ma, &Mb, s);
    FS_REQUIRE(Ma > 0 && Mb > 0, FS_EINVAL, "both measures need positive mass");
    const double eps = p.lambda, den = 2.0 * rho + eps;
    const double c = std::exp(-D / (Ma * Mb * den)) * std::pow(Ma, -rho / den) *
                     std::pow(Mb, -rho / den);
    if (cstar) *cstar = c;
    if (bound)
        *bound = c * D + eps * Ma * Mb * (c * std::log(c) - c + 1.0) +
                 rho * Ma * (c * Mb * std::log(c * Mb) - c * Mb + 1.0) +
                 rho * Mb * (c * Ma * std::log(c * Ma) - c * Ma + 1.0);
}

}  // namespace

}  // namespace fs

using namespace fs;

extern "C" {

const char *fs_last_error(void) { return fs::last_error(); }

int fs_version(void) { return (1 << 16) | 0; }

void fs_release_cache(void) {
    try {
        fs::plan_release_mult_cache();
    } catch (...) {
    }
    ws_release_all();
}

int fs_profile_enable(int enable) { return fs::profile_enable(enable); }

int fs_profile_select(const char *pass, int period) { return fs::profile_select(pass, period); }

int fs_profile_query(const char *pass, double *total_ms, int64_t *count) {
    return fs::profile_query(pass, total_ms, count);
}

void fs_profile_reset(void) { fs::profile_reset(); }

int fastsum_apply(const float *x, int64_t n, const float *y, int64_t m, int d, const float *v,
                  float *out, const fs_params *p, void *stream) {
    return guarded([&] {
        check_params(p);
        check_points(x, n, "x");
        check_points(y, m, "y");
        check_points(v, m, "v");
        check_points(out, n, "out");
        FS_REQUIRE(d >= 1, FS_EINVAL, "d must be >= 1");
        hipStream_t s = as_stream(stream);
        if (n == 0) return;
        if (m == 0) {
            fill_f32(out, n, 0.0f, s);
            return;
        }
        auto op = make_op(x, n, y, m, d, *p, s);
        if (op->fast) {
            DevBuf<float> wo(m + 1), to(n + 1);
            op->to_op(1, v, wo.p, s);
            op->apply(wo.p, to.p, nullptr, 0, s);
            op->from_op(0, to.p, out, s);
            FS_HIP(hipStreamSynchronize(s));  // temporaries are released after this
        } else {
            op->apply(v, out, nullptr, 0, s);
            FS_HIP(hipStreamSynchronize(s));
        }
    });
}

struct fs_plan_s {
    std::unique_ptr<Op> op;
};

int fs_plan_create(const float *x, int64_t n, const float *y, int64_t m, int d,
                   const fs_params *p, void *stream, fs_plan *plan_out) {
    return guarded([&] {
        FS_REQUIRE(plan_out != nullptr, FS_EINVAL, "plan_out is NULL");
        *plan_out = nullptr;
        check_params(p);
        check_points(x, n, "x");
        check_points(y, m, "y");
        FS_REQUIRE(d >= 1, FS_EINVAL, "d must be >= 1");
        hipStream_t s = as_stream(stream);
        auto pl = std::make_unique<fs_plan_s>();
        pl->op = make_op(x, n, y, m, d, *p, s);
        if (!pl->op->fast) {
            // the direct path reads the points at apply time: keep private copies
            pl->op->xcopy.alloc(n * d + 1);
            if (n > 0)
                FS_HIP(hipMemcpyAsync(pl->op->xcopy.p, x, n * d * sizeof(float), hipMemcpyDeviceToDevice, s));
            pl->op->x = pl->op->xcopy.p;
            if (pl->op->same) {
                pl->op->y = pl->op->xcopy.p;
            } else {
                pl->op->ycopy.alloc(m * d + 1);
                if (m > 0)
                    FS_HIP(hipMemcpyAsync(pl->op->ycopy.p, y, m * d * sizeof(float), hipMemcpyDeviceToDevice, s));
                pl->op->y = pl->op->ycopy.p;
            }
        }
        FS_HIP(hipStreamSynchronize(s));
        *plan_out = pl.release();
    });
}

int fs_plan_apply(fs_plan plan, const float *v, float *out, int transpose, void *stream) {
    return guarded([&] {
        FS_REQUIRE(plan != nullptr && plan->op, FS_EINVAL, "plan is NULL");
        Op &op = *plan->op;
        const int64_t nt = transpose ? op.m : op.n, ns = transpose ? op.n : op.m;
        check_points(v, ns, "v");
        check_points(out, nt, "out");
        hipStream_t s = as_stream(stream);
        if (nt == 0) return;
        if (ns == 0) {
            fill_f32(out, nt, 0.0f, s);
            return;
        }
        if (op.fast) {
            // stream-ordered: the temporaries return to the workspace cache once the stream has
            // passed the work queued here, so the call does not wait for it
            DevBuf<float> wo(ns + 1), to(nt + 1);
            op.to_op(transpose ? 0 : 1, v, wo.p, s);
            op.apply(wo.p, to.p, nullptr, transpose, s);
            op.from_op(transpose ? 1 : 0, to.p, out, s);
            wo.reset_after(s);
            to.reset_after(s);
        } else {
            op.apply(v, out, nullptr, transpose, s);
        }
    });
}

int fs_plan_apply_noalloc(fs_plan plan, const float *v, float *out, int transpose,
                          void *stream) {
    return guarded([&] {
        FS_REQUIRE(plan != nullptr && plan->op, FS_EINVAL, "plan is NULL");
        Op &op = *plan->op;
        const int64_t nt = transpose ? op.m : op.n, ns = transpose ? op.n : op.m;
        check_points(v, ns, "v");
        check_points(out, nt, "out");
        hipStream_t s = as_stream(stream);
        if (nt == 0) return;
        if (ns == 0) {
            fill_f32(out, nt, 0.0f, s);
            return;
        }
        if (op.fast) {
            // operator-order weights and sums, each rounded up to 256 bytes
            const size_t wbytes = ((size_t)(ns + 1) * sizeof(float) + 255) & ~size_t(255);
            const size_t tbytes = ((size_t)(nt + 1) * sizeof(float) + 255) & ~size_t(255);
            FS_REQUIRE(wbytes + tbytes <= FS_NOALLOC_SCRATCH_BYTES, FS_EINVAL,
                       "fs_plan_apply_noalloc: %lld sources + %lld targets need %zu bytes of "
                       "scratch, more than the %zu available (at most about 4.19 million points "
                       "in total)",
                       (long long)ns, (long long)nt, wbytes + tbytes, FS_NOALLOC_SCRATCH_BYTES);
            char *sp = noalloc_scratch();
            float *wo = reinterpret_cast<float *>(sp);
            float *to = reinterpret_cast<float *>(sp + wbytes);
            op.to_op(transpose ? 0 : 1, v, wo, s);
            op.apply(wo, to, nullptr, transpose, s);
            op.from_op(transpose ? 1 : 0, to, out, s);
        } else if (op.mfma) {
            double *part = reinterpret_cast<double *>(noalloc_scratch());
            op.apply(v, out, nullptr, transpose, s, part, FS_NOALLOC_SCRATCH_BYTES / sizeof(double));
        } else {
            op.apply(v, out, nullptr, transpose, s);
        }
    });
}

int fs_plan_multiplier(fs_plan plan, float *mult_host, double *phihat_host, int64_t count,
                       double *period_host, int *bandwidth_host, void *stream) {
    return guarded([&] {
        FS_REQUIRE(plan != nullptr && plan->op, FS_EINVAL, "plan is NULL");
        FS_REQUIRE(plan->op->fast, FS_EINVAL, "a direct-summation plan has no multiplier");
        plan_multiplier(*plan->op->plan, mult_host, phihat_host, count, period_host,
                        bandwidth_host, as_stream(stream));
    });
}

void fs_plan_destroy(fs_plan plan) {
    if (!plan) return;
    // applications are stream-ordered and may still be queued: wait before the plan's device
    // buffers go back to the workspace cache
    (void)hipDeviceSynchronize();
    delete plan;
}

int uot_sinkhorn(const float *x, const float *a, int64_t n, const float *y, const float *b,
                 int64_t m, int d, const fs_params *p, double rho, int iters, double *f, double *g,
                 double *objective_host, void *stream) {
    return guarded([&] {
        check_params(p);
        check_transport(p, rho);
        check_points(x, n, "x");
        check_points(a, n, "a");
        check_points(y, m, "y");
        check_points(b, m, "b");
        check_points(f, n, "f");
        check_points(g, m, "g");
        FS_REQUIRE(iters >= 0, FS_EINVAL, "iters must be >= 0");
        FS_REQUIRE(d >= 1, FS_EINVAL, "d must be >= 1");
        const bool warm = (p->flags & FS_FLAG_WARM_START) != 0;
        const double obj = solve_uot(x, a, n, y, b, m, d, *p, rho, iters, warm, f, g,
                                     as_stream(stream));
        if (objective_host) *objective_host = obj;
    });
}

int uot_upper_bound(const float *x, const float *a, int64_t n, const float *y, const float *b,
                    int64_t m, int d, const fs_params *p, double rho, double *cstar_host,
                    double *bound_host, void *stream) {
    return guarded([&] {
        check_params(p);
        check_transport(p, rho);
        check_points(x, n, "x");
        check_points(a, n, "a");
        check_points(y, m, "y");
        check_points(b, m, "b");
        FS_REQUIRE(d >= 1, FS_EINVAL, "d must be >= 1");
        cstar_bound(x, a, n, y, b, m, d, *p, rho, cstar_host, bound_host, as_stream(stream));
    });
}

int uot_sinkhorn_scaling(const float *x, const float *a, int64_t n, const float *y, const float *b,
                         int64_t m, int d, const fs_params *p, const double *eps_stages,
                         int nstages, double rho, int max_sweeps, double tol, int init, double *f,
                         double *g, int *sweeps_host, double *objective_host, void *stream) {
    return guarded([&] {
        check_params(p);
        FS_REQUIRE(nstages >= 1 && eps_stages != nullptr, FS_EINVAL, "need at least one stage");
        for (int k = 0; k < nstages; ++k)
            FS_REQUIRE(eps_stages[k] > 0 && std::isfinite(eps_stages[k]), FS_EINVAL,
                       "stage %d: temperature must be > 0", k);
        fs_params q = *p;
        q.lambda = eps_stages[0];
        check_transport(&q, rho);
        check_points(x, n, "x");
        check_points(a, n, "a");
        check_points(y, m, "y");
        check_points(b, m, "b");
        check_points(f, n, "f");
        check_points(g, m, "g");
        FS_REQUIRE(d >= 1, FS_EINVAL, "d must be >= 1");
        FS_REQUIRE(max_sweeps >= 0, FS_EINVAL, "max_sweeps must be >= 0");
        FS_REQUIRE(tol >= 0 && std::isfinite(tol), FS_EINVAL, "tol must be finite and >= 0");
        FS_REQUIRE(init == FS_INIT_ZERO || init == FS_INIT_CSTAR || init == FS_INIT_WARM,
                   FS_EINVAL, "unknown init %d", init);
        hipStream_t s = as_stream(stream);
        bool warm = init == FS_INIT_WARM;
        if (init == FS_INIT_CSTAR) {
            double c = 0.0;
            cstar_bound(x, a, n, y, b, m, d, q, rho, &c, nullptr, s);
            fill_f64(f, n, 0.0, s);
            fill_f64(g, m, eps_stages[0] * std::log(c), s);
            warm = true;
        }
        double obj = 0.0;
        for (int k = 0; k < nstages; ++k) {
            q.lambda = eps_stages[k];
            int done = 0;
            obj = solve_uot(x, a, n, y, b, m, d, q, rho, max_sweeps, warm, f, g, s, tol, &done);
            if (sweeps_host) sweeps_host[k] = done;
            warm = true;
        }
        if (objective_host) *objective_host = obj;
    });
}

int uot_sinkhorn_grad(const float *x, const float *a, int64_t n, const float *y, const float *b,
                      int64_t m, int d, const fs_params *p, double rho, const double *f,
                      const double *g, double scale, float *dx, float *da, float *dy, float *db,
                      void *stream) {
    return guarded([&] {
        check_params(p);
        check_transport(p, rho);
        check_points(x, n, "x");
        check_points(a, n, "a");
        check_points(y, m, "y");
        check_points(b, m, "b");
        check_points(f, n, "f");
        check_points(g, m, "g");
        FS_REQUIRE(d >= 1, FS_EINVAL, "d must be >= 1");
        hipStream_t s = as_stream(stream);
        auto op = make_op(x, n, y, m, d, *p, s);
        uot_grad_core(*op, a, b, f, g, p->lambda, rho, scale, dx, da, dy, db, s);
        FS_HIP(hipStreamSynchronize(s));
    });
}

int sinkhorn_divergence(const float *x, const float *a, int64_t n, const float *y, const float *b,
                        int64_t m, int d, const fs_params *p, double rho, int iters,
                        double *f_ab, double *g_ab, double *f_aa, double *f_bb,
                        double *value_host, double *terms3_host, void *stream) {
    return guarded([&] {
        check_params(p);
        check_transport(p, rho);
        check_points(x, n, "x");
        check_points(a, n, "a");
        check_points(y, m, "y");
        check_points(b, m, "b");
        FS_REQUIRE(iters >= 0, FS_EINVAL, "iters must be >= 0");
        FS_REQUIRE(d >= 1, FS_EINVAL, "d must be >= 1");
        hipStream_t s = as_stream(stream);
        fs_params q = *p;
        q.flags &= ~FS_FLAG_WARM_START;
        DevBuf<double> t1(n + 1), t2(m + 1), t3(n + 1), t4(n + 1), t5(m + 1), t6(m + 1);
        double *fab = f_ab ? f_ab : t1.p, *gab = g_ab ? g_ab : t2.p;
        double *faa = f_aa ? f_aa : t3.p, *fbb = f_bb ? f_bb : t5.p;
        // the three transport problems are independent: they run side by side
        double uab = 0.0, uaa = 0.0, ubb = 0.0;
        run_side_by_side(
            s, {[&](hipStream_t st) {
                    uab = solve_uot(x, a, n, y, b, m, d, q, rho, iters, false, fab, gab, st);
                },
                [&](hipStream_t st) {
                    uaa = solve_uot(x, a, n, x, a, n, d, q, rho, iters, false, faa, t4.p, st);
                },
                [&](hipStream_t st) {
                    ubb = solve_uot(y, b, m, y, b, m, d, q, rho, iters, false, fbb, t6.p, st);
                }});
        const double Ma = device_sum(a, n, s), Mb = device_sum(b, m, s);
        // eq. (586) with the paper's 1/lambda equal to the temperature lambda here
        const double val = uab - 0.5 * uaa - 0.5 * ubb + 0.5 * p->lambda * (Ma - Mb) * (Ma - Mb);
        if (value_host) *value_host = val;
        if (terms3_host) {
            terms3_host[0] = uab;
            terms3_host[1] = uaa;
            terms3_host[2] = ubb;
        }
    });
}

int sinkhorn_divergence_grad(const float *x, const float *a, int64_t n, const float *y,
                             const float *b, int64_t m, int d, const fs_params *p, double rho,
                             const double *f_ab, const double *g_ab, const double *f_aa,
                             const double *f_bb, double scale, float *dx, float *da, float *dy,
                             float *db, void *stream) {
    return guarded([&] {
        check_params(p);
        check_transport(p, rho);
        check_points(x, n, "x");
        check_points(a, n, "a");
        check_points(y, m, "y");
        check_points(b, m, "b");
        check_points(f_ab, n, "f_ab");
        check_points(g_ab, m, "g_ab");
        check_points(f_aa, n, "f_aa");
        check_points(f_bb, m, "f_bb");
        FS_REQUIRE(d >= 1, FS_EINVAL, "d must be >= 1");
        hipStream_t s = as_stream(stream);
        const double Ma = device_sum(a, n, s), Mb = device_sum(b, m, s);
        const double eps = p->lambda;
        // d/d(x, a) of UOT(a,b) - UOT(a,a)/2: the self term moves both of its slots, which at the
        // symmetric optimum is twice the one-slot envelope gradient, so the 1/2 cancels.
        DevBuf<float> gx1(n * d + 1), ga1(n + 1), gx2(n * d + 1), ga2(n + 1);
        DevBuf<float> gy1(m * d + 1), gb1(m + 1), gy2(m * d + 1), gb2(m + 1);
        // the envelope gradients are independent: the (a, b) term's two sides (each with an
        // operator of its own, as one plan may not be applied from two streams at once) and the
        // two self terms run side by side
        run_side_by_side(
            s, {[&](hipStream_t st) {
                    if (!(dx || da)) return;
                    auto op = make_op(x, n, y, m, d, *p, st);
                    uot_grad_core(*op, a, b, f_ab, g_ab, eps, rho, 1.0, dx ? gx1.p : nullptr,
                                  da ? ga1.p : nullptr, nullptr, nullptr, st);
                    FS_HIP(hipStreamSynchronize(st));
                },
                [&](hipStream_t st) {
                    if (!(dy || db)) return;
                    auto op = make_op(x, n, y, m, d, *p, st);
                    uot_grad_core(*op, a, b, f_ab, g_ab, eps, rho, 1.0, nullptr, nullptr,
                                  dy ? gy1.p : nullptr, db ? gb1.p : nullptr, st);
                    FS_HIP(hipStreamSynchronize(st));
                },
                [&](hipStream_t st) {
                    if (!(dx || da)) return;
                    auto op = make_op(x, n, x, n, d, *p, st);
                    uot_grad_core(*op, a, a, f_aa, f_aa, eps, rho, 1.0, dx ? gx2.p : nullptr,
                                  da ? ga2.p : nullptr, nullptr, nullptr, st);
                    FS_HIP(hipStreamSynchronize(st));
                },
                [&](hipStream_t st) {
                    if (!(dy || db)) return;
                    auto op = make_op(y, m, y, m, d, *p, st);
                    uot_grad_core(*op, b, b, f_bb, f_bb, eps, rho, 1.0, dy ? gy2.p : nullptr,
                                  db ? gb2.p : nullptr, nullptr, nullptr, st);
                    FS_HIP(hipStreamSynchronize(st));
                }});
        if (dx) combine(gx1.p, gx2.p, n * d, scale, -scale, 0.0, dx, s);
        if (da) combine(ga1.p, ga2.p, n, scale, -scale, scale * eps * (Ma - Mb), da, s);
        if (dy) combine(gy1.p, gy2.p, m * d, scale, -scale, 0.0, dy, s);
        if (db) combine(gb1.p, gb2.p, m, scale, -scale, -scale * eps * (Ma - Mb), db, s);
        FS_HIP(hipStreamSynchronize(s));
    });
}

int mmd(const float *x, const float *a, int64_t n, const float *y, const float *b, int64_t m,
        int d, const fs_params *p, double *mmd2_host, double *terms3_host, void *stream) {
    return guarded([&] {
        check_params(p);
        check_points(x, n, "x");
        check_points(a, n, "a");
        check_points(y, m, "y");
        check_points(b, m, "b");
        FS_REQUIRE(d >= 1, FS_EINVAL, "d must be >= 1");
        mmd_core(x, a, n, y, b, m, d, *p, mmd2_host, terms3_host, as_stream(stream));
    });
}

int mmd_grad(const float *x, const float *a, int64_t n, const float *y, const float *b, int64_t m,
             int d, const fs_params *p, double scale, float *dx, float *da, float *dy, float *db,
             void *stream) {
    return guarded([&] {
        check_params(p);
        check_points(x, n, "x");
        check_points(a, n, "a");
        check_points(y, m, "y");
        check_points(b, m, "b");
        FS_REQUIRE(d >= 1, FS_EINVAL, "d must be >= 1");
        mmd_grad_core(x, a, n, y, b, m, d, *p, scale, dx, da, dy, db, as_stream(stream));
    });
}

}  // extern "C"
