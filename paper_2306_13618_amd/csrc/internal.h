// Internal declarations shared by the HIP sources of libfastuot (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/fastuot.h"

namespace fs {

// ------------------------------------------------------------------ errors
struct Error {
    int code;
};
void set_error(const char *fmt, ...);
void clear_error();

#define FS_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess) {                                                        \
            ::fs::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),     \
                            __FILE__, __LINE__);                                       \
            throw ::fs::Error{FS_EHIP};                                                \
        }                                                                              \
    } while (0)

#define FS_REQUIRE(cond, code, ...)          \
    do {                                     \
        if (!(cond)) {                       \
            ::fs::set_error(__VA_ARGS__);    \
            throw ::fs::Error{code};         \
        }                                    \
    } while (0)

#define FS_LAUNCHED() FS_HIP(hipGetLastError())

// ------------------------------------------------------------------ workspace
// Device allocations come from a per-process cache of freed blocks (exact-size reuse), so that
// repeated solves do not pay for hipMalloc/hipFree.
// ws_free_after returns a block whose last use is queued on stream s: it is handed out again only
// after the work queued on s so far has finished (an event recorded there), so a caller may
// return without waiting for the stream.
void *ws_alloc(size_t bytes);
void ws_free(void *p);
void ws_free_after(void *p, hipStream_t s);
void ws_release_all();

template <class T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    explicit DevBuf(size_t count) { alloc(count); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) { reset(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
        return *this;
    }
    ~DevBuf() { reset(); }
    void alloc(size_t count) {
        reset();
        n = count;
        p = count ? static_cast<T *>(ws_alloc(count * sizeof(T))) : nullptr;
    }
    void ensure(size_t count) {
        if (count > n) alloc(count);
    }
    void reset() {
        if (p) ws_free(p);
        p = nullptr;
        n = 0;
    }
    // release a block whose last use is queued on s (reused only after that work has finished)
    void reset_after(hipStream_t s) {
        if (p) ws_free_after(p, s);
        p = nullptr;
        n = 0;
    }
    T *get() const { return p; }
    // give up ownership (the caller frees the block with ws_free)
    T *release() {
        T *q = p;
        p = nullptr;
        n = 0;
        return q;
    }
};

// ------------------------------------------------------------------ pinned staging
// Small host <-> device copies of a plan build go through pinned host memory: a copy from or to
// pageable memory makes the host wait for the stream, a pinned one is queued like a kernel.  The
// pinned blocks come from a per-process pool and go back to it when the stage is destroyed,
// after a synchronisation of its stream (a queued copy may still read them until then).  Device
// temporaries whose last use is queued can be handed to the stage too: they are freed after that
// same synchronisation, so the build synchronises once at its end instead of after each step.
class HostStage {
public:
    explicit HostStage(hipStream_t s) : s_(s) {}
    HostStage(const HostStage &) = delete;
    HostStage &operator=(const HostStage &) = delete;
    ~HostStage();
    // pinned host memory for `bytes`, valid until the stage is destroyed
    void *pinned(size_t bytes);
    // queue a copy of host memory (any kind) to the device through the stage
    void upload(void *dst, const void *src, size_t bytes);
    // queue a copy of device memory into pinned memory; its contents are valid after a
    // synchronisation of the stream
    template <class T>
    T *download(const T *src, size_t count) {
        T *h = static_cast<T *>(pinned(count * sizeof(T)));
        if (count) FS_HIP(hipMemcpyAsync(h, src, count * sizeof(T), hipMemcpyDeviceToHost, s_));
        return h;
    }
    // free the device buffer after the final synchronisation
    template <class T>
    void hold(DevBuf<T> &b) {
        if (T *q = b.release()) held_.push_back(q);
    }

private:
    hipStream_t s_;
    std::vector<std::pair<char *, size_t>> blocks_;  // pinned blocks held: pointer, size
    size_t used_ = 0;                                  // bytes used in the last block
    std::vector<void *> held_;                         // device blocks to free at the end
};

// ------------------------------------------------------------------ stable ranks
// rank[i] = position of node i among the nodes with its key, in input order (a stable counting
// sort's ranks), given the keys (0 <= key < nkeys) and each key's exclusive start kstart.
void stable_ranks(const int *key, int64_t n, int64_t nkeys, const int *kstart, int *rank,
                  hipStream_t s);

// ------------------------------------------------------------------ launch helpers
inline unsigned blocks_for(int64_t work, int threads, int64_t cap = 1 << 20) {
    int64_t b = (work + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return static_cast<unsigned>(b);
}

// Several device-to-device copies in one launch (byte counts multiples of 4): ranges collected
// by add(), copied by launch() (also called by add() when the batch is full).
class CopyBatch {
public:
    static constexpr int MAX = 8;
    struct Args {
        const void *src[MAX];
        void *dst[MAX];
        int64_t words[MAX];
        int k;
    };
    explicit CopyBatch(hipStream_t s) : s_(s) { a_.k = 0; }
    void add(void *dst, const void *src, size_t bytes);
    void launch();

private:
    hipStream_t s_;
    Args a_;
    int64_t nmax_ = 0;
};

// Streams the library keeps per device (default priority, not synchronising with the null
// stream), created on first use: they carry the independent pieces of a Sinkhorn divergence
// (its self terms, and in the backward its gradients) beside the caller's stream.  Work on them
// is ordered against the caller's stream by events.
constexpr int LIB_STREAMS = 3;
hipStream_t library_stream(int k);

// Device fill (used instead of hipMemsetAsync so that callers may capture the work in a graph).
void fill_f32(float *p, int64_t n, float v, hipStream_t s);
void fill_f64(double *p, int64_t n, double v, hipStream_t s);
void fill_i32(int *p, int64_t n, int v, hipStream_t s);
// Several fills in one launch: ranges are collected by add_* and written by launch() (also
// called by add_* when the batch is full).  Elements of 4 or 8 bytes.
class FillBatch {
public:
    static constexpr int MAX = 12;
    struct Args {
        void *p[MAX];
        int64_t n[MAX];
        uint64_t v[MAX];
        int wide[MAX];  // 8-byte elements
        int k;
    };
    explicit FillBatch(hipStream_t s) : s_(s) { a_.k = 0; }
    void add_f64(double *p, int64_t n, double v);
    void add_f32(float *p, int64_t n, float v);
    void add_i32(int *p, int64_t n, int v);
    void launch();

private:
    void add(void *p, int64_t n, uint64_t bits, int wide);
    hipStream_t s_;
    Args a_;
    int64_t nmax_ = 0;
};

// ------------------------------------------------------------------ pass timing
// When enabled (fs_profile_enable), a ProfScope records HIP events on the launch stream around
// the kernels of one pass; the events are folded into per-name totals on query.
bool prof_enabled();
struct ProfScope {
    int slot = -1;
    hipStream_t s = nullptr;
    ProfScope(const char *name, hipStream_t stream);
    ~ProfScope();
};

// ------------------------------------------------------------------ Sinkhorn weights
// base * e^x for an FP64 exponent x <= 0, to FP32 accuracy: x = k ln 2 + r with the integer k
// and |r| <= ln(2)/2 formed in FP64, e^r in FP32 (r is small, so its FP32 rounding costs at most
// 3e-8 relative), then scaled by 2^k.  About a fifth of the arithmetic of an FP64 exponential.
__device__ __forceinline__ float weight_exp(float base, double x) {
    const double kd = rint(x * 1.4426950408889634);  // x / ln 2, rounded
    const float r = (float)fma(-kd, 0.6931471805599453, x);
    const int k = (int)fmax(kd, -300.0);
    return ldexpf(base * expf(r), k);
}

// log v of a positive FP32 kernel sum, returned in FP64 to FP32 accuracy: v = f 2^e with f in
// [0.5, 1) (frexp), log v = e ln 2 + log f with log f in FP32 (|log f| <= ln 2, so its error is
// about 4e-8 absolute, below the relative error of the FP32 sum itself).
__device__ __forceinline__ double sum_log(float v) {
    int e = 0;
    const float f = frexpf(v, &e);
    return (double)e * 0.6931471805599453 + (double)logf(f);
}

// ------------------------------------------------------------------ Kaiser-Bessel window
// Window in grid units (s = distance to the grid point times the grid size), cutoff m, shape b,
// normalised to phi(0) = 1:
//   phi(s) = [sinh(b q)/q] / [sinh(b m)/m],  q = sqrt(m^2 - s^2),  |s| < m;  0 otherwise.
// The NFFT literature's form (1/pi) sinh(b q)/q differs by the constant factor; the Fourier
// transform used for deconvolution is scaled consistently on the host.
struct KB {
    float m, b, inv_one_minus;  // inv_one_minus = 1/(1 - exp(-2 b m))
};

__device__ __forceinline__ float kb_phi(const KB &w, float s) {
    float q2 = w.m * w.m - s * s;
    q2 = fmaxf(q2, 0.0f);
    float q = sqrtf(q2);
    // sinh(bq)/sinh(bm) * m/q = exp(b(q - m)) * (1 - exp(-2bq)) / (1 - exp(-2bm)) * m / q
    float e = __expf(w.b * (q - w.m));
    float bq = w.b * q;
    float ratio;  // (1 - exp(-2bq)) / q, with the q -> 0 limit 2b
    if (bq > 1e-3f)
        ratio = -expm1f(-2.0f * bq) / q;
    else
        ratio = 2.0f * w.b * (1.0f - bq);
    return e * ratio * w.m * w.inv_one_minus;
}

// d phi / d s for the same window.
__device__ __forceinline__ float kb_dphi(const KB &w, float s) {
    float q2 = fmaxf(w.m * w.m - s * s, 0.0f);
    float q = sqrtf(q2);
    float bq = w.b * q;
    float e = __expf(w.b * (q - w.m));
    // phi = C e^{b(q-m)} (1 - e^{-2bq})/q,  C = m/(1-e^{-2bm})
    // dphi/dq = C e^{b(q-m)} [ b(1+e^{-2bq})/q - (1-e^{-2bq})/q^2 ],  dq/ds = -s/q
    float t;
    if (bq > 0.1f) {
        float em = __expf(-2.0f * bq);
        t = (w.b * (1.0f + em) * q + expm1f(-2.0f * bq)) / (q2 * q);  // [b(1+e)q - (1-e)]/q^3
    } else {
        // [b(1+e)q - (1-e)] = 2 e^{-bq} (bq cosh bq - sinh bq) = 2 e^{-bq} ((bq)^3/3 + (bq)^5/30 + ..)
        t = (2.0f / 3.0f) * w.b * w.b * w.b * __expf(-bq) * (1.0f + 0.1f * bq * bq);
    }
    return -s * e * t * w.m * w.inv_one_minus;
}

}  // namespace fs
