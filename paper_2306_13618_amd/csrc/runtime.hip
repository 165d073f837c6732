// Error state, workspace cache and small utility kernels of libfastuot.
#include <algorithm>
#include <cstdarg>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>

#include "internal.h"

namespace fs {

static thread_local char g_err[1024] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}
void clear_error() { g_err[0] = 0; }
const char *last_error() { return g_err; }

// ------------------------------------------------------------------ workspace cache
namespace {
struct Pending {
    hipEvent_t done;  // recorded on the stream of the block's last use
    void *p;
    size_t sz;
};
struct Cache {
    std::mutex mu;
    std::map<void *, size_t> live;              // pointer -> size
    size_t live_bytes = 0;
    std::multimap<size_t, void *> free_blocks;  // size -> pointer
    std::vector<Pending> pending;               // freed, but queued work may still use them
    std::vector<hipEvent_t> events;             // idle events for `pending`
    size_t free_bytes = 0;
};
Cache &cache() {
    static Cache *c = new Cache();  // never destroyed: blocks live until process exit
    return *c;
}
// Move the pending blocks whose last use has finished to the free list (lock held).
void reclaim_pending(Cache &c) {
    size_t k = 0;
    for (size_t i = 0; i < c.pending.size(); ++i) {
        Pending &q = c.pending[i];
        const hipError_t e = hipEventQuery(q.done);
        if (e == hipErrorNotReady) {
            (void)hipGetLastError();
            c.pending[k++] = q;
            continue;
        }
        c.free_blocks.emplace(q.sz, q.p);
        c.free_bytes += q.sz;
        c.events.push_back(q.done);
    }
    c.pending.resize(k);
}
}  // namespace

// Failure injection: FASTUOT_WORKSPACE_LIMIT (bytes) caps the live workspace; an allocation that
// would exceed it fails as a device allocation failure would (FS_ENOMEM).
static size_t workspace_limit() {
    const char *e = std::getenv("FASTUOT_WORKSPACE_LIMIT");
    if (!e || !*e) return SIZE_MAX;
    char *end = nullptr;
    const unsigned long long v = std::strtoull(e, &end, 10);
    return (end && *end == 0) ? (size_t)v : SIZE_MAX;
}

void *ws_alloc(size_t bytes) {
    // round to 256 B so that nearby sizes share blocks
    size_t sz = (bytes + 255) & ~size_t(255);
    Cache &c = cache();
    {
        std::lock_guard<std::mutex> lk(c.mu);
        const size_t limit = workspace_limit();
        if (c.live_bytes + sz > limit) {
            set_error("device allocation of %zu bytes refused: the workspace limit "
                      "(FASTUOT_WORKSPACE_LIMIT = %zu bytes, %zu in use) would be exceeded",
                      sz, limit, c.live_bytes);
            throw Error{FS_ENOMEM};
        }
        if (!c.pending.empty()) reclaim_pending(c);
        auto it = c.free_blocks.find(sz);
        if (it != c.free_blocks.end()) {
            void *p = it->second;
            c.free_blocks.erase(it);
            c.free_bytes -= sz;
            c.live[p] = sz;
            c.live_bytes += sz;
            return p;
        }
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, sz);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        // give cached blocks back and retry once
        ws_release_all();
        e = hipMalloc(&p, sz);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            set_error("device allocation of %zu bytes failed: %s", sz, hipGetErrorString(e));
            throw Error{FS_ENOMEM};
        }
    }
    std::lock_guard<std::mutex> lk(c.mu);
    c.live[p] = sz;
    c.live_bytes += sz;
    return p;
}

void ws_free(void *p) {
    if (!p) return;
    Cache &c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.live.find(p);
    if (it == c.live.end()) return;
    c.free_blocks.emplace(it->second, p);
    c.free_bytes += it->second;
    c.live_bytes -= it->second;
    c.live.erase(it);
}

void ws_free_after(void *p, hipStream_t s) {
    if (!p) return;
    Cache &c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.live.find(p);
    if (it == c.live.end()) return;
    hipEvent_t ev = nullptr;
    if (!c.events.empty()) {
        ev = c.events.back();
        c.events.pop_back();
    } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        ev = nullptr;
    }
    if (!ev || hipEventRecord(ev, s) != hipSuccess) {
        // no event to order the reuse after the stream: wait for the stream instead
        (void)hipGetLastError();
        if (ev) c.events.push_back(ev);
        (void)hipStreamSynchronize(s);
        c.free_blocks.emplace(it->second, p);
        c.free_bytes += it->second;
        c.live_bytes -= it->second;
        c.live.erase(it);
        return;
    }
    c.pending.push_back(Pending{ev, p, it->second});
    c.live_bytes -= it->second;
    c.live.erase(it);
}

void ws_release_all() {
    Cache &c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    // the caller guarantees no queued work still uses cached blocks (they were freed by it);
    // blocks freed behind an event are complete after the device synchronisation
    (void)hipDeviceSynchronize();
    reclaim_pending(c);
    for (auto &kv : c.free_blocks) (void)hipFree(kv.second);
    c.free_blocks.clear();
    c.free_bytes = 0;
}

// ------------------------------------------------------------------ pinned staging
namespace {
struct PinnedPool {
    std::mutex mu;
    std::multimap<size_t, char *> free_blocks;  // size -> pointer, never freed
};
PinnedPool &pinned_pool() {
    static PinnedPool *p = new PinnedPool();
    return *p;
}
constexpr size_t PIN_BLOCK = size_t(1) << 20;
}  // namespace

void *HostStage::pinned(size_t bytes) {
    used_ = (used_ + 63) & ~size_t(63);
    if (blocks_.empty() || used_ + bytes > blocks_.back().second) {
        const size_t want = std::max(PIN_BLOCK, (bytes + PIN_BLOCK - 1) & ~(PIN_BLOCK - 1));
        char *b = nullptr;
        size_t got = 0;
        {
            PinnedPool &pp = pinned_pool();
            std::lock_guard<std::mutex> lk(pp.mu);
            auto it = pp.free_blocks.lower_bound(want);
            if (it != pp.free_blocks.end()) {
                got = it->first;
                b = it->second;
                pp.free_blocks.erase(it);
            }
        }
        if (!b) {
            void *q = nullptr;
            const hipError_t e = hipHostMalloc(&q, want, hipHostMallocDefault);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                set_error("pinned host allocation of %zu bytes failed: %s", want,
                          hipGetErrorString(e));
                throw Error{FS_ENOMEM};
            }
            b = static_cast<char *>(q);
            got = want;
        }
        blocks_.emplace_back(b, got);
        used_ = 0;
    }
    char *p = blocks_.back().first + used_;
    used_ += bytes;
    return p;
}

void HostStage::upload(void *dst, const void *src, size_t bytes) {
    if (!bytes) return;
    void *h = pinned(bytes);
    std::memcpy(h, src, bytes);
    FS_HIP(hipMemcpyAsync(dst, h, bytes, hipMemcpyHostToDevice, s_));
}

HostStage::~HostStage() {
    if (blocks_.empty() && held_.empty()) return;
    (void)hipStreamSynchronize(s_);  // queued copies and kernels may still use the blocks
    for (void *q : held_) ws_free(q);
    PinnedPool &pp = pinned_pool();
    std::lock_guard<std::mutex> lk(pp.mu);
    for (auto &b : blocks_) pp.free_blocks.emplace(b.second, b.first);
}

// ------------------------------------------------------------------ pass timing
namespace {
struct ProfRec {
    std::string name;
    hipEvent_t e0, e1;
};
struct Prof {
    std::mutex mu;
    bool on = false;
    std::string only;    // record only scopes of this name (empty: all)
    int period = 1;      // record every period-th eligible scope
    int64_t seen = 0;
    std::vector<ProfRec> recs;
    std::vector<hipEvent_t> pool;
    std::map<std::string, std::pair<double, int64_t>> totals;
};
Prof &prof() {
    static Prof *p = new Prof();
    return *p;
}
hipEvent_t take_event(Prof &p) {
    if (!p.pool.empty()) {
        hipEvent_t e = p.pool.back();
        p.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    FS_HIP(hipEventCreate(&e));
    return e;
}
void fold_records(Prof &p) {
    for (auto &r : p.recs) {
        FS_HIP(hipEventSynchronize(r.e1));
        float ms = 0.0f;
        FS_HIP(hipEventElapsedTime(&ms, r.e0, r.e1));
        auto &t = p.totals[r.name];
        t.first += ms;
        t.second += 1;
        p.pool.push_back(r.e0);
        p.pool.push_back(r.e1);
    }
    p.recs.clear();
}
}  // namespace

bool prof_enabled() { return prof().on; }

ProfScope::ProfScope(const char *name, hipStream_t stream) : s(stream) {
    Prof &p = prof();
    if (!p.on) return;
    std::lock_guard<std::mutex> lk(p.mu);
    if (!p.only.empty() && p.only != name) return;
    if (p.seen++ % p.period != 0) return;
    ProfRec r{name, take_event(p), take_event(p)};
    FS_HIP(hipEventRecord(r.e0, s));
    p.recs.push_back(r);
    slot = (int)p.recs.size() - 1;
}

ProfScope::~ProfScope() {
    if (slot < 0) return;
    Prof &p = prof();
    std::lock_guard<std::mutex> lk(p.mu);
    if (slot < (int)p.recs.size()) (void)hipEventRecord(p.recs[slot].e1, s);
}

int profile_enable(int on) {
    prof().on = (on != 0);
    return FS_OK;
}

int profile_select(const char *pass, int period) {
    if (period < 1) {
        set_error("fs_profile_select: period must be at least 1 (got %d)", period);
        return FS_EINVAL;
    }
    Prof &p = prof();
    std::lock_guard<std::mutex> lk(p.mu);
    p.only = pass ? pass : "";
    p.period = period;
    p.seen = 0;
    return FS_OK;
}

int profile_query(const char *pass, double *total_ms, int64_t *count) {
    if (!pass || !total_ms || !count) {
        set_error("fs_profile_query: NULL argument");
        return FS_EINVAL;
    }
    Prof &p = prof();
    std::lock_guard<std::mutex> lk(p.mu);
    try {
        fold_records(p);
    } catch (const Error &e) {
        return e.code;
    }
    auto it = p.totals.find(pass);
    *total_ms = (it == p.totals.end()) ? 0.0 : it->second.first;
    *count = (it == p.totals.end()) ? 0 : it->second.second;
    return FS_OK;
}

void profile_reset() {
    Prof &p = prof();
    std::lock_guard<std::mutex> lk(p.mu);
    for (auto &r : p.recs) {
        (void)hipEventSynchronize(r.e1);
        p.pool.push_back(r.e0);
        p.pool.push_back(r.e1);
    }
    p.recs.clear();
    p.totals.clear();
}

// ------------------------------------------------------------------ batched copies
__global__ void k_copy_batch(CopyBatch::Args a) {
    const int r = blockIdx.y;
    const uint32_t *src = static_cast<const uint32_t *>(a.src[r]);
    uint32_t *dst = static_cast<uint32_t *>(a.dst[r]);
    const int64_t n = a.words[r];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

void CopyBatch::add(void *dst, const void *src, size_t bytes) {
    FS_REQUIRE(bytes % 4 == 0, FS_EINVAL, "batched copy of %zu bytes", bytes);
    if (bytes == 0) return;
    if (a_.k == MAX) launch();
    a_.src[a_.k] = src;
    a_.dst[a_.k] = dst;
    a_.words[a_.k] = (int64_t)(bytes / 4);
    nmax_ = std::max(nmax_, a_.words[a_.k]);
    ++a_.k;
}
void CopyBatch::launch() {
    if (a_.k == 0) return;
    hipLaunchKernelGGL(k_copy_batch, dim3(blocks_for(nmax_, 256, 2048), a_.k), dim3(256), 0, s_,
                       a_);
    FS_LAUNCHED();
    a_.k = 0;
    nmax_ = 0;
}

// ------------------------------------------------------------------ library streams
namespace {
constexpr int LIB_DEVICES = 64;
std::mutex g_lib_stream_mu;
hipStream_t g_lib_stream[LIB_DEVICES][LIB_STREAMS] = {};
}  // namespace

hipStream_t library_stream(int k) {
    int dev = 0;
    FS_HIP(hipGetDevice(&dev));
    FS_REQUIRE(dev >= 0 && dev < LIB_DEVICES, FS_EUNSUPPORTED, "device index %d out of range", dev);
    FS_REQUIRE(k >= 0 && k < LIB_STREAMS, FS_EINVAL, "library stream %d out of range", k);
    std::lock_guard<std::mutex> lk(g_lib_stream_mu);
    if (!g_lib_stream[dev][k])
        FS_HIP(hipStreamCreateWithFlags(&g_lib_stream[dev][k], hipStreamNonBlocking));
    return g_lib_stream[dev][k];
}

// ------------------------------------------------------------------ fills
template <class T>
__global__ void k_fill(T *p, int64_t n, T v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

void fill_f32(float *p, int64_t n, float v, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill<float>, dim3(blocks_for(n, 256, 4096)), dim3(256), 0, s, p, n, v);
    FS_LAUNCHED();
}
void fill_f64(double *p, int64_t n, double v, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill<double>, dim3(blocks_for(n, 256, 4096)), dim3(256), 0, s, p, n, v);
    FS_LAUNCHED();
}
void fill_i32(int *p, int64_t n, int v, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill<int>, dim3(blocks_for(n, 256, 4096)), dim3(256), 0, s, p, n, v);
    FS_LAUNCHED();
}


__global__ void k_fill_batch(FillBatch::Args a) {
    const int r = blockIdx.y;
    const int64_t n = a.n[r];
    const int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x, step = (int64_t)gridDim.x * blockDim.x;
    if (a.wide[r]) {
        uint64_t *p = static_cast<uint64_t *>(a.p[r]);
        for (int64_t i = i0; i < n; i += step) p[i] = a.v[r];
    } else {
        uint32_t *p = static_cast<uint32_t *>(a.p[r]);
        const uint32_t v = (uint32_t)a.v[r];
        for (int64_t i = i0; i < n; i += step) p[i] = v;
    }
}

void FillBatch::add(void *p, int64_t n, uint64_t bits, int wide) {
    if (n <= 0) return;
    if (a_.k == MAX) launch();
    a_.p[a_.k] = p;
    a_.n[a_.k] = n;
    a_.v[a_.k] = bits;
    a_.wide[a_.k] = wide;
    ++a_.k;
    nmax_ = std::max(nmax_, n);
}
void FillBatch::add_f64(double *p, int64_t n, double v) {
    add(p, n, __builtin_bit_cast(uint64_t, v), 1);
}
void FillBatch::add_f32(float *p, int64_t n, float v) {
    add(p, n, __builtin_bit_cast(uint32_t, v), 0);
}
void FillBatch::add_i32(int *p, int64_t n, int v) { add(p, n, (uint32_t)v, 0); }
void FillBatch::launch() {
    if (a_.k == 0) return;
    hipLaunchKernelGGL(k_fill_batch, dim3(blocks_for(nmax_, 256, 2048), a_.k), dim3(256), 0, s_,
                       a_);
    FS_LAUNCHED();
    a_.k = 0;
    nmax_ = 0;
}

}  // namespace fs
