// Stable ranks for the counting sorts of the plan build (deterministic mode): the order of the
// nodes that share a key follows their input index, so a plan built twice from the same points
// is identical.  The keys and the identity permutation are sorted as pairs by a stable LSD radix
// sort (hipCUB over rocPRIM); the rank of node i inside its key is then its sorted position minus
// the key's start.
#include <hipcub/hipcub.hpp>

#include "internal.h"

namespace fs {

namespace {

__global__ void k_iota(int *__restrict__ v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        v[i] = (int)i;
}

__global__ void k_stable_rank(const int *__restrict__ skey, const int *__restrict__ sidx,
                              int64_t n, const int *__restrict__ kstart, int *__restrict__ rank) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x)
        rank[sidx[p]] = (int)(p - kstart[skey[p]]);
}

}  // namespace

void stable_ranks(const int *key, int64_t n, int64_t nkeys, const int *kstart, int *rank,
                  hipStream_t s) {
    if (n <= 0) return;
    FS_REQUIRE(n < (int64_t(1) << 31), FS_EINVAL, "stable ranks: too many points");
    int bits = 1;
    while (bits < 31 && (int64_t(1) << bits) < nkeys) ++bits;
    DevBuf<int> idx(n), skey(n), sidx(n);
    hipLaunchKernelGGL(k_iota, dim3(blocks_for(n, 256, 8192)), dim3(256), 0, s, idx.p, n);
    FS_LAUNCHED();
    const unsigned *kin = reinterpret_cast<const unsigned *>(key);
    unsigned *kout = reinterpret_cast<unsigned *>(skey.p);
    size_t tbytes = 0;
    FS_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tbytes, kin, kout, idx.p, sidx.p, (int)n, 0,
                                              bits, s));
    DevBuf<char> tmp(std::max<size_t>(tbytes, 1));
    FS_HIP(hipcub::DeviceRadixSort::SortPairs(tmp.p, tbytes, kin, kout, idx.p, sidx.p, (int)n, 0,
                                              bits, s));
    hipLaunchKernelGGL(k_stable_rank, dim3(blocks_for(n, 256, 8192)), dim3(256), 0, s, skey.p,
                       sidx.p, n, kstart, rank);
    FS_LAUNCHED();
    // the temporaries are still used by the queued sort and rank kernels
    idx.reset_after(s);
    skey.reset_after(s);
    sidx.reset_after(s);
    tmp.reset_after(s);
}

}  // namespace fs
