// Probes.  Gather: the rate at which the device streams a graph's stored
// column indices and gathers one random 8-byte (label, volume) pair per
// entry, with no other work.  Every sweep of the move kernels must do at
// least this, so it bounds their entry rate from above far more tightly than
// HBM bandwidth does (the pairs are gathered line by line from all over the
// array).  Copy: a STREAM-style copy of the same index array, the measured
// bandwidth that the HBM roofline is set against.
#include <algorithm>

#include "lv_device.h"

namespace lv {

namespace {

constexpr int PG_U = 8;  // gathers in flight per lane

__global__ __launch_bounds__(256) void k_probe_gather(const int32_t* __restrict__ idx, const int2* __restrict__ tab,
                                                      int64_t nnz, unsigned long long* sink)
{
    unsigned long long acc = 0;
    const int64_t stride = (int64_t)gridDim.x * 256 * PG_U;
    for (int64_t e0 = (int64_t)blockIdx.x * 256 * PG_U + threadIdx.x; e0 < nnz; e0 += stride) {
        int32_t j[PG_U];
#pragma unroll
        for (int u = 0; u < PG_U; ++u) j[u] = e0 + u * 256 < nnz ? __builtin_nontemporal_load(&idx[e0 + u * 256]) : -1;
        int2 v[PG_U];
#pragma unroll
        for (int u = 0; u < PG_U; ++u) v[u] = j[u] >= 0 ? tab[j[u]] : make_int2(0, 0);
#pragma unroll
        for (int u = 0; u < PG_U; ++u) acc += (unsigned)(v[u].x ^ v[u].y);
    }
    // keeps the gathers live; the sum itself is never read
    if (acc == 0x9E3779B97F4A7C15ull) atomicAdd(sink, acc);
}

constexpr int PC_U = 4;  // 16-byte copies in flight per lane

__global__ __launch_bounds__(256) void k_probe_copy(const int4* __restrict__ src, int4* __restrict__ dst, int64_t n4,
                                                    const int32_t* __restrict__ src1, int32_t* __restrict__ dst1,
                                                    int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * 256 * PC_U;
    for (int64_t t0 = (int64_t)blockIdx.x * 256 * PC_U + threadIdx.x; t0 < n4; t0 += stride) {
        int4 v[PC_U];
#pragma unroll
        for (int u = 0; u < PC_U; ++u)
            if (t0 + u * 256 < n4) v[u] = src[t0 + u * 256];
#pragma unroll
        for (int u = 0; u < PC_U; ++u)
            if (t0 + u * 256 < n4) dst[t0 + u * 256] = v[u];
    }
    // the last n mod 4 elements
    for (int64_t e = 4 * n4 + (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256)
        dst1[e] = src1[e];
}

}  // namespace

hipError_t launch_probe_copy(const int32_t* src, int32_t* dst, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t n4 = n / 4;
    const int64_t per = 256 * PC_U;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(16384, (n4 + per - 1) / per));
    k_probe_copy<<<grid, 256, 0, s>>>((const int4*)src, (int4*)dst, n4, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_probe_gather(const int32_t* idx, const int2* tab, int64_t nnz, unsigned long long* sink, hipStream_t s)
{
    if (nnz <= 0) return hipSuccess;
    k_probe_gather<<<2048, 256, 0, s>>>(idx, tab, nnz, sink);
    return hipGetLastError();
}

}  // namespace lv
