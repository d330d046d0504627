// Device-wide primitives (gfx950): fill/iota/copy, exclusive scan (K12) and a
// stable LSD radix sort of (key, value) pairs (K10) used by degree classing
// and aggregation.
#include "lv_device.h"

namespace lv {

using namespace dev;

namespace {

// ------------------------------------------------------------------ basics
__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        p[t] = v;
}
__global__ void k_iota(int32_t* p, int32_t n)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        p[t] = (int32_t)t;
}
__global__ void k_copy_i32(int32_t* d, const int32_t* s, int64_t n)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        d[t] = s[t];
}

// ------------------------------------------------------------------ scan (K12)
constexpr int SCAN_IT = 8;
constexpr int64_t SCAN_TILE = 256 * SCAN_IT;

template <typename T>
__global__ __launch_bounds__(256) void k_scan_reduce(const T* in, int64_t n, T* sums)
{
    __shared__ T red[4];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    T s = 0;
    for (int it = 0; it < SCAN_IT; ++it) {
        int64_t p = base + it * 256 + threadIdx.x;
        if (p < n) s += in[p];
    }
    T t = block_sum<256>(s, red);
    if (threadIdx.x == 0) sums[blockIdx.x] = t;
}

template <typename T>
__global__ __launch_bounds__(256) void k_scan_apply(const T* in, T* out, int64_t n, const T* block_off, T* total)
{
    __shared__ T tile[SCAN_TILE];
    __shared__ T wsum[4];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    for (int it = 0; it < SCAN_IT; ++it) {
        int64_t p = base + it * 256 + threadIdx.x;
        tile[it * 256 + threadIdx.x] = p < n ? in[p] : (T)0;
    }
    __syncthreads();
    T loc[SCAN_IT];
    T run = 0;
#pragma unroll
    for (int j = 0; j < SCAN_IT; ++j) { loc[j] = run; run += tile[threadIdx.x * SCAN_IT + j]; }
    // exclusive scan of per-thread totals across the block
    T x = run;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        T y = __shfl_up(x, d);
        if ((int)lane_id() >= d) x += y;
    }
    const int wid = threadIdx.x / WAVE;
    if (lane_id() == WAVE - 1) wsum[wid] = x;
    __syncthreads();
    T woff = 0, btot = 0;
    for (int w = 0; w < 4; ++w) { if (w < wid) woff += wsum[w]; btot += wsum[w]; }
    const T excl = woff + x - run + (block_off ? block_off[blockIdx.x] : (T)0);
#pragma unroll
    for (int j = 0; j < SCAN_IT; ++j) tile[threadIdx.x * SCAN_IT + j] = excl + loc[j];
    __syncthreads();
    for (int it = 0; it < SCAN_IT; ++it) {
        int64_t p = base + it * 256 + threadIdx.x;
        if (p < n) out[p] = tile[it * 256 + threadIdx.x];
    }
    if (total && threadIdx.x == 0) *total = btot;
}

template <typename T>
hipError_t scan_exclusive_t(const T* in, T* out, int64_t n, T* total, char* tmp, size_t tmp_bytes, hipStream_t s)
{
    if (n <= 0) {
        if (total) return hipMemsetAsync(total, 0, sizeof(T), s);
        return hipSuccess;
    }
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb == 1) {
        k_scan_apply<T><<<1, 256, 0, s>>>(in, out, n, nullptr, total);
        return hipGetLastError();
    }
    const size_t need = ((size_t)nb * sizeof(T) + 255) & ~(size_t)255;
    if (need > tmp_bytes) return hipErrorInvalidValue;
    T* sums = (T*)tmp;
    k_scan_reduce<T><<<(unsigned)nb, 256, 0, s>>>(in, n, sums);
    hipError_t e = scan_exclusive_t<T>(sums, sums, nb, total, tmp + need, tmp_bytes - need, s);
    if (e != hipSuccess) return e;
    k_scan_apply<T><<<(unsigned)nb, 256, 0, s>>>(in, out, n, sums, nullptr);
    return hipGetLastError();
}

// ------------------------------------------------------------------ radix sort (K10)
constexpr int RADIX_IT = 8;
constexpr int64_t RADIX_TILE = 256 * RADIX_IT;

// mask of lanes (among `active`) whose 8-bit digit equals the calling lane's
__device__ __forceinline__ uint64_t match_digit(uint32_t d, uint64_t active)
{
    uint64_t peers = active;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t m = __ballot(bit);
        peers &= bit ? m : ~m;
    }
    return peers;
}

template <typename K>
__global__ __launch_bounds__(256) void k_radix_hist(const K* keys, int64_t n, int shift, int32_t* counts, int nblocks)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RADIX_TILE;
    for (int it = 0; it < RADIX_IT; ++it) {
        const int64_t p = base + it * 256 + threadIdx.x;
        const bool valid = p < n;
        const uint32_t d = valid ? (uint32_t)(keys[p] >> shift) & 255u : 0u;
        const uint64_t act = __ballot(valid);
        const uint64_t peers = match_digit(d, act);
        if (valid && lane_rank(peers) == 0) atomicAdd(&h[d], (uint32_t)__popcll(peers));
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * nblocks + blockIdx.x] = (int32_t)h[threadIdx.x];
}

// Stable scatter of one tile by the current digit.  The tile is first ranked
// and reordered by digit in LDS (stable: tile order within a digit), then
// written out so that each digit's run of the tile lands contiguously at its
// global offset.  counts/offsets are digit-major: offsets[d * nblocks + b] is
// where tile b's elements with digit d start.
template <typename K>
__global__ __launch_bounds__(256) void k_radix_scatter(const K* keys, const int32_t* vals, K* keys_out, int32_t* vals_out,
                                                       int64_t n, int shift, const int32_t* offsets, int nblocks)
{
    __shared__ K s_key[RADIX_TILE];
    __shared__ int32_t s_val[RADIX_TILE];
    __shared__ uint32_t s_gbase[256];  // global start of each digit's run of this tile
    __shared__ uint32_t s_lbase[256];  // its start inside the tile
    __shared__ uint32_t s_run[256];    // elements of each digit placed so far
    __shared__ uint32_t s_wcnt[4][256];
    const int t = threadIdx.x, wid = t / WAVE;
    const int64_t base = (int64_t)blockIdx.x * RADIX_TILE;
    const int64_t total = (int64_t)256 * nblocks;
    const int64_t at = (int64_t)t * nblocks + blockIdx.x;
    const uint32_t g0 = (uint32_t)offsets[at];
    const uint32_t next = at + 1 < total ? (uint32_t)offsets[at + 1] : (uint32_t)n;
    s_gbase[t] = g0;
    s_lbase[t] = next - g0;  // this tile's count of digit t, scanned below
    s_run[t] = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) s_wcnt[w][t] = 0;
    __syncthreads();
    // exclusive scan of the 256 digit counts: inclusive scan within each
    // wavefront by shuffles, then the four wavefront totals
    {
        const uint32_t own = s_lbase[t];
        uint32_t v = own;
#pragma unroll
        for (int d = 1; d < WAVE; d <<= 1) {
            const uint32_t y = __shfl_up(v, d);
            if ((int)lane_id() >= d) v += y;
        }
        if ((int)lane_id() == WAVE - 1) s_wcnt[0][wid] = v;
        __syncthreads();
        uint32_t before = 0;
        for (int w = 0; w < wid; ++w) before += s_wcnt[0][w];
        __syncthreads();
        s_lbase[t] = before + v - own;
        s_wcnt[0][t] = 0;
    }
    __syncthreads();
    for (int it = 0; it < RADIX_IT; ++it) {
        const int64_t p = base + it * 256 + t;
        const bool valid = p < n;
        const K key = valid ? keys[p] : (K)0;
        const int32_t v = valid ? vals[p] : 0;
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        const uint64_t act = __ballot(valid);
        const uint64_t peers = match_digit(d, act);
        const uint32_t rank = lane_rank(peers);
        const uint32_t tag = (uint32_t)(it + 1) << 16;
        if (valid && rank == 0) s_wcnt[wid][d] = tag | (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t o = s_lbase[d] + s_run[d] + rank;
            for (int w = 0; w < wid; ++w) {
                const uint32_t x = s_wcnt[w][d];
                if ((x & 0xFFFF0000u) == tag) o += x & 0xFFFFu;
            }
            s_key[o] = key;
            s_val[o] = v;
        }
        uint32_t add = 0;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const uint32_t x = s_wcnt[w][t];
            if ((x & 0xFFFF0000u) == tag) add += x & 0xFFFFu;
        }
        __syncthreads();
        s_run[t] += add;
    }
    __syncthreads();
    const int64_t cnt = n - base < RADIX_TILE ? n - base : RADIX_TILE;
    for (int64_t q = t; q < cnt; q += 256) {
        const K key = s_key[q];
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        const uint32_t g = s_gbase[d] + ((uint32_t)q - s_lbase[d]);
        keys_out[g] = key;
        vals_out[g] = s_val[q];
    }
}

template <typename K>
hipError_t radix_sort_t(K* keys, int32_t* vals, K* keys_alt, int32_t* vals_alt, int64_t n, int bits, char* tmp,
                        size_t tmp_bytes, bool* in_alt, hipStream_t s)
{
    *in_alt = false;
    if (n <= 1 || bits <= 0) return hipSuccess;
    const int64_t nb = (n + RADIX_TILE - 1) / RADIX_TILE;
    const size_t cbytes = (((size_t)nb * 256 * sizeof(int32_t)) + 255) & ~(size_t)255;
    if (cbytes > tmp_bytes) return hipErrorInvalidValue;
    int32_t* counts = (int32_t*)tmp;
    K* src_k = keys; int32_t* src_v = vals;
    K* dst_k = keys_alt; int32_t* dst_v = vals_alt;
    for (int shift = 0; shift < bits; shift += 8) {
        k_radix_hist<K><<<(unsigned)nb, 256, 0, s>>>(src_k, n, shift, counts, (int)nb);
        hipError_t e = scan_exclusive_t<int32_t>(counts, counts, nb * 256, nullptr, tmp + cbytes, tmp_bytes - cbytes, s);
        if (e != hipSuccess) return e;
        k_radix_scatter<K><<<(unsigned)nb, 256, 0, s>>>(src_k, src_v, dst_k, dst_v, n, shift, counts, (int)nb);
        K* tk = src_k; src_k = dst_k; dst_k = tk;
        int32_t* tv = src_v; src_v = dst_v; dst_v = tv;
        *in_alt = !*in_alt;
    }
    return hipGetLastError();
}

__global__ void k_gather_i32(const int32_t* src, const int32_t* idx, int32_t m, int32_t* dst)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = src[idx[t]];
        dst[t] = v;
    }
}

}  // namespace

hipError_t launch_gather_i32(const int32_t* src, const int32_t* idx, int32_t m, int32_t* dst, hipStream_t s)
{
    if (m <= 0) return hipSuccess;
    k_gather_i32<<<LV_GRID(m)>>>(src, idx, m, dst);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_fill_i32<<<LV_GRID(n)>>>(p, v, n);
    return hipGetLastError();
}
hipError_t launch_iota(int32_t* p, int32_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_iota<<<LV_GRID(n)>>>(p, n);
    return hipGetLastError();
}
hipError_t launch_copy_i32(int32_t* d, const int32_t* src, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_copy_i32<<<LV_GRID(n)>>>(d, src, n);
    return hipGetLastError();
}

size_t scan_tmp_bytes(int64_t n, size_t elem)
{
    size_t b = 0;
    while (n > SCAN_TILE) {
        n = (n + SCAN_TILE - 1) / SCAN_TILE;
        b += ((size_t)n * elem + 255) & ~(size_t)255;
    }
    return b + 256;
}
hipError_t scan_exclusive_i32(const int32_t* in, int32_t* out, int64_t n, int32_t* total, void* tmp, size_t tb,
                              hipStream_t s)
{
    return scan_exclusive_t<int32_t>(in, out, n, total, (char*)tmp, tb, s);
}
hipError_t scan_exclusive_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* total, void* tmp, size_t tb,
                              hipStream_t s)
{
    return scan_exclusive_t<int64_t>(in, out, n, total, (char*)tmp, tb, s);
}

size_t radix_tmp_bytes(int64_t n)
{
    const int64_t nb = (n + RADIX_TILE - 1) / RADIX_TILE;
    const size_t c = (((size_t)(nb > 0 ? nb : 1) * 256 * sizeof(int32_t)) + 255) & ~(size_t)255;
    return c + scan_tmp_bytes(nb * 256, sizeof(int32_t));
}
hipError_t radix_sort_u64(uint64_t* keys, int32_t* vals, uint64_t* ka, int32_t* va, int64_t n, int bits, void* tmp,
                          size_t tb, bool* in_alt, hipStream_t s)
{
    return radix_sort_t<uint64_t>(keys, vals, ka, va, n, bits, (char*)tmp, tb, in_alt, s);
}
hipError_t radix_sort_u32(uint32_t* keys, int32_t* vals, uint32_t* ka, int32_t* va, int64_t n, int bits, void* tmp,
                          size_t tb, bool* in_alt, hipStream_t s)
{
    return radix_sort_t<uint32_t>(keys, vals, ka, va, n, bits, (char*)tmp, tb, in_alt, s);
}

}  // namespace lv
