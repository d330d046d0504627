// HIP kernels (gfx950, wave64) of the Louvain local-moving library.
//
// Paper: Li, Du, Bader, arXiv 2507.06471.  Algorithm 2 (local moving) is the
// hot path: for every vertex, sum its edge weights per neighbouring community
// (cut_w(v, C) of Equation 1), pick the best community and record a move.
// Commits update community volumes with integer atomics.  Aggregation
// (Algorithm 3) renumbers communities and rebuilds the CSR by sort + segmented
// reduce.  All decisions are integer: score = M*W - k_i*Sigma_tot with every
// factor < 2^31, exact in int64.
#include "lv_internal.h"

#include <limits.h>

namespace lv {

namespace {

constexpr int WAVE = 64;

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// number of set bits of `mask` below the calling lane
__device__ __forceinline__ uint32_t lane_rank(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint32_t mix32(int32_t key)
{
    uint32_t h = (uint32_t)key * 0x9E3779B1u;
    return h ^ (h >> 15);
}

// (s1, c1) ranks before (s2, c2): larger score, then smaller community id.
__device__ __forceinline__ bool better(int64_t s1, int32_t c1, int64_t s2, int32_t c2)
{
    return s1 > s2 || (s1 == s2 && c1 < c2);
}

// Wave-aggregated append: one atomic per wavefront.  Must be reached by all
// lanes of the wave.  Returns the slot for lanes with pred, else -1.
__device__ __forceinline__ int32_t wave_append(bool pred, uint32_t* counter)
{
    uint64_t m = __ballot(pred);
    if (m == 0) return -1;
    uint32_t leader = (uint32_t)__ffsll((unsigned long long)m) - 1u;
    uint32_t base = 0;
    if (lane_id() == leader) base = atomicAdd(counter, (uint32_t)__popcll(m));
    base = __shfl(base, (int)leader);
    return pred ? (int32_t)(base + lane_rank(m)) : -1;
}

// Reduce (score, community, own-weight) over aligned groups of G lanes (G <= 64).
template <int G>
__device__ __forceinline__ void group_reduce(int64_t& s, int32_t& c, int32_t& wo)
{
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1) {
        long long s2 = __shfl_xor((long long)s, m, G);
        int32_t c2 = __shfl_xor(c, m, G);
        int32_t w2 = __shfl_xor(wo, m, G);
        if (better(s2, c2, s, c)) { s = s2; c = c2; }
        wo = max(wo, w2);
    }
}

// Block-wide reduce of (score, community, own-weight); result valid in thread 0.
template <int BS>
__device__ __forceinline__ void block_reduce_best(int64_t& s, int32_t& c, int32_t& wo, int64_t* rs, int32_t* rc,
                                                  int32_t* rw)
{
    group_reduce<WAVE>(s, c, wo);
    constexpr int NW = BS / WAVE;
    if constexpr (NW > 1) {
        const int wid = threadIdx.x / WAVE;
        if (lane_id() == 0) { rs[wid] = s; rc[wid] = c; rw[wid] = wo; }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 1; w < NW; ++w) {
                if (better(rs[w], rc[w], s, c)) { s = rs[w]; c = rc[w]; }
                wo = max(wo, rw[w]);
            }
        }
    }
}

template <typename T>
__device__ __forceinline__ T block_sum256(T v, T* red)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    if (lane_id() == 0) red[threadIdx.x / WAVE] = v;
    __syncthreads();
    T t = 0;
    if (threadIdx.x == 0) t = red[0] + red[1] + red[2] + red[3];
    __syncthreads();
    return t;
}

// first index x in [lo, hi) with a[x] > v (a non-decreasing); hi if none
__device__ __forceinline__ int64_t upper_bound_i32(const int32_t* a, int64_t lo, int64_t hi, int64_t v)
{
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if ((int64_t)a[mid] <= v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Visit the CSR entries of this block's tile with their row index.  Thread t
// handles entries e0 + t*IT + j (j < IT).  The row offsets spanned by the tile
// are staged in LDS when they fit, else rows are found in global memory.
template <int BS, int IT, typename F>
__device__ __forceinline__ void for_tile_entries(const int32_t* off, int32_t n, int64_t nnz, F&& f)
{
    constexpr int CAP = BS * IT + 1;
    __shared__ int32_t s_off[CAP];
    __shared__ int64_t s_r0, s_cnt;
    const int64_t e0 = (int64_t)blockIdx.x * BS * IT;
    const int64_t e1 = min(e0 + (int64_t)BS * IT, nnz);
    if (threadIdx.x == 0) {
        int64_t r0 = upper_bound_i32(off, 0, (int64_t)n + 1, e0) - 1;
        int64_t r1 = upper_bound_i32(off, 0, (int64_t)n + 1, e1 - 1) - 1;
        s_r0 = r0;
        s_cnt = r1 - r0 + 2;
    }
    __syncthreads();
    const int64_t r0 = s_r0, cnt = s_cnt;
    const bool staged = cnt <= CAP;
    if (staged)
        for (int64_t t = threadIdx.x; t < cnt; t += BS) s_off[t] = off[r0 + t];
    __syncthreads();
    const int64_t my0 = e0 + (int64_t)threadIdx.x * IT;
    if (my0 >= e1) return;
    int64_t r;
    if (staged) {
        int64_t lo = 0, hi = cnt;
        while (lo < hi) {
            int64_t mid = (lo + hi) / 2;
            if ((int64_t)s_off[mid] <= my0) lo = mid + 1; else hi = mid;
        }
        r = r0 + lo - 1;
    } else {
        r = upper_bound_i32(off, r0, r0 + cnt, my0) - 1;
    }
    for (int j = 0; j < IT; ++j) {
        const int64_t e = my0 + j;
        if (e >= e1) break;
        while ((int64_t)(staged ? s_off[r + 1 - r0] : off[r + 1]) <= e) ++r;
        f((int32_t)r, e);
    }
}

constexpr int TILE_BS = 256;
constexpr int TILE_IT = 8;
constexpr int64_t TILE = TILE_BS * TILE_IT;

inline int grid_for(int64_t n, int64_t per_block, int64_t cap = 1 << 20)
{
    int64_t b = (n + per_block - 1) / per_block;
    if (b < 1) b = 1;
    return (int)(b < cap ? b : cap);
}

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
    T t = block_sum256(s, red);
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
constexpr int RADIX_IT = 16;
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

template <typename K>
__global__ __launch_bounds__(256) void k_radix_scatter(const K* keys, const int32_t* vals, K* keys_out, int32_t* vals_out,
                                                       int64_t n, int shift, const int32_t* offsets, int nblocks)
{
    __shared__ uint32_t s_base[256];
    __shared__ uint32_t s_wcnt[4][256];
    const int t = threadIdx.x, wid = t / WAVE;
    s_base[t] = (uint32_t)offsets[(int64_t)t * nblocks + blockIdx.x];
#pragma unroll
    for (int w = 0; w < 4; ++w) s_wcnt[w][t] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RADIX_TILE;
    for (int it = 0; it < RADIX_IT; ++it) {
        const int64_t p = base + it * 256 + t;
        const bool valid = p < n;
        K key = valid ? keys[p] : (K)0;
        int32_t v = valid ? vals[p] : 0;
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        const uint64_t act = __ballot(valid);
        const uint64_t peers = match_digit(d, act);
        const uint32_t rank = lane_rank(peers);
        const uint32_t tag = (uint32_t)(it + 1) << 16;
        if (valid && rank == 0) s_wcnt[wid][d] = tag | (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t o = s_base[d] + rank;
            for (int w = 0; w < wid; ++w) {
                const uint32_t x = s_wcnt[w][d];
                if ((x & 0xFFFF0000u) == tag) o += x & 0xFFFFu;
            }
            keys_out[o] = key;
            vals_out[o] = v;
        }
        uint32_t add = 0;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const uint32_t x = s_wcnt[w][t];
            if ((x & 0xFFFF0000u) == tag) add += x & 0xFFFFu;
        }
        __syncthreads();
        s_base[t] += add;
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

// ------------------------------------------------------------------ graph preparation
// err bits: 1 = offsets, 2 = index range / order, 4 = weight, 8 = asymmetric, 16 = overflow
__global__ void k_check_offsets(int32_t n, const int32_t* off, int64_t nnz, int32_t* err)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += (int64_t)gridDim.x * blockDim.x) {
        bool bad = false;
        if (i == 0) bad = off[0] != 0;
        if (i == n) bad = bad || (int64_t)off[n] != nnz;
        if (i < n) bad = bad || off[i] > off[i + 1];
        if (bad) atomicOr(err, 1);
    }
}

__global__ __launch_bounds__(TILE_BS) void k_check_entries(int32_t n, const int32_t* off, const int32_t* idx,
                                                            const int32_t* w, int64_t nnz, int32_t* err)
{
    for_tile_entries<TILE_BS, TILE_IT>(off, n, nnz, [&](int32_t r, int64_t e) {
        const int32_t j = idx[e];
        if (j < 0 || j >= n) atomicOr(err, 2);
        else if (e > off[r] && idx[e - 1] >= j) atomicOr(err, 2);
        if (w && w[e] < 1) atomicOr(err, 4);
    });
}

__global__ __launch_bounds__(TILE_BS) void k_check_symmetric(int32_t n, const int32_t* off, const int32_t* idx,
                                                              const int32_t* w, int64_t nnz, int32_t* err)
{
    for_tile_entries<TILE_BS, TILE_IT>(off, n, nnz, [&](int32_t r, int64_t e) {
        const int32_t j = idx[e];
        if (j == r) return;
        int64_t lo = off[j], hi = off[j + 1];
        while (lo < hi) {
            int64_t mid = (lo + hi) / 2;
            if (idx[mid] < r) lo = mid + 1; else hi = mid;
        }
        if (lo >= off[j + 1] || idx[lo] != r || (w && w[lo] != w[e])) atomicOr(err, 8);
    });
}

// diag_pos[i] = entry of the loop (i, i) or -1
__global__ void k_diag_scan(int32_t n, const int32_t* off, const int32_t* idx, int32_t* diag_pos, int32_t* any)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = off[i], hi = off[i + 1];
        while (lo < hi) {
            int64_t mid = (lo + hi) / 2;
            if (idx[mid] < i) lo = mid + 1; else hi = mid;
        }
        const bool has = lo < off[i + 1] && idx[lo] == i;
        diag_pos[i] = has ? (int32_t)lo : -1;
        if (has) atomicOr(any, 1);
    }
}

// A = caller weights (or 1) with each loop entry doubled (weighted degree counts loops twice)
__global__ void k_adjacency_copy(const int32_t* w_in, int64_t nnz, int32_t* w_out)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x)
        w_out[e] = w_in ? w_in[e] : 1;
}
__global__ void k_adjacency_double(int32_t n, const int32_t* diag_pos, int32_t* w_out, int32_t* err)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t p = diag_pos[i];
        if (p < 0) continue;
        const int64_t v = 2 * (int64_t)w_out[p];
        if (v > INT32_MAX) atomicOr(err, 16);
        else w_out[p] = (int32_t)v;
    }
}

// k64[r] = sum of row r; total (int64) via block partials
__global__ __launch_bounds__(TILE_BS) void k_row_sums(int32_t n, const int32_t* off, const int32_t* w, int64_t nnz,
                                                       unsigned long long* k64)
{
    int32_t cur = -1;
    int64_t acc = 0;
    for_tile_entries<TILE_BS, TILE_IT>(off, n, nnz, [&](int32_t r, int64_t e) {
        if (r != cur) {
            if (cur >= 0) atomicAdd(&k64[cur], (unsigned long long)acc);
            cur = r;
            acc = 0;
        }
        acc += w[e];
    });
    if (cur >= 0) atomicAdd(&k64[cur], (unsigned long long)acc);
}

__global__ __launch_bounds__(256) void k_narrow_sum(int32_t n, const unsigned long long* k64, int32_t* k,
                                                     unsigned long long* total)
{
    __shared__ unsigned long long red[4];
    unsigned long long s = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const unsigned long long v = k64[i];
        k[i] = v > (unsigned long long)INT32_MAX ? INT32_MAX : (int32_t)v;
        s += v;
    }
    s = block_sum256(s, red);
    if (threadIdx.x == 0) atomicAdd(total, s);
}

__global__ void k_degree_unit(int32_t n, const int32_t* off, int32_t* k)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        k[i] = off[i + 1] - off[i];
}

// out[0] += sum k^2, out[1] += trace (sum of diagonal entries)
__global__ __launch_bounds__(256) void k_sum_sq(int32_t n, const int32_t* k, unsigned long long* out)
{
    __shared__ unsigned long long red[4];
    unsigned long long s = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        s += (unsigned long long)((int64_t)k[i] * (int64_t)k[i]);
    s = block_sum256(s, red);
    if (threadIdx.x == 0) atomicAdd(&out[0], s);
}
__global__ __launch_bounds__(TILE_BS) void k_trace(int32_t n, const int32_t* off, const int32_t* idx, const int32_t* w,
                                                    int64_t nnz, unsigned long long* out)
{
    __shared__ unsigned long long red[4];
    unsigned long long s = 0;
    for_tile_entries<TILE_BS, TILE_IT>(off, n, nnz, [&](int32_t r, int64_t e) {
        if (idx[e] == r) s += (unsigned long long)(w ? w[e] : 1);
    });
    s = block_sum256(s, red);
    if (threadIdx.x == 0 && s) atomicAdd(&out[1], s);
}

// ------------------------------------------------------------------ degree classes
struct Bounds { int32_t b[NUM_CLS]; };
__global__ void k_classify(int32_t n, const int32_t* off, Bounds bd, uint32_t* cls, int32_t* vert)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t L = off[i + 1] - off[i];
        uint32_t c = CLS_NONE;
        if (L > 0) {
            c = CLS_HUB;
            for (int q = CLS_G8; q < CLS_HUB; ++q)
                if (L <= bd.b[q]) { c = (uint32_t)q; break; }
        }
        cls[i] = c;
        vert[i] = (int32_t)i;
    }
}

// ------------------------------------------------------------------ move step (K4-K6)
// One group of G lanes decides one vertex: aggregate W_i(C) over neighbours
// j != i in an LDS open-addressing table (or, in the singleton state where
// every community is a single vertex and CSR columns are unique, score each
// entry directly), then take the best community and record a move if it beats
// staying and lies in the sweep's direction.
template <int BS, int G, int SLOTS, bool SINGLETON>
__global__ __launch_bounds__(BS) void k_move(MoveArgs a)
{
    constexpr int NG = BS / G;
    constexpr int TBL = SINGLETON ? 1 : NG * SLOTS;
    __shared__ int32_t s_key[TBL];
    __shared__ int32_t s_val[TBL];
    __shared__ int64_t rs[BS / WAVE];
    __shared__ int32_t rc[BS / WAVE], rw[BS / WAVE];

    const int g = threadIdx.x / G, lane = threadIdx.x % G;
    const int64_t vi = (int64_t)blockIdx.x * NG + g;
    const bool has = vi < a.nverts;
    const int32_t i = has ? a.verts[vi] : 0;
    const int32_t beg = has ? a.off[i] : 0, end = has ? a.off[i + 1] : 0;
    const int32_t A = has ? a.comm[i] : 0;
    const int64_t ki = has ? a.k[i] : 0;
    const bool louvain = a.mode == MODE_LOUVAIN;
    int64_t best_s = INT64_MIN;
    int32_t best_c = INT32_MAX, w_own = 0;

    if constexpr (SINGLETON) {
        for (int32_t e = beg + lane; e < end; e += G) {
            const int32_t j = a.idx[e];
            if (j == i) continue;
            const int32_t W = a.w ? a.w[e] : 1;
            const int64_t s = louvain ? a.M * W - ki * (int64_t)a.sigma[j] : (int64_t)W;
            if (better(s, j, best_s, best_c)) { best_s = s; best_c = j; }
        }
    } else {
        int32_t* key = s_key + g * SLOTS;
        int32_t* val = s_val + g * SLOTS;
        for (int t = lane; t < SLOTS; t += G) { key[t] = EMPTY_KEY; val[t] = 0; }
        __syncthreads();
        for (int32_t e = beg + lane; e < end; e += G) {
            const int32_t j = a.idx[e];
            if (j == i) continue;
            const int32_t C = a.comm[j];
            const int32_t W = a.w ? a.w[e] : 1;
            uint32_t h = mix32(C) & (SLOTS - 1);
            for (;;) {
                const int32_t prev = atomicCAS(&key[h], EMPTY_KEY, C);
                if (prev == EMPTY_KEY || prev == C) { atomicAdd(&val[h], W); break; }
                h = (h + 1) & (SLOTS - 1);
            }
        }
        __syncthreads();
        for (int t = lane; t < SLOTS; t += G) {
            const int32_t C = key[t];
            if (C == EMPTY_KEY) continue;
            const int32_t W = val[t];
            if (C == A) { w_own = W; continue; }
            const int64_t s = louvain ? a.M * W - ki * (int64_t)a.sigma[C] : (int64_t)W;
            if (better(s, C, best_s, best_c)) { best_s = s; best_c = C; }
        }
    }

    if constexpr (G <= WAVE) {
        group_reduce<G>(best_s, best_c, w_own);
    } else {
        group_reduce<WAVE>(best_s, best_c, w_own);
        const int wid = threadIdx.x / WAVE;
        if (lane_id() == 0) { rs[wid] = best_s; rc[wid] = best_c; rw[wid] = w_own; }
        __syncthreads();
        if (lane == 0) {
            constexpr int WPG = G / WAVE;
            for (int w = 1; w < WPG; ++w) {
                const int src = g * WPG + w;
                if (better(rs[src], rc[src], best_s, best_c)) { best_s = rs[src]; best_c = rc[src]; }
                w_own = max(w_own, rw[src]);
            }
        }
    }

    bool mover = false;
    if (has && lane == 0 && best_c != INT32_MAX) {
        const int64_t stay = louvain ? a.M * w_own - ki * ((int64_t)a.sigma[A] - ki) : (int64_t)w_own;
        const bool dir_ok = a.dir == DIR_DOWN ? best_c < A : best_c > A;
        mover = best_s > stay && dir_ok;
    }
    const int32_t slot = wave_append(mover, a.mv_count);
    if (mover) { a.mv_vert[slot] = i; a.mv_comm[slot] = best_c; }
}

template <int BS, int G, int SLOTS>
hipError_t launch_move_t(bool singleton, const MoveArgs& a, hipStream_t s)
{
    if (a.nverts <= 0) return hipSuccess;
    constexpr int NG = BS / G;
    const unsigned grid = (unsigned)((a.nverts + NG - 1) / NG);
    if (singleton) k_move<BS, G, SLOTS, true><<<grid, BS, 0, s>>>(a);
    else k_move<BS, G, SLOTS, false><<<grid, BS, 0, s>>>(a);
    return hipGetLastError();
}

// ------------------------------------------------------------------ hub path (global table)
constexpr int HUB_BS = 256;

// Singleton sweep: per-chunk best over entries.  Later sweeps: insert the
// chunk's entries into the hub's global open-addressing table.
template <bool SINGLETON>
__global__ __launch_bounds__(HUB_BS) void k_hub_insert(MoveArgs a, HubArgs h)
{
    __shared__ int64_t rs[HUB_BS / WAVE];
    __shared__ int32_t rc[HUB_BS / WAVE], rw[HUB_BS / WAVE];
    const int b = blockIdx.x;
    const int32_t hh = h.ins_hub[b];
    const int32_t i = h.hub_vert[hh];
    const int32_t beg = h.ins_beg[b], end = h.ins_end[b];
    if constexpr (SINGLETON) {
        const int64_t ki = a.k[i];
        const bool louvain = a.mode == MODE_LOUVAIN;
        int64_t best_s = INT64_MIN;
        int32_t best_c = INT32_MAX, w_own = 0;
        for (int32_t e = beg + threadIdx.x; e < end; e += HUB_BS) {
            const int32_t j = a.idx[e];
            if (j == i) continue;
            const int32_t W = a.w ? a.w[e] : 1;
            const int64_t s = louvain ? a.M * W - ki * (int64_t)a.sigma[j] : (int64_t)W;
            if (better(s, j, best_s, best_c)) { best_s = s; best_c = j; }
        }
        block_reduce_best<HUB_BS>(best_s, best_c, w_own, rs, rc, rw);
        if (threadIdx.x == 0) { h.part_score[b] = best_s; h.part_comm[b] = best_c; h.part_wown[b] = 0; }
    } else {
        const uint32_t mask = (uint32_t)h.tab_cap[hh] - 1u;
        int32_t* tab = h.table + 2 * h.tab_off[hh];
        for (int32_t e = beg + threadIdx.x; e < end; e += HUB_BS) {
            const int32_t j = a.idx[e];
            if (j == i) continue;
            const int32_t C = a.comm[j];
            const int32_t W = a.w ? a.w[e] : 1;
            uint32_t slot = mix32(C) & mask;
            for (;;) {
                const int32_t prev = atomicCAS(&tab[2 * slot], EMPTY_KEY, C);
                if (prev == EMPTY_KEY || prev == C) { atomicAdd(&tab[2 * slot + 1], W); break; }
                slot = (slot + 1) & mask;
            }
        }
    }
}

// Scan a slot range of a hub table: partial best, own-community weight, and
// reset of the slots for the next sweep.
__global__ __launch_bounds__(HUB_BS) void k_hub_scan(MoveArgs a, HubArgs h)
{
    __shared__ int64_t rs[HUB_BS / WAVE];
    __shared__ int32_t rc[HUB_BS / WAVE], rw[HUB_BS / WAVE];
    const int b = blockIdx.x;
    const int32_t hh = h.scan_hub[b];
    const int32_t i = h.hub_vert[hh];
    const int32_t A = a.comm[i];
    const int64_t ki = a.k[i];
    const bool louvain = a.mode == MODE_LOUVAIN;
    int32_t* tab = h.table + 2 * h.tab_off[hh];
    int64_t best_s = INT64_MIN;
    int32_t best_c = INT32_MAX, w_own = 0;
    for (int32_t t = h.scan_beg[b] + threadIdx.x; t < h.scan_end[b]; t += HUB_BS) {
        const int32_t C = tab[2 * t];
        if (C == EMPTY_KEY) continue;
        const int32_t W = tab[2 * t + 1];
        tab[2 * t] = EMPTY_KEY;
        tab[2 * t + 1] = 0;
        if (C == A) { w_own = W; continue; }
        const int64_t s = louvain ? a.M * W - ki * (int64_t)a.sigma[C] : (int64_t)W;
        if (better(s, C, best_s, best_c)) { best_s = s; best_c = C; }
    }
    block_reduce_best<HUB_BS>(best_s, best_c, w_own, rs, rc, rw);
    if (threadIdx.x == 0) { h.part_score[b] = best_s; h.part_comm[b] = best_c; h.part_wown[b] = w_own; }
}

// One wavefront per hub: combine partials, decide, append the move.
__global__ __launch_bounds__(256) void k_hub_finalize(MoveArgs a, HubArgs h, int singleton)
{
    const int64_t hh64 = (int64_t)blockIdx.x * (256 / WAVE) + threadIdx.x / WAVE;
    const bool has = hh64 < h.nhubs;
    const int32_t hh = has ? (int32_t)hh64 : 0;
    const int32_t* first = singleton ? h.part_first_ins : h.part_first_scan;
    int64_t best_s = INT64_MIN;
    int32_t best_c = INT32_MAX, w_own = 0;
    int32_t i = 0, A = 0;
    int64_t ki = 0;
    if (has) {
        i = h.hub_vert[hh];
        A = a.comm[i];
        ki = a.k[i];
        for (int32_t p = first[hh] + (int32_t)lane_id(); p < first[hh + 1]; p += WAVE) {
            if (better(h.part_score[p], h.part_comm[p], best_s, best_c)) { best_s = h.part_score[p]; best_c = h.part_comm[p]; }
            w_own = max(w_own, h.part_wown[p]);
        }
    }
    group_reduce<WAVE>(best_s, best_c, w_own);
    bool mover = false;
    if (has && lane_id() == 0 && best_c != INT32_MAX) {
        const bool louvain = a.mode == MODE_LOUVAIN;
        const int64_t stay = louvain ? a.M * w_own - ki * ((int64_t)a.sigma[A] - ki) : (int64_t)w_own;
        const bool dir_ok = a.dir == DIR_DOWN ? best_c < A : best_c > A;
        mover = best_s > stay && dir_ok;
    }
    const int32_t slot = wave_append(mover, a.mv_count);
    if (mover) { a.mv_vert[slot] = i; a.mv_comm[slot] = best_c; }
}

// ------------------------------------------------------------------ commit (K7)
__global__ __launch_bounds__(256) void k_apply(const int32_t* mv_vert, const int32_t* mv_comm, const uint32_t* mv_count,
                                               const int32_t* k, int32_t* comm, int32_t* sigma)
{
    const uint32_t cnt = *mv_count;
    for (uint32_t t = blockIdx.x * 256 + threadIdx.x; t < cnt; t += gridDim.x * 256) {
        const int32_t v = mv_vert[t], C = mv_comm[t];
        const int32_t A = comm[v], kv = k[v];
        atomicSub(&sigma[A], kv);
        atomicAdd(&sigma[C], kv);
        comm[v] = C;
    }
}

// ------------------------------------------------------------------ renumber (K9) and aggregation (K10/K11)
__global__ void k_minv(int32_t n, const int32_t* comm, int32_t* minv)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        atomicMin(&minv[comm[i]], (int32_t)i);
}
__global__ void k_first_flag(int32_t n, const int32_t* comm, const int32_t* minv, int32_t* flag)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        flag[i] = minv[comm[i]] == (int32_t)i ? 1 : 0;
}
__global__ void k_label(int32_t n, const int32_t* comm, const int32_t* minv, const int32_t* pos, int32_t* labels)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        labels[i] = pos[minv[comm[i]]];
}
__global__ void k_coarse_degree(int32_t n, const int32_t* comm, const int32_t* flag, const int32_t* labels,
                                const int32_t* sigma, int32_t* k2)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (flag[i]) k2[labels[i]] = sigma[comm[i]];
}

__global__ __launch_bounds__(TILE_BS) void k_build_keys(int32_t n, const int32_t* off, const int32_t* idx,
                                                         const int32_t* w, int64_t nnz, const int32_t* labels,
                                                         int colbits, uint64_t* keys, int32_t* vals)
{
    for_tile_entries<TILE_BS, TILE_IT>(off, n, nnz, [&](int32_t r, int64_t e) {
        keys[e] = ((uint64_t)(uint32_t)labels[r] << colbits) | (uint64_t)(uint32_t)labels[idx[e]];
        vals[e] = w ? w[e] : 1;
    });
}

__global__ void k_segment_heads(const uint64_t* keys, int64_t n, int32_t* head)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        head[e] = (e == 0 || keys[e] != keys[e - 1]) ? 1 : 0;
}

__global__ void k_segment_reduce(const uint64_t* keys, const int32_t* vals, const int32_t* pos, int64_t n, int colbits,
                                 int32_t* idx2, int32_t* w2, int32_t* rowcnt)
{
    const uint64_t cmask = (colbits >= 64) ? ~0ull : ((1ull << colbits) - 1ull);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t key = keys[e];
        const bool head = e == 0 || key != keys[e - 1];
        const int32_t o = pos[e] + (head ? 1 : 0) - 1;
        atomicAdd(&w2[o], vals[e]);
        if (head) {
            idx2[o] = (int32_t)(key & cmask);
            atomicAdd(&rowcnt[(int32_t)(key >> colbits)], 1);
        }
    }
}

__global__ void k_compose(int32_t n0, int32_t* fin, const int32_t* labels)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n0; v += (int64_t)gridDim.x * blockDim.x)
        fin[v] = labels[fin[v]];
}

// modularity parts of arbitrary labels: tot[c] += k_i; out[0] += Sigma_in
__global__ void k_label_volumes(int32_t n, const int32_t* k, const int32_t* labels, unsigned long long* tot)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&tot[labels[i]], (unsigned long long)k[i]);
}
__global__ __launch_bounds__(TILE_BS) void k_sigma_in(int32_t n, const int32_t* off, const int32_t* idx, const int32_t* w,
                                                       int64_t nnz, const int32_t* labels, unsigned long long* out)
{
    __shared__ unsigned long long red[4];
    unsigned long long s = 0;
    for_tile_entries<TILE_BS, TILE_IT>(off, n, nnz, [&](int32_t r, int64_t e) {
        if (labels[idx[e]] == labels[r]) s += (unsigned long long)(w ? w[e] : 1);
    });
    s = block_sum256(s, red);
    if (threadIdx.x == 0 && s) atomicAdd(&out[0], s);
}
__global__ __launch_bounds__(256) void k_sum_sq_i64(const unsigned long long* v, int64_t n, unsigned long long* out)
{
    __shared__ unsigned long long red[4];
    unsigned long long s = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        s += v[i] * v[i];
    s = block_sum256(s, red);
    if (threadIdx.x == 0) atomicAdd(out, s);
}
__global__ void k_check_labels(const int32_t* labels, int32_t n, int32_t* err)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (labels[i] < 0 || labels[i] >= n) atomicOr(err, 1);
}

__global__ void k_class_starts(const uint32_t* cls, int32_t n, int32_t* start)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        if (t == 0 || cls[t] != cls[t - 1]) start[cls[t]] = (int32_t)t;
}
__global__ void k_gather_rows(const int32_t* verts, int32_t m, const int32_t* off, int32_t* beg, int32_t* len)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = verts[t];
        beg[t] = off[v];
        len[t] = off[v + 1] - off[v];
    }
}

}  // namespace

// ====================================================================== launchers
#define LV_GRID(n) grid_for((n), 256, 65536), 256, 0, s

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

hipError_t launch_check_offsets(int32_t n, const int32_t* off, int64_t nnz, int32_t* err, hipStream_t s)
{
    k_check_offsets<<<LV_GRID((int64_t)n + 1)>>>(n, off, nnz, err);
    return hipGetLastError();
}
hipError_t launch_check_entries(int32_t n, const int32_t* off, const int32_t* idx, const int32_t* w, int64_t nnz,
                                int32_t* err, hipStream_t s)
{
    if (nnz <= 0) return hipSuccess;
    k_check_entries<<<(unsigned)((nnz + TILE - 1) / TILE), TILE_BS, 0, s>>>(n, off, idx, w, nnz, err);
    return hipGetLastError();
}
hipError_t launch_check_symmetric(int32_t n, const int32_t* off, const int32_t* idx, const int32_t* w, int64_t nnz,
                                  int32_t* err, hipStream_t s)
{
    if (nnz <= 0) return hipSuccess;
    k_check_symmetric<<<(unsigned)((nnz + TILE - 1) / TILE), TILE_BS, 0, s>>>(n, off, idx, w, nnz, err);
    return hipGetLastError();
}
hipError_t launch_diag_scan(int32_t n, const int32_t* off, const int32_t* idx, int32_t* diag_pos, int32_t* any,
                            hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_diag_scan<<<LV_GRID(n)>>>(n, off, idx, diag_pos, any);
    return hipGetLastError();
}
hipError_t launch_adjacency_weights(int32_t n, const int32_t* w_in, const int32_t* diag_pos, int64_t nnz,
                                    int32_t* w_out, int32_t* err, hipStream_t s)
{
    if (nnz > 0) k_adjacency_copy<<<LV_GRID(nnz)>>>(w_in, nnz, w_out);
    if (n > 0) k_adjacency_double<<<LV_GRID(n)>>>(n, diag_pos, w_out, err);
    return hipGetLastError();
}
hipError_t launch_row_sums(int32_t n, const int32_t* off, const int32_t* w, int64_t nnz, int32_t* k, int64_t* k64,
                           int64_t* total, hipStream_t s)
{
    hipError_t e = hipMemsetAsync(k64, 0, sizeof(int64_t) * (size_t)(n > 0 ? n : 1), s);
    if (e != hipSuccess) return e;
    if (nnz > 0)
        k_row_sums<<<(unsigned)((nnz + TILE - 1) / TILE), TILE_BS, 0, s>>>(n, off, w, nnz, (unsigned long long*)k64);
    if (n > 0)
        k_narrow_sum<<<grid_for(n, 256, 4096), 256, 0, s>>>(n, (const unsigned long long*)k64, k,
                                                            (unsigned long long*)total);
    return hipGetLastError();
}
hipError_t launch_degree_unit(int32_t n, const int32_t* off, int32_t* k, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_degree_unit<<<LV_GRID(n)>>>(n, off, k);
    return hipGetLastError();
}
hipError_t launch_sum_sq_trace(int32_t n, const int32_t* off, const int32_t* idx, const int32_t* w, int64_t nnz,
                               const int32_t* k, int64_t* out2, hipStream_t s)
{
    if (n > 0) k_sum_sq<<<grid_for(n, 256, 4096), 256, 0, s>>>(n, k, (unsigned long long*)out2);
    if (nnz > 0)
        k_trace<<<(unsigned)((nnz + TILE - 1) / TILE), TILE_BS, 0, s>>>(n, off, idx, w, nnz,
                                                                         (unsigned long long*)out2);
    return hipGetLastError();
}

hipError_t launch_classify(int32_t n, const int32_t* off, const int32_t* bounds, uint32_t* cls, int32_t* vert,
                           hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    Bounds bd;
    for (int q = 0; q < NUM_CLS; ++q) bd.b[q] = bounds[q];
    k_classify<<<LV_GRID(n)>>>(n, off, bd, cls, vert);
    return hipGetLastError();
}

hipError_t launch_move_class(int cls, bool singleton, const MoveArgs& a, hipStream_t s)
{
    switch (cls) {
    case CLS_G8: return launch_move_t<256, 8, 16>(singleton, a, s);
    case CLS_G32: return launch_move_t<256, 32, 64>(singleton, a, s);
    case CLS_G64: return launch_move_t<256, 64, 256>(singleton, a, s);
    case CLS_B256: return launch_move_t<256, 256, 1024>(singleton, a, s);
    case CLS_B512: return launch_move_t<512, 512, 8192>(singleton, a, s);
    default: return hipErrorInvalidValue;
    }
}

__global__ void k_hub_fill_keys(int32_t* table, int64_t slots)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < slots; t += (int64_t)gridDim.x * blockDim.x) {
        table[2 * t] = EMPTY_KEY;
        table[2 * t + 1] = 0;
    }
}
hipError_t launch_hub_clear(int32_t* table, int64_t slots, hipStream_t s)
{
    if (slots <= 0) return hipSuccess;
    k_hub_fill_keys<<<LV_GRID(slots)>>>(table, slots);
    return hipGetLastError();
}

hipError_t launch_hub_sweep(bool singleton, const MoveArgs& a, const HubArgs& h, hipStream_t s)
{
    if (h.nhubs <= 0) return hipSuccess;
    if (singleton) {
        k_hub_insert<true><<<(unsigned)h.nins, HUB_BS, 0, s>>>(a, h);
    } else {
        k_hub_insert<false><<<(unsigned)h.nins, HUB_BS, 0, s>>>(a, h);
        k_hub_scan<<<(unsigned)h.nscan, HUB_BS, 0, s>>>(a, h);
    }
    k_hub_finalize<<<(unsigned)((h.nhubs + 3) / 4), 256, 0, s>>>(a, h, singleton ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_apply(const int32_t* mv_vert, const int32_t* mv_comm, const uint32_t* mv_count, int32_t max_movers,
                        const int32_t* k, int32_t* comm, int32_t* sigma, hipStream_t s)
{
    if (max_movers <= 0) return hipSuccess;
    k_apply<<<grid_for(max_movers, 256, 8192), 256, 0, s>>>(mv_vert, mv_comm, mv_count, k, comm, sigma);
    return hipGetLastError();
}

hipError_t launch_renumber(int32_t n, const int32_t* comm, int32_t* minv, int32_t* flag, int32_t* pos, int32_t* labels,
                           int32_t* n_out, void* tmp, size_t tb, hipStream_t s)
{
    if (n <= 0) return hipMemsetAsync(n_out, 0, sizeof(int32_t), s);
    k_fill_i32<<<LV_GRID(n)>>>(minv, INT32_MAX, n);
    k_minv<<<LV_GRID(n)>>>(n, comm, minv);
    k_first_flag<<<LV_GRID(n)>>>(n, comm, minv, flag);
    hipError_t e = scan_exclusive_i32(flag, pos, n, n_out, tmp, tb, s);
    if (e != hipSuccess) return e;
    k_label<<<LV_GRID(n)>>>(n, comm, minv, pos, labels);
    return hipGetLastError();
}
hipError_t launch_coarse_degree(int32_t n, const int32_t* comm, const int32_t* flag, const int32_t* labels,
                                const int32_t* sigma, int32_t* k2, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_coarse_degree<<<LV_GRID(n)>>>(n, comm, flag, labels, sigma, k2);
    return hipGetLastError();
}
hipError_t launch_build_keys(int32_t n, const int32_t* off, const int32_t* idx, const int32_t* w, int64_t nnz,
                             const int32_t* labels, int colbits, uint64_t* keys, int32_t* vals, hipStream_t s)
{
    if (nnz <= 0) return hipSuccess;
    k_build_keys<<<(unsigned)((nnz + TILE - 1) / TILE), TILE_BS, 0, s>>>(n, off, idx, w, nnz, labels, colbits, keys,
                                                                          vals);
    return hipGetLastError();
}
hipError_t launch_segment_heads(const uint64_t* keys, int64_t n, int32_t* head, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_segment_heads<<<LV_GRID(n)>>>(keys, n, head);
    return hipGetLastError();
}
hipError_t launch_segment_reduce(const uint64_t* keys, const int32_t* vals, const int32_t* pos, int64_t n, int colbits,
                                 int32_t* idx2, int32_t* w2, int32_t* rowcnt, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_segment_reduce<<<LV_GRID(n)>>>(keys, vals, pos, n, colbits, idx2, w2, rowcnt);
    return hipGetLastError();
}
hipError_t launch_compose(int32_t n0, int32_t* fin, const int32_t* labels, hipStream_t s)
{
    if (n0 <= 0) return hipSuccess;
    k_compose<<<LV_GRID(n0)>>>(n0, fin, labels);
    return hipGetLastError();
}
hipError_t launch_modularity_parts(int32_t n, const int32_t* off, const int32_t* idx, const int32_t* w, int64_t nnz,
                                   const int32_t* k, const int32_t* labels, int64_t* tot, int64_t* out2, hipStream_t s)
{
    if (n > 0) k_label_volumes<<<LV_GRID(n)>>>(n, k, labels, (unsigned long long*)tot);
    if (nnz > 0)
        k_sigma_in<<<(unsigned)((nnz + TILE - 1) / TILE), TILE_BS, 0, s>>>(n, off, idx, w, nnz, labels,
                                                                           (unsigned long long*)out2);
    if (n > 0) k_sum_sq_i64<<<grid_for(n, 256, 4096), 256, 0, s>>>((const unsigned long long*)tot, n,
                                                                   (unsigned long long*)(out2 + 1));
    return hipGetLastError();
}
hipError_t launch_sum_sq_i64(const int64_t* v, int64_t n, int64_t* out, hipStream_t s)
{
    if (n > 0) k_sum_sq_i64<<<grid_for(n, 256, 4096), 256, 0, s>>>((const unsigned long long*)v, n,
                                                                   (unsigned long long*)out);
    return hipGetLastError();
}
hipError_t launch_check_labels(const int32_t* labels, int32_t n, int32_t* err, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_check_labels<<<LV_GRID(n)>>>(labels, n, err);
    return hipGetLastError();
}

}  // namespace lv

namespace lv {
hipError_t launch_class_starts(const uint32_t* cls_sorted, int32_t n, int32_t* start, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_class_starts<<<LV_GRID(n)>>>(cls_sorted, n, start);
    return hipGetLastError();
}
hipError_t launch_gather_rows(const int32_t* verts, int32_t m, const int32_t* off, int32_t* beg, int32_t* len,
                              hipStream_t s)
{
    if (m <= 0) return hipSuccess;
    k_gather_rows<<<LV_GRID(m)>>>(verts, m, off, beg, len);
    return hipGetLastError();
}
}  // namespace lv

namespace lv {
namespace {
// out[c] = CSR entries of the vertices of class c (sorted lists: class c spans
// [start[c], start[c+1]))
__global__ __launch_bounds__(256) void k_class_entries(const int32_t* verts, int32_t lo, int32_t hi,
                                                        const int32_t* off, unsigned long long* out)
{
    __shared__ unsigned long long red[4];
    unsigned long long s = 0;
    for (int64_t t = lo + (int64_t)blockIdx.x * 256 + threadIdx.x; t < hi; t += (int64_t)gridDim.x * 256) {
        const int32_t v = verts[t];
        s += (unsigned long long)(off[v + 1] - off[v]);
    }
    s = block_sum256(s, red);
    if (threadIdx.x == 0 && s) atomicAdd(out, s);
}
}  // namespace

hipError_t launch_class_entries(const int32_t* verts_sorted, const int32_t* start, const int32_t* off,
                                int64_t* out, hipStream_t s)
{
    for (int c = CLS_G8; c < NUM_CLS; ++c) {
        const int32_t lo = start[c], hi = start[c + 1];
        if (hi <= lo) continue;
        k_class_entries<<<grid_for(hi - lo, 256, 4096), 256, 0, s>>>(verts_sorted, lo, hi, off,
                                                                     (unsigned long long*)(out + c));
    }
    return hipGetLastError();
}
}  // namespace lv
