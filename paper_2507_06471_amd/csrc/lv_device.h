// Device-side helpers shared by the kernel translation units (gfx950, wave64).
#pragma once

#include "lv_internal.h"

#include <limits.h>

namespace lv {
namespace dev {

constexpr int WAVE = 64;

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// number of set bits of `mask` below the calling lane
__device__ __forceinline__ uint32_t lane_rank(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// slot hash of a community id in an open-addressing table
__device__ __forceinline__ uint32_t mix32(int32_t key)
{
    uint32_t h = (uint32_t)key * 0x9E3779B1u;
    return h ^ (h >> 15);
}

// partition of a community id among P partitions (independent of mix32)
__device__ __forceinline__ uint32_t part_of(int32_t key, uint32_t P)
{
    uint32_t h = (uint32_t)key * 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return (uint32_t)(((uint64_t)h * P) >> 32);
}

__device__ __forceinline__ uint32_t pow2_at_least(uint32_t x)
{
    return x <= 1u ? 1u : 1u << (32 - __builtin_clz(x - 1u));
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
    const uint64_t m = __ballot(pred);
    if (m == 0) return -1;
    const uint32_t leader = (uint32_t)__ffsll((unsigned long long)m) - 1u;
    uint32_t base = 0;
    if (lane_id() == leader) base = atomicAdd(counter, (uint32_t)__popcll(m));
    base = __shfl(base, (int)leader);
    return pred ? (int32_t)(base + lane_rank(m)) : -1;
}

// Add `val` to arr[key] for every valid lane with one atomic per distinct key
// of the wave (lanes with equal keys are summed first).  Must be reached by
// all lanes of the wave.
template <typename T, typename A>
__device__ __forceinline__ void wave_grouped_add(A* arr, int64_t key, T val, bool valid)
{
    uint64_t pending = __ballot(valid);
    while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const int64_t lk = __shfl((long long)key, leader);
        const uint64_t grp = __ballot(valid && key == lk) & pending;
        T c = ((grp >> lane_id()) & 1ull) ? val : (T)0;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d);
        if ((int)lane_id() == leader) atomicAdd(&arr[lk], (A)c);
        pending &= ~grp;
    }
}

// Reduce (score, community, own-weight) over aligned groups of G lanes (G <= 64).
template <int G>
__device__ __forceinline__ void group_reduce(int64_t& s, int32_t& c, int32_t& wo)
{
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1) {
        const long long s2 = __shfl_xor((long long)s, m, G);
        const int32_t c2 = __shfl_xor(c, m, G);
        const int32_t w2 = __shfl_xor(wo, m, G);
        if (better(s2, c2, s, c)) { s = s2; c = c2; }
        wo = max(wo, w2);
    }
}

// Workgroup-wide reduce of (score, community, own-weight); result in thread 0.
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

// Workgroup sum; result valid in thread 0 (all threads must call).
template <int BS, typename T>
__device__ __forceinline__ T block_sum(T v, T* red)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    if (lane_id() == 0) red[threadIdx.x / WAVE] = v;
    __syncthreads();
    T t = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < BS / WAVE; ++w) t += red[w];
    __syncthreads();
    return t;
}

// Merge path over the sequence that interleaves the n row ends (row r ends at
// position off[r+1] + r) with the nnz CSR entries: the number of row ends
// among the first d items.
__device__ __forceinline__ int64_t mp_rows(const int32_t* off, int32_t n, int64_t d)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if ((int64_t)off[mid + 1] + mid < d) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Visit the CSR entries of merge-path tile `tile` with their row.
// Tile b covers merged items [b*T, (b+1)*T), T = BS*IT, so it spans at most T
// rows (empty rows included) and its row offsets always fit in LDS.  Thread t
// visits the tile's entries y0 + t*IT + j, j < IT, in order.  Every thread of
// the workgroup must call it (it synchronises).
template <int BS, int IT, typename F>
__device__ __forceinline__ void for_tile_entries_at(int64_t tile, const int32_t* off, int32_t n, int64_t nnz, F&& f)
{
    constexpr int T = BS * IT;
    __shared__ int32_t s_off[T + 2];
    __shared__ int64_t s_x[2];
    const int64_t total = (int64_t)n + nnz;
    const int64_t d0 = tile * T;
    const int64_t d1 = d0 + T < total ? d0 + T : total;
    if (threadIdx.x < 2) s_x[threadIdx.x] = mp_rows(off, n, threadIdx.x ? d1 : d0);
    __syncthreads();
    const int64_t x0 = s_x[0], x1 = s_x[1];
    const int64_t y0 = d0 - x0, y1 = d1 - x1;
    const int64_t last = x1 + 1 < n ? x1 + 1 : n;
    const int64_t cnt = last - x0 + 1;
    for (int64_t t = threadIdx.x; t < cnt; t += BS) s_off[t] = off[x0 + t];
    __syncthreads();
    const int64_t my0 = y0 + (int64_t)threadIdx.x * IT;
    if (my0 >= y1) return;
    int64_t lo = 0, hi = cnt;
    while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if ((int64_t)s_off[mid] <= my0) lo = mid + 1; else hi = mid;
    }
    int64_t r = x0 + lo - 1;
    for (int j = 0; j < IT; ++j) {
        const int64_t e = my0 + j;
        if (e >= y1) break;
        while ((int64_t)s_off[r + 1 - x0] <= e) ++r;
        f((int32_t)r, e);
    }
}

template <int BS, int IT, typename F>
__device__ __forceinline__ void for_tile_entries(const int32_t* off, int32_t n, int64_t nnz, F&& f)
{
    for_tile_entries_at<BS, IT>((int64_t)blockIdx.x, off, n, nnz, f);
}

// As for_tile_entries_at, but consecutive threads take consecutive entries
// (thread t visits y0 + t + j*BS), so loads and stores indexed by the entry
// coalesce.  The row of each entry is found first, by each thread walking IT
// consecutive entries, and kept in LDS.  Every thread of the workgroup must
// call it (it synchronises).
template <int BS, int IT, typename F>
__device__ __forceinline__ void for_tile_entries_co_at(int64_t tile, const int32_t* off, int32_t n, int64_t nnz, F&& f)
{
    constexpr int T = BS * IT;
    __shared__ int32_t s_off[T + 2];
    __shared__ int32_t s_row[T];
    __shared__ int64_t s_x[2];
    const int64_t total = (int64_t)n + nnz;
    const int64_t d0 = tile * T;
    const int64_t d1 = d0 + T < total ? d0 + T : total;
    if (threadIdx.x < 2) s_x[threadIdx.x] = mp_rows(off, n, threadIdx.x ? d1 : d0);
    __syncthreads();
    const int64_t x0 = s_x[0], x1 = s_x[1];
    const int64_t y0 = d0 - x0, y1 = d1 - x1;
    const int64_t last = x1 + 1 < n ? x1 + 1 : n;
    const int64_t cnt = last - x0 + 1;
    for (int64_t t = threadIdx.x; t < cnt; t += BS) s_off[t] = off[x0 + t];
    __syncthreads();
    const int64_t my0 = y0 + (int64_t)threadIdx.x * IT;
    if (my0 < y1) {
        int64_t lo = 0, hi = cnt;
        while (lo < hi) {
            const int64_t mid = (lo + hi) / 2;
            if ((int64_t)s_off[mid] <= my0) lo = mid + 1; else hi = mid;
        }
        int64_t r = x0 + lo - 1;
        for (int j = 0; j < IT; ++j) {
            const int64_t e = my0 + j;
            if (e >= y1) break;
            while ((int64_t)s_off[r + 1 - x0] <= e) ++r;
            s_row[e - y0] = (int32_t)r;
        }
    }
    __syncthreads();
    for (int j = 0; j < IT; ++j) {
        const int64_t e = y0 + threadIdx.x + (int64_t)j * BS;
        if (e >= y1) break;
        f(s_row[e - y0], e);
    }
}

// Probe sequence of key C in an LDS table (double hashing: start and stride
// from the key's hash, so that keys landing near each other do not follow
// one another's runs).  A power-of-two table (mask = slots - 1) takes an odd
// stride, which visits every slot within `slots` steps; a table of any size
// (MOD, mask = slots >= 2) takes a stride in [1, slots - 1] for 8 steps and
// then continues slot by slot, so it too reaches every slot.  Every lane
// holding key C walks the same sequence, which is all an insert needs:
// slots only change from empty to a key, so the first lane to claim takes the
// first empty slot of the sequence and every later one passes the same
// occupied slots to reach it.
struct Probe {
    uint32_t h, st, n;
};
template <bool MOD>
__device__ __forceinline__ Probe probe_start(int32_t C, uint32_t mask)
{
    const uint32_t hv = mix32(C);
    if constexpr (MOD)
        return Probe{(uint32_t)(((uint64_t)hv * mask) >> 32),
                     1u + (uint32_t)(((uint64_t)(hv * 0x85EBCA6Bu) * (mask - 1u)) >> 32), 0u};
    else
        return Probe{hv & mask, ((hv >> 16) | 1u) & mask, 0u};
}
template <bool MOD>
__device__ __forceinline__ void probe_next(Probe& p, uint32_t mask)
{
    if constexpr (MOD) {
        if (++p.n == 8u) p.st = 1u;
        p.h += p.st;
        if (p.h >= mask) p.h -= mask;
    } else {
        p.h = (p.h + p.st) & mask;
    }
}

// Insert (C, W) into an LDS open-addressing table that is guaranteed to have
// room (distinct keys < slots); the thread that claims a slot stores the
// community's volume S beside it.  The table has mask+1 slots (a power of
// two), or with MOD exactly `mask` slots of any count, hashed by a
// multiply-high reduction.
template <bool SIG, bool MOD = false>
__device__ __forceinline__ void lds_insert(int32_t* key, int32_t* val, int32_t* sig, uint32_t mask, int32_t C,
                                           int32_t W, int32_t S)
{
    Probe p = probe_start<MOD>(C, mask);
    int32_t prev;
    for (;;) {  // one exit test per probe; the stores after the loop
        prev = atomicCAS(&key[p.h], EMPTY_KEY, C);
        if (prev == EMPTY_KEY || prev == C) break;
        probe_next<MOD>(p, mask);
    }
    if constexpr (SIG) if (prev == EMPTY_KEY) sig[p.h] = S;
    atomicAdd(&val[p.h], W);
}

// Make a group's LDS writes visible to the whole group.  A group within one
// wavefront needs no workgroup barrier: a wavefront's LDS operations are
// performed in order, so a wavefront-scope fence (which keeps the compiler
// from moving LDS accesses across it) suffices, and the wavefronts of a
// workgroup do not wait for each other.
template <int G>
__device__ __forceinline__ void group_sync()
{
    if constexpr (G <= WAVE) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    } else {
        __syncthreads();
    }
}

constexpr int TILE_BS = 256;
constexpr int TILE_IT = 8;
constexpr int64_t TILE = TILE_BS * TILE_IT;

inline unsigned tiles_for(int32_t n, int64_t nnz)
{
    const int64_t t = ((int64_t)n + nnz + TILE - 1) / TILE;
    return (unsigned)(t > 0 ? t : 1);
}

// Block-wide flush of per-thread (graph, sum) accumulators: when every
// pending sum of the workgroup belongs to one graph, a single atomic;
// otherwise one atomic per distinct graph per wavefront.  All threads of the
// workgroup must call it.
template <int BS, typename T>
__device__ __forceinline__ void block_flush_sums(T* out, int64_t g, T s)
{
    __shared__ int64_t s_key[BS / WAVE];
    __shared__ T s_val[BS / WAVE];
    __shared__ int32_t s_mixed;
    const bool valid = g >= 0 && s != 0;
    const uint64_t vm = __ballot(valid);
    const int leader = vm ? __ffsll((unsigned long long)vm) - 1 : 0;
    const int64_t lk = __shfl((long long)g, leader);
    const bool uniform = __ballot(valid && g != lk) == 0;
    T c = valid ? s : (T)0;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d);
    if (threadIdx.x == 0) s_mixed = 0;
    __syncthreads();
    if (lane_id() == 0) {
        s_key[threadIdx.x / WAVE] = vm ? lk : -1;
        s_val[threadIdx.x / WAVE] = c;
        if (!uniform) s_mixed = 1;
    }
    __syncthreads();
    if (s_mixed) {
        wave_grouped_add<T, T>(out, valid ? g : 0, s, valid);
    } else if (threadIdx.x == 0) {
        int64_t cur = -1;
        T acc = 0;
        for (int w = 0; w < BS / WAVE; ++w) {
            if (s_key[w] < 0) continue;
            if (s_key[w] != cur) {
                if (cur >= 0 && acc) atomicAdd(&out[cur], acc);
                cur = s_key[w];
                acc = 0;
            }
            acc += s_val[w];
        }
        if (cur >= 0 && acc) atomicAdd(&out[cur], acc);
    }
}

inline int grid_for(int64_t n, int64_t per_block, int64_t cap = 1 << 20)
{
    int64_t b = (n + per_block - 1) / per_block;
    if (b < 1) b = 1;
    return (int)(b < cap ? b : cap);
}

}  // namespace dev
}  // namespace lv

#define LV_GRID(n) ::lv::dev::grid_for((n), 256, 65536), 256, 0, s
