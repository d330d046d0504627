// Graph preparation, validation and modularity kernels (gfx950).
//
// Graph model of the paper's Section II-A: undirected, integer weights, a loop
// counts twice in the weighted degree (stored as A_vv = 2w).  Modularity of
// Section II-C in integer form: Q_int = M * Sigma_in - sum_C Sigma_tot(C)^2.
#include "lv_device.h"

namespace lv {

using namespace dev;

namespace {

// err bits: 1 offsets, 2 indices, 4 weights, 8 asymmetric, 16 overflow
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
            const int64_t mid = (lo + hi) / 2;
            if (idx[mid] < r) lo = mid + 1; else hi = mid;
        }
        if (lo >= off[j + 1] || idx[lo] != r || (w && w[lo] != w[e])) atomicOr(err, 8);
    });
}

// diag_pos[i] = entry of the loop (i, i), or -1
__global__ void k_diag_scan(int32_t n, const int32_t* off, const int32_t* idx, int32_t* diag_pos, int32_t* any)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = off[i], hi = off[i + 1];
        while (lo < hi) {
            const int64_t mid = (lo + hi) / 2;
            if (idx[mid] < i) lo = mid + 1; else hi = mid;
        }
        const bool has = lo < off[i + 1] && idx[lo] == i;
        diag_pos[i] = has ? (int32_t)lo : -1;
        if (has) atomicOr(any, 1);
    }
}

// A = caller weights (or 1); each loop entry doubled
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

// k64[r] += row sums: per-thread runs of one row, one atomic per run
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
    s = block_sum<256>(s, red);
    if (threadIdx.x == 0) atomicAdd(total, s);
}

__global__ void k_degree_unit(int32_t n, const int32_t* off, int32_t* k)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        k[i] = off[i + 1] - off[i];
}

// Per-thread running sum for one graph, flushed when the graph changes and at
// the end (one atomic per graph per wavefront in the common case).
struct GraphAcc {
    int32_t g = -1;
    unsigned long long s = 0;
    __device__ void add(unsigned long long* out, int32_t gg, unsigned long long x)
    {
        if (gg != g) {
            if (g >= 0 && s) atomicAdd(&out[g], s);
            g = gg;
            s = 0;
        }
        s += x;
    }
    // all threads of a 256-thread workgroup must call it
    __device__ void flush_block(unsigned long long* out) { block_flush_sums<256, unsigned long long>(out, g, s); }
};

// Merge-path tiles visited by each workgroup of a grid of at most this many
// (fewer workgroups, fewer atomics on the per-graph sums)
constexpr unsigned SUM_GRID = 2048;

// out[g] += sum of v_i^2 (or v_i) over the vertices of graph g (gid null: one graph)
template <bool SQUARE>
__global__ __launch_bounds__(256) void k_sum_sq(int64_t n, const int32_t* v, const int32_t* gid,
                                                unsigned long long* out)
{
    GraphAcc acc;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int64_t x = (int64_t)v[i];
        acc.add(out, gid ? gid[i] : 0, (unsigned long long)(SQUARE ? x * x : x));
    }
    acc.flush_block(out);
}

// gid[v] = graph of vertex v: the last g with voff[g] <= v
__global__ void k_fill_gid(const int32_t* voff, int32_t G, int32_t n, int32_t* gid)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        int32_t lo = 0, hi = G;
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) / 2;
            if (voff[mid] <= v) lo = mid; else hi = mid;
        }
        gid[v] = lo;
    }
}

// out[g] += trace (sum of diagonal entries) of graph g
__global__ __launch_bounds__(TILE_BS) void k_trace(int32_t n, const int32_t* off, const int32_t* idx, const int32_t* w,
                                                    int64_t nnz, const int32_t* gid, unsigned long long* out)
{
    GraphAcc acc;
    const int64_t tiles = ((int64_t)n + nnz + TILE - 1) / TILE;
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x)
        for_tile_entries_co_at<TILE_BS, TILE_IT>(t, off, n, nnz, [&](int32_t r, int64_t e) {
            if (idx[e] == r) acc.add(out, gid ? gid[r] : 0, (unsigned long long)(w ? w[e] : 1));
        });
    acc.flush_block(out);
}

// out[g] += Sigma_in of graph g: entries whose endpoints share a label
__global__ __launch_bounds__(TILE_BS) void k_sigma_in(int32_t n, const int32_t* off, const int32_t* idx, const int32_t* w,
                                                       int64_t nnz, const int32_t* labels, const int32_t* gid,
                                                       unsigned long long* out)
{
    GraphAcc acc;
    const int64_t tiles = ((int64_t)n + nnz + TILE - 1) / TILE;
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x)
        for_tile_entries_co_at<TILE_BS, TILE_IT>(t, off, n, nnz, [&](int32_t r, int64_t e) {
            if (labels[idx[e]] == labels[r]) acc.add(out, gid ? gid[r] : 0, (unsigned long long)(w ? w[e] : 1));
        });
    acc.flush_block(out);
}

// Sigma_in without gathers: the neighbour's label of every entry is read
// from the entry cache, in entry order (loop entries, EMPTY_KEY there, are
// left to the caller).
__global__ __launch_bounds__(TILE_BS) void k_sigma_in_cached(int32_t n, const int32_t* off, const int2* ce,
                                                              const int32_t* w, int64_t nnz, const int32_t* labels,
                                                              unsigned long long* out)
{
    GraphAcc acc;
    const int64_t tiles = ((int64_t)n + nnz + TILE - 1) / TILE;
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x)
        for_tile_entries_co_at<TILE_BS, TILE_IT>(t, off, n, nnz, [&](int32_t r, int64_t e) {
            if (__builtin_nontemporal_load(&ce[e].x) == labels[r])
                acc.add(out, 0, (unsigned long long)(w ? w[e] : 1));
        });
    acc.flush_block(out);
}

// tot[label] += k_i, one atomic per distinct label of a wavefront
__global__ __launch_bounds__(256) void k_label_volumes(int32_t n, const int32_t* k, const int32_t* labels,
                                                       unsigned long long* tot)
{
    for (int64_t base = (int64_t)blockIdx.x * 256; base < n; base += (int64_t)gridDim.x * 256) {
        const int64_t i = base + threadIdx.x;
        const bool valid = i < n;
        const int32_t lab = valid ? labels[i] : 0;
        const unsigned long long kv = valid ? (unsigned long long)k[i] : 0ull;
        wave_grouped_add<unsigned long long, unsigned long long>(tot, lab, kv, valid);
    }
}

__global__ __launch_bounds__(256) void k_sum_sq_u64(const unsigned long long* v, int64_t n, unsigned long long* out)
{
    __shared__ unsigned long long red[4];
    unsigned long long s = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) s += v[i] * v[i];
    s = block_sum<256>(s, red);
    if (threadIdx.x == 0 && s) atomicAdd(out, s);
}

__global__ void k_check_labels(const int32_t* labels, int32_t n, int32_t* err)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (labels[i] < 0 || labels[i] >= n) atomicOr(err, 1);
}

// ---- storage order by descending degree
// key of position v: graph id above (maxdeg - degree), so that a stable sort
// keeps each packed graph's segment in place and puts its high-degree
// vertices first (ties keep their order)
__global__ void k_degree_keys(int32_t n, const int32_t* off, const int32_t* gid, int32_t maxdeg, int db, uint64_t* keys,
                              int32_t* vals)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t g = gid ? (uint64_t)gid[v] : 0ull;
        keys[v] = (g << db) | (uint64_t)(maxdeg - (off[v + 1] - off[v]));
        vals[v] = (int32_t)v;
    }
}
__global__ __launch_bounds__(256) void k_max_degree(int32_t n, const int32_t* off, int32_t* out)
{
    int32_t m = 0;
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < n; v += (int64_t)gridDim.x * 256)
        m = max(m, off[v + 1] - off[v]);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) m = max(m, __shfl_xor(m, d));
    if (lane_id() == 0) atomicMax(out, m);
}
__global__ void k_inverse(const int32_t* perm, int32_t n, int32_t* inv)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        inv[perm[q]] = (int32_t)q;
}
__global__ void k_perm_lengths(const int32_t* perm, int32_t n, const int32_t* off, int32_t* len)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = perm[q];
        len[q] = off[v + 1] - off[v];
    }
}
// new row q = old row perm[q], its column positions mapped through inv
__global__ __launch_bounds__(TILE_BS) void k_perm_rows(int32_t n, const int32_t* off_new, int64_t nnz,
                                                        const int32_t* perm, const int32_t* off, const int32_t* idx,
                                                        const int32_t* w, const int32_t* inv, int32_t* idx_new,
                                                        int32_t* w_new, const int32_t* rank, int32_t* rev_new)
{
    for_tile_entries_co_at<TILE_BS, TILE_IT>((int64_t)blockIdx.x, off_new, n, nnz, [&](int32_t q, int64_t e) {
        const int64_t src = (int64_t)off[perm[q]] + (e - off_new[q]);
        const int32_t p = inv[idx[src]];
        idx_new[e] = p;
        if (w) w_new[e] = w[src];
        // the reverse entry keeps its rank within its (moved) row
        if (rank) rev_new[e] = off_new[p] + rank[src];
    });
}

// Reverse-entry ranks of a CSR with sorted rows.  Each unordered pair {i, j}
// (i != j) is handled once, by its entry in the longer row (ties: the larger
// row id), which binary-searches the shorter row for the reverse entry and
// writes both ranks; a loop is its own reverse.
__global__ __launch_bounds__(TILE_BS) void k_reverse_rank(int32_t n, const int32_t* off, const int32_t* idx,
                                                           int64_t nnz, int32_t* rank, int32_t* err)
{
    for_tile_entries<TILE_BS, TILE_IT>(off, n, nnz, [&](int32_t r, int64_t e) {
        const int32_t j = idx[e];
        const int32_t rb = off[r];
        if (j == r) { rank[e] = (int32_t)(e - rb); return; }
        const int32_t jb = off[j], je = off[j + 1];
        const int32_t dr = off[r + 1] - rb, dj = je - jb;
        if (!(dj < dr || (dj == dr && j < r))) return;
        int32_t lo = jb, hi = je;
        while (lo < hi) {
            const int32_t mid = lo + (hi - lo) / 2;
            if (idx[mid] < r) lo = mid + 1; else hi = mid;
        }
        if (lo >= je || idx[lo] != r) { atomicOr(err, 32); return; }
        rank[e] = lo - jb;
        rank[lo] = (int32_t)(e - rb);
    });
}

__global__ void k_reverse_from_rank(const int32_t* off, const int32_t* idx, int64_t nnz, const int32_t* rank,
                                    int32_t* rev)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x)
        rev[e] = off[idx[e]] + rank[e];
}
__global__ void k_scatter_i32(const int32_t* src, const int32_t* idx, int32_t m, int32_t* dst)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x)
        dst[idx[t]] = src[t];
}

}  // namespace

hipError_t launch_degree_keys(int32_t n, const int32_t* off, const int32_t* gid, int32_t maxdeg, int db, uint64_t* keys,
                              int32_t* vals, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_degree_keys<<<LV_GRID(n)>>>(n, off, gid, maxdeg, db, keys, vals);
    return hipGetLastError();
}
hipError_t launch_max_degree(int32_t n, const int32_t* off, int32_t* out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_max_degree<<<grid_for(n, 256, 4096), 256, 0, s>>>(n, off, out);
    return hipGetLastError();
}
hipError_t launch_inverse(const int32_t* perm, int32_t n, int32_t* inv, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_inverse<<<LV_GRID(n)>>>(perm, n, inv);
    return hipGetLastError();
}
hipError_t launch_perm_lengths(const int32_t* perm, int32_t n, const int32_t* off, int32_t* len, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_perm_lengths<<<LV_GRID(n)>>>(perm, n, off, len);
    return hipGetLastError();
}
hipError_t launch_perm_rows(int32_t n, const int32_t* off_new, int64_t nnz, const int32_t* perm, const int32_t* off,
                            const int32_t* idx, const int32_t* w, const int32_t* inv, int32_t* idx_new, int32_t* w_new,
                            const int32_t* rank, int32_t* rev_new, hipStream_t s)
{
    if (nnz <= 0) return hipSuccess;
    k_perm_rows<<<tiles_for(n, nnz), TILE_BS, 0, s>>>(n, off_new, nnz, perm, off, idx, w, inv, idx_new, w_new, rank,
                                                      rev_new);
    return hipGetLastError();
}
hipError_t launch_reverse_rank(int32_t n, const int32_t* off, const int32_t* idx, int64_t nnz, int32_t* rank,
                               int32_t* err, hipStream_t s)
{
    if (nnz <= 0) return hipSuccess;
    k_reverse_rank<<<tiles_for(n, nnz), TILE_BS, 0, s>>>(n, off, idx, nnz, rank, err);
    return hipGetLastError();
}
hipError_t launch_reverse_from_rank(int32_t n, const int32_t* off, const int32_t* idx, int64_t nnz,
                                    const int32_t* rank, int32_t* rev, hipStream_t s)
{
    if (nnz <= 0) return hipSuccess;
    (void)n;
    k_reverse_from_rank<<<LV_GRID(nnz)>>>(off, idx, nnz, rank, rev);
    return hipGetLastError();
}
hipError_t launch_scatter_i32(const int32_t* src, const int32_t* idx, int32_t m, int32_t* dst, hipStream_t s)
{
    if (m <= 0) return hipSuccess;
    k_scatter_i32<<<LV_GRID(m)>>>(src, idx, m, dst);
    return hipGetLastError();
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
    k_check_entries<<<tiles_for(n, nnz), TILE_BS, 0, s>>>(n, off, idx, w, nnz, err);
    return hipGetLastError();
}
hipError_t launch_check_symmetric(int32_t n, const int32_t* off, const int32_t* idx, const int32_t* w, int64_t nnz,
                                  int32_t* err, hipStream_t s)
{
    if (nnz <= 0) return hipSuccess;
    k_check_symmetric<<<tiles_for(n, nnz), TILE_BS, 0, s>>>(n, off, idx, w, nnz, err);
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
    if (nnz > 0) k_row_sums<<<tiles_for(n, nnz), TILE_BS, 0, s>>>(n, off, w, nnz, (unsigned long long*)k64);
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
hipError_t launch_sum_sq(const int32_t* v, int64_t n, const int32_t* gid, int64_t* out, hipStream_t s)
{
    if (n > 0) k_sum_sq<true><<<grid_for(n, 256, 4096), 256, 0, s>>>(n, v, gid, (unsigned long long*)out);
    return hipGetLastError();
}
hipError_t launch_seg_sum(const int32_t* v, int64_t n, const int32_t* gid, int64_t* out, hipStream_t s)
{
    if (n > 0) k_sum_sq<false><<<grid_for(n, 256, 4096), 256, 0, s>>>(n, v, gid, (unsigned long long*)out);
    return hipGetLastError();
}
hipError_t launch_fill_gid(const int32_t* voff, int32_t G, int32_t n, int32_t* gid, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_fill_gid<<<LV_GRID(n)>>>(voff, G, n, gid);
    return hipGetLastError();
}
hipError_t launch_trace(int32_t n, const int32_t* off, const int32_t* idx, const int32_t* w, int64_t nnz,
                        const int32_t* gid, int64_t* out, hipStream_t s)
{
    if (nnz > 0) k_trace<<<std::min(tiles_for(n, nnz), SUM_GRID), TILE_BS, 0, s>>>(n, off, idx, w, nnz, gid, (unsigned long long*)out);
    return hipGetLastError();
}
hipError_t launch_sigma_in(int32_t n, const int32_t* off, const int32_t* idx, const int32_t* w, int64_t nnz,
                           const int32_t* labels, const int32_t* gid, int64_t* out, hipStream_t s)
{
    if (nnz > 0)
        k_sigma_in<<<std::min(tiles_for(n, nnz), SUM_GRID), TILE_BS, 0, s>>>(n, off, idx, w, nnz, labels, gid, (unsigned long long*)out);
    return hipGetLastError();
}
hipError_t launch_sigma_in_cached(int32_t n, const int32_t* off, const int2* ce, const int32_t* w, int64_t nnz,
                                  const int32_t* labels, int64_t* out, hipStream_t s)
{
    if (nnz > 0)
        k_sigma_in_cached<<<std::min(tiles_for(n, nnz), SUM_GRID), TILE_BS, 0, s>>>(n, off, ce, w, nnz, labels,
                                                                                     (unsigned long long*)out);
    return hipGetLastError();
}
hipError_t launch_modularity_parts(int32_t n, const int32_t* off, const int32_t* idx, const int32_t* w, int64_t nnz,
                                   const int32_t* k, const int32_t* labels, int64_t* tot, int64_t* out2, hipStream_t s)
{
    if (n > 0) k_label_volumes<<<grid_for(n, 256, 65536), 256, 0, s>>>(n, k, labels, (unsigned long long*)tot);
    if (nnz > 0)
        k_sigma_in<<<std::min(tiles_for(n, nnz), SUM_GRID), TILE_BS, 0, s>>>(n, off, idx, w, nnz, labels, nullptr,
                                                         (unsigned long long*)out2);
    if (n > 0)
        k_sum_sq_u64<<<grid_for(n, 256, 4096), 256, 0, s>>>((const unsigned long long*)tot, n,
                                                            (unsigned long long*)(out2 + 1));
    return hipGetLastError();
}
hipError_t launch_check_labels(const int32_t* labels, int32_t n, int32_t* err, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_check_labels<<<LV_GRID(n)>>>(labels, n, err);
    return hipGetLastError();
}

}  // namespace lv
