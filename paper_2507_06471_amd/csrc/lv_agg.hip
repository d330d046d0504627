// Aggregation by community (Algorithm 3's coarse graph A' = S^T A S) without
// sorting every entry.
//
// The entries of a level are first laid out community by community: members
// of coarse vertex P (vertices with label P) have their rows copied, with
// every column replaced by its label, into one contiguous segment
// [seg[P], seg[P+1]) of a staging array.  Row P of A' is then the sum of
// equal labels within that segment.  Segments of up to 8192 entries are
// summed in an LDS table by one group of lanes (the degree classes of the
// local-moving kernels, applied to segment lengths); longer segments go
// through the sort-and-reduce path.  Each segment's distinct (label, weight)
// pairs land at its own start in a second staging array, and a final pass
// packs them into the coarse CSR.  Columns within a coarse row are in table
// order, not sorted: every consumer of a coarse level sums over a row.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "lv_device.h"

namespace lv {
using namespace dev;

namespace {

constexpr int AGG_UNROLL = 4;

// dm[q] = row length of vertex mem[q]
__global__ void k_member_lengths(int32_t n, const int32_t* mem, const int32_t* off, int32_t* dm)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = mem[q];
        dm[q] = off[v + 1] - off[v];
    }
}

// seg[P] = first staging entry of coarse vertex P: the entry offset of its
// first member in label order (every label in [0, n2) has a member);
// seg[n2] = nnz.
__global__ void k_segment_starts(int32_t n, const uint32_t* lab_sorted, const int32_t* voff, int32_t n2, int32_t nnz,
                                 int32_t* seg)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t P = lab_sorted[q];
        if (q == 0 || lab_sorted[q - 1] != P) seg[P] = voff[q];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) seg[n2] = nnz;
}

// One group of G lanes per listed coarse vertex P: sum its segment's
// (label, weight) pairs in an LDS table of up to SLOTS slots, write the
// distinct pairs to [seg[P], seg[P] + c) of the output staging arrays and
// c to cnt[P]; the pair whose label is P itself adds its weight to the
// graph's Sigma_in.
template <int BS, int G, int SLOTS>
__global__ __launch_bounds__(BS) void k_agg_class(const int32_t* __restrict__ verts, int32_t m,
                                                  const int32_t* __restrict__ seg, const int32_t* __restrict__ col,
                                                  const int32_t* __restrict__ wt, int32_t* __restrict__ col2,
                                                  int32_t* __restrict__ wt2, int32_t* __restrict__ cnt,
                                                  const int32_t* __restrict__ gid2, unsigned long long* sigma_in)
{
    constexpr int NG = BS / G;
    constexpr bool POW2 = (SLOTS & (SLOTS - 1)) == 0;
    __shared__ int32_t s_key[NG * SLOTS];
    __shared__ int32_t s_val[NG * SLOTS];
    __shared__ int32_t s_n[NG];
    const int g = threadIdx.x / G, lane = threadIdx.x % G;
    const int64_t vi = (int64_t)blockIdx.x * NG + g;
    const bool has = vi < m;
    const int32_t P = has ? verts[vi] : 0;
    const int32_t beg = has ? seg[P] : 0, end = has ? seg[P + 1] : 0;
    int32_t* key = s_key + g * SLOTS;
    int32_t* val = s_val + g * SLOTS;
    // a segment of L entries has at most L distinct labels; SLOTS exceeds the
    // class's longest segment, so the table never fills
    const uint32_t L2 = 2u * (uint32_t)(end - beg);
    const uint32_t T = POW2 ? min((uint32_t)SLOTS, max(2u, pow2_at_least(L2))) : min((uint32_t)SLOTS, L2 + 1u);
    for (uint32_t t = lane; t < T; t += G) { key[t] = EMPTY_KEY; val[t] = 0; }
    if (lane == 0) s_n[g] = 0;
    group_sync<G>();
    for (int32_t e0 = beg + lane; e0 < end; e0 += G * AGG_UNROLL) {
        int32_t cc[AGG_UNROLL], ww[AGG_UNROLL];
#pragma unroll
        for (int u = 0; u < AGG_UNROLL; ++u) {
            const int32_t e = e0 + u * G;
            const bool ok = e < end;
            cc[u] = ok ? col[e] : EMPTY_KEY;
            ww[u] = ok ? (wt ? wt[e] : 1) : 0;
        }
#pragma unroll
        for (int u = 0; u < AGG_UNROLL; ++u)
            if (cc[u] != EMPTY_KEY) lds_insert<false, !POW2>(key, val, nullptr, POW2 ? T - 1u : T, cc[u], ww[u], 0);
    }
    group_sync<G>();
    unsigned long long own = 0;
    for (uint32_t t = lane; t < T; t += G) {
        const int32_t C = key[t];
        if (C == EMPTY_KEY) continue;
        const int32_t p = atomicAdd(&s_n[g], 1);
        col2[beg + p] = C;
        wt2[beg + p] = val[t];
        if (C == P) own = (unsigned long long)val[t];
    }
    group_sync<G>();
    if (has && lane == 0) cnt[P] = s_n[g];
    block_flush_sums<BS, unsigned long long>(sigma_in, own ? (gid2 ? gid2[P] : 0) : -1, own);
}

// Long segments: key (P << colbits) | label and weight of every entry, laid
// out by hoff (row r = coarse vertex hv[r]).
__global__ __launch_bounds__(TILE_BS) void k_long_keys(int32_t nh, const int32_t* hv, const int32_t* hoff, int64_t eh,
                                                       const int32_t* seg, const int32_t* col, const int32_t* wt,
                                                       int colbits, uint64_t* keys, int32_t* vals)
{
    for_tile_entries_co_at<TILE_BS, TILE_IT>((int64_t)blockIdx.x, hoff, nh, eh, [&](int32_t r, int64_t e) {
        const int32_t P = hv[r];
        const int64_t src = (int64_t)seg[P] + (e - hoff[r]);
        keys[e] = ((uint64_t)(uint32_t)P << colbits) | (uint64_t)(uint32_t)col[src];
        vals[e] = wt ? wt[src] : 1;
    });
}

// hd[r] = segment length of coarse vertex hv[r]
__global__ void k_long_lengths(int32_t nh, const int32_t* hv, const int32_t* seg, int32_t* hd)
{
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nh; r += (int64_t)gridDim.x * blockDim.x)
        hd[r] = seg[hv[r] + 1] - seg[hv[r]];
}

// The sorted, reduced pairs of long segments (distinct key u: row keys2[u] >>
// colbits, first pair of row P at uoff[P]) to their segments' starts.
__global__ void k_long_place(int64_t eu, const uint64_t* keys2, const int32_t* col_u, const int32_t* wt_u,
                             const int32_t* uoff, const int32_t* seg, int colbits, int32_t* col2, int32_t* wt2,
                             const int32_t* gid2, unsigned long long* sigma_in)
{
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < eu; u += (int64_t)gridDim.x * blockDim.x) {
        const int32_t P = (int32_t)(keys2[u] >> colbits);
        const int64_t dst = (int64_t)seg[P] + (u - uoff[P]);
        col2[dst] = col_u[u];
        wt2[dst] = wt_u[u];
        if (col_u[u] == P) atomicAdd(&sigma_in[gid2 ? gid2[P] : 0], (unsigned long long)wt_u[u]);
    }
}

__global__ void k_long_counts(int32_t nh, const int32_t* hv, const int32_t* uoff, int32_t* cnt)
{
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nh; r += (int64_t)gridDim.x * blockDim.x) {
        const int32_t P = hv[r];
        cnt[P] = uoff[P + 1] - uoff[P];
    }
}

// Pack: entry e of coarse row P (off2) from seg[P] + (e - off2[P]).
__global__ __launch_bounds__(TILE_BS) void k_pack_rows(int32_t n2, const int32_t* off2, int64_t e2, const int32_t* seg,
                                                       const int32_t* col2, const int32_t* wt2, int32_t* idx,
                                                       int32_t* w)
{
    for_tile_entries_co_at<TILE_BS, TILE_IT>((int64_t)blockIdx.x, off2, n2, e2, [&](int32_t P, int64_t e) {
        const int64_t src = (int64_t)seg[P] + (e - off2[P]);
        idx[e] = col2[src];
        w[e] = wt2[src];
    });
}

// Row sort of a CSR (export): keys (row << colbits) | column, then back.
__global__ __launch_bounds__(TILE_BS) void k_row_keys(int32_t n, const int32_t* off, int64_t nnz, const int32_t* idx,
                                                      const int32_t* w, int colbits, uint64_t* keys, int32_t* vals)
{
    for_tile_entries_co_at<TILE_BS, TILE_IT>((int64_t)blockIdx.x, off, n, nnz, [&](int32_t r, int64_t e) {
        keys[e] = ((uint64_t)(uint32_t)r << colbits) | (uint64_t)(uint32_t)idx[e];
        vals[e] = w[e];
    });
}
__global__ void k_unpack_keys(int64_t nnz, const uint64_t* keys, const int32_t* vals, int colbits, int32_t* idx,
                              int32_t* w)
{
    const uint64_t mask = (1ull << colbits) - 1ull;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
        idx[e] = (int32_t)(keys[e] & mask);
        w[e] = vals[e];
    }
}

template <int BS, int G, int SLOTS>
hipError_t launch_agg_t(const AggArgs& a, hipStream_t s)
{
    static_assert(BS % G == 0, "groups per workgroup");
    if (a.m <= 0) return hipSuccess;
    constexpr int NG = BS / G;
    const unsigned grid = (unsigned)((a.m + NG - 1) / NG);
    k_agg_class<BS, G, SLOTS><<<grid, BS, 0, s>>>(a.verts, a.m, a.seg, a.col, a.wt, a.col2, a.wt2, a.cnt, a.gid2,
                                                  (unsigned long long*)a.sigma_in);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_member_lengths(int32_t n, const int32_t* mem, const int32_t* off, int32_t* dm, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_member_lengths<<<LV_GRID(n)>>>(n, mem, off, dm);
    return hipGetLastError();
}
hipError_t launch_segment_starts(int32_t n, const uint32_t* lab_sorted, const int32_t* voff, int32_t n2, int32_t nnz,
                                 int32_t* seg, hipStream_t s)
{
    k_segment_starts<<<LV_GRID(std::max(n, 1))>>>(n, lab_sorted, voff, n2, nnz, seg);
    return hipGetLastError();
}
// Table sizes as the local-moving classes, in 8-byte slots (no volumes).
hipError_t launch_agg_class(int cls, const AggArgs& a, hipStream_t s)
{
    switch (cls) {
    case CLS_L4: return launch_agg_t<256, 4, 8>(a, s);
    case CLS_L8: return launch_agg_t<256, 8, 16>(a, s);
    case CLS_L32: return launch_agg_t<256, 16, 64>(a, s);
    case CLS_L128: return launch_agg_t<256, 32, 208>(a, s);
    case CLS_L256: return launch_agg_t<256, 64, 424>(a, s);
    case CLS_L512: return launch_agg_t<256, 128, 848>(a, s);
    case CLS_L1K: return launch_agg_t<256, 256, 1696>(a, s);
    case CLS_L2K: return launch_agg_t<512, 512, 3392>(a, s);
    case CLS_L3K: return launch_agg_t<512, 512, 4096>(a, s);
    case CLS_L8K: return launch_agg_t<1024, 1024, L8K_SLOTS>(a, s);
    default: return hipErrorInvalidValue;
    }
}
hipError_t launch_long_lengths(int32_t nh, const int32_t* hv, const int32_t* seg, int32_t* hd, hipStream_t s)
{
    if (nh <= 0) return hipSuccess;
    k_long_lengths<<<LV_GRID(nh)>>>(nh, hv, seg, hd);
    return hipGetLastError();
}
hipError_t launch_long_keys(int32_t nh, const int32_t* hv, const int32_t* hoff, int64_t eh, const int32_t* seg,
                            const int32_t* col, const int32_t* wt, int colbits, uint64_t* keys, int32_t* vals,
                            hipStream_t s)
{
    if (nh <= 0 || eh <= 0) return hipSuccess;
    k_long_keys<<<tiles_for(nh, eh), TILE_BS, 0, s>>>(nh, hv, hoff, eh, seg, col, wt, colbits, keys, vals);
    return hipGetLastError();
}
hipError_t launch_long_place(int64_t eu, const uint64_t* keys2, const int32_t* col_u, const int32_t* wt_u,
                             const int32_t* uoff, const int32_t* seg, int colbits, int32_t* col2, int32_t* wt2,
                             const int32_t* gid2, int64_t* sigma_in, hipStream_t s)
{
    if (eu <= 0) return hipSuccess;
    k_long_place<<<LV_GRID(eu)>>>(eu, keys2, col_u, wt_u, uoff, seg, colbits, col2, wt2, gid2,
                                  (unsigned long long*)sigma_in);
    return hipGetLastError();
}
hipError_t launch_long_counts(int32_t nh, const int32_t* hv, const int32_t* uoff, int32_t* cnt, hipStream_t s)
{
    if (nh <= 0) return hipSuccess;
    k_long_counts<<<LV_GRID(nh)>>>(nh, hv, uoff, cnt);
    return hipGetLastError();
}
hipError_t launch_pack_rows(int32_t n2, const int32_t* off2, int64_t e2, const int32_t* seg, const int32_t* col2,
                            const int32_t* wt2, int32_t* idx, int32_t* w, hipStream_t s)
{
    if (n2 <= 0 || e2 <= 0) return hipSuccess;
    k_pack_rows<<<tiles_for(n2, e2), TILE_BS, 0, s>>>(n2, off2, e2, seg, col2, wt2, idx, w);
    return hipGetLastError();
}
hipError_t launch_row_keys(int32_t n, const int32_t* off, int64_t nnz, const int32_t* idx, const int32_t* w,
                           int colbits, uint64_t* keys, int32_t* vals, hipStream_t s)
{
    if (n <= 0 || nnz <= 0) return hipSuccess;
    k_row_keys<<<tiles_for(n, nnz), TILE_BS, 0, s>>>(n, off, nnz, idx, w, colbits, keys, vals);
    return hipGetLastError();
}
hipError_t launch_unpack_keys(int64_t nnz, const uint64_t* keys, const int32_t* vals, int colbits, int32_t* idx,
                              int32_t* w, hipStream_t s)
{
    if (nnz <= 0) return hipSuccess;
    k_unpack_keys<<<LV_GRID(nnz)>>>(nnz, keys, vals, colbits, idx, w);
    return hipGetLastError();
}

}  // namespace lv
