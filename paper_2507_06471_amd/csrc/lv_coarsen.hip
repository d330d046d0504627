// Renumbering and aggregation by sorting (Algorithm 3 of arXiv 2507.06471) on
// gfx950; aggregation by community is in lv_agg.hip.
//
// Renumber: a community's new id is the rank of its smallest member vertex.
// Aggregation by sorting: every CSR entry (i, j, A_ij) becomes the key
// (label(i), label(j)) with weight A_ij; keys are radix-sorted and equal keys
// merged with their weights summed, giving the coarse CSR A' = S^T A S with
// sorted columns.  The community's internal weight lands on the diagonal,
// already in the doubled-loop convention, so degrees and M carry over.
#include "lv_device.h"

namespace lv {

using namespace dev;

namespace {

// Vertices are stored at positions i; orig[i] is the vertex id (null: i).
// Community ids are vertex ids, and renumbering goes by the smallest member
// id, so minv and the first-member flags are indexed by id.
// The lanes of a wavefront that share the first lane's community take one
// atomic together (a label held by most vertices, as after label
// propagation, would otherwise see one atomic per member); the others read
// the current minimum from L2 first and skip the atomic when it is smaller.
__device__ __forceinline__ void min_if_smaller(int32_t* at, int32_t v)
{
    if (__hip_atomic_load(at, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > v) atomicMin(at, v);
}
__global__ __launch_bounds__(256) void k_minv(int32_t n, const int32_t* comm, const int32_t* orig, int32_t* minv)
{
    for (int64_t base = (int64_t)blockIdx.x * 256; base < n; base += (int64_t)gridDim.x * 256) {
        const int64_t i = base + threadIdx.x;
        const bool ok = i < n;
        const int32_t c = ok ? comm[i] : 0;
        const int32_t id = ok ? (orig ? orig[i] : (int32_t)i) : INT32_MAX;
        const uint64_t live = __ballot(ok);
        if (live == 0) continue;
        const int leader = __ffsll((unsigned long long)live) - 1;
        const int32_t lc = __shfl(c, leader);
        const bool with = ok && c == lc;
        int32_t m = with ? id : INT32_MAX;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) m = min(m, __shfl_xor(m, d));
        if ((int)lane_id() == leader) min_if_smaller(&minv[lc], m);
        if (ok && !with) min_if_smaller(&minv[c], id);
    }
}
__global__ void k_first_flag(int32_t n, const int32_t* comm, const int32_t* orig, const int32_t* minv, int32_t* flag)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t id = orig ? orig[i] : (int32_t)i;
        flag[id] = minv[comm[i]] == id ? 1 : 0;
    }
}
__global__ void k_label(int32_t n, const int32_t* comm, const int32_t* minv, const int32_t* pos, int32_t* labels)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        labels[i] = pos[minv[comm[i]]];
}
// coarse degree of community P = its volume Sigma_tot, and its graph id
// (every member writes the same values)
__global__ void k_coarse_degree(int32_t n, const int32_t* comm, const int32_t* labels, const int32_t* sigma,
                                const int32_t* gid, int32_t* k2, int32_t* gid2)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        k2[labels[i]] = sigma[comm[i]];
        if (gid) gid2[labels[i]] = gid[i];
    }
}

// Aggregation keys.  Tile b covers merge-path items [b*AG_T, (b+1)*AG_T) of
// the n row ends and nnz entries; thread t takes AG_IT consecutive entries of
// it, loads their indices and weights and gathers their column labels before
// using any.  Each entry (i, j, w) becomes the key label(i) << colbits |
// label(j) with weight w.
//   SUM = false: every entry's key and weight go to keys[e], vals[e].
//   SUM = true (levels that merged strongly): the keys are added into the
// tile's LDS hash table.  An entry that finds no slot within AG_PROBE
// probes, or arrives once the table holds AG_FILL keys (a tile whose keys
// barely repeat stops summing early), is written out as it is (the global
// sort merges equal keys anyway), from the end of the tile's range.  Out: the table's distinct keys
// at keys[y0 + r], r < cnt[b], and the unplaced entries at
// keys[y0 + ne - ovf[b] + r], r < ovf[b].  meta holds four arrays of one
// int per tile: keys contributed (cnt + ovf), y0, cnt, ne.
// sigma_in[g] += weight of graph g's entries inside one community.
constexpr int AG_IT = 16;
constexpr int AG_T = TILE_BS * AG_IT;  // merge-path items per tile
constexpr int AG_HS = 2048;            // hash slots (24 KiB)
constexpr int AG_PROBE = 16;
constexpr int AG_FILL = AG_HS * 3 / 4;
constexpr uint64_t AG_EMPTY = ~0ull;   // keys use at most 62 bits

__device__ __forceinline__ uint32_t key_slot(uint64_t k)
{
    return (uint32_t)((k * 0x9E3779B97F4A7C15ull) >> 40) & (uint32_t)(AG_HS - 1);
}

// Adds (key, wv) to the table; *fill counts the keys placed so far.
__device__ __forceinline__ bool hash_add(uint64_t* h_key, int32_t* h_val, int32_t* fill, uint64_t key, int32_t wv)
{
    uint32_t h = key_slot(key);
    for (int p = 0; p < AG_PROBE; ++p) {
        const uint64_t prev =
            atomicCAS((unsigned long long*)&h_key[h], (unsigned long long)AG_EMPTY, (unsigned long long)key);
        if (prev == AG_EMPTY) atomicAdd(fill, 1);
        if (prev == AG_EMPTY || prev == key) { atomicAdd(&h_val[h], wv); return true; }
        h = (h + 1) & (uint32_t)(AG_HS - 1);
    }
    return false;
}

template <bool SUM>
__global__ __launch_bounds__(TILE_BS) void k_tile_keys(int32_t n, const int32_t* off, const int32_t* idx,
                                                        const int32_t* w, int64_t nnz, const int32_t* labels,
                                                        int colbits, uint64_t* keys, int32_t* vals, int32_t* meta,
                                                        const int32_t* gid, unsigned long long* sigma_in)
{
    __shared__ uint64_t h_key[SUM ? AG_HS : 1];
    __shared__ int32_t h_val[SUM ? AG_HS : 1];
    __shared__ int64_t s_x[2];
    __shared__ int32_t s_cnt, s_ovf, s_fill;
    const int64_t total = (int64_t)n + nnz;
    const int64_t d0 = (int64_t)blockIdx.x * AG_T;
    const int64_t d1 = d0 + AG_T < total ? d0 + AG_T : total;
    if (threadIdx.x < 2) s_x[threadIdx.x] = mp_rows(off, n, threadIdx.x ? d1 : d0);
    if (threadIdx.x == 0) { s_cnt = 0; s_ovf = 0; s_fill = 0; }
    if constexpr (SUM)
        for (int t = threadIdx.x; t < AG_HS; t += TILE_BS) { h_key[t] = AG_EMPTY; h_val[t] = 0; }
    __syncthreads();
    const int64_t x0 = s_x[0], x1 = s_x[1];
    const int64_t y0 = d0 - x0, y1 = d1 - x1;
    const int32_t ne = (int32_t)(y1 - y0);
    const int64_t last = x1 + 1 < n ? x1 + 1 : n;
    int32_t g_cur = -1;
    unsigned long long s = 0;
    const int32_t q0 = threadIdx.x * AG_IT;
    if (q0 < ne) {
        const int32_t m = ne - q0 < AG_IT ? ne - q0 : AG_IT;
        int32_t jj[AG_IT], ww[AG_IT];
#pragma unroll
        for (int u = 0; u < AG_IT; ++u) {
            jj[u] = u < m ? idx[y0 + q0 + u] : 0;
            ww[u] = (u < m && w) ? w[y0 + q0 + u] : 1;
        }
#pragma unroll
        for (int u = 0; u < AG_IT; ++u) jj[u] = u < m ? labels[jj[u]] : 0;
        int64_t lo = x0, hi = last;  // row of entry y0 + q0: last r with off[r] <= y0 + q0
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) / 2;
            if ((int64_t)off[mid] <= y0 + q0) lo = mid; else hi = mid - 1;
        }
        int64_t r = lo;
        int64_t rend = off[r + 1];
        uint32_t a = (uint32_t)labels[r];
        for (int u = 0; u < AG_IT; ++u) {  // left to the compiler: the early exit keeps it rolled
            if (u >= m) break;
            const int64_t e = y0 + q0 + u;
            if (e >= rend) {
                do { ++r; rend = off[r + 1]; } while (e >= rend);
                a = (uint32_t)labels[r];
            }
            const uint32_t b = (uint32_t)jj[u];
            const uint64_t key = ((uint64_t)a << colbits) | (uint64_t)b;
            if constexpr (SUM) {
                const bool full = *(volatile int32_t*)&s_fill >= AG_FILL;
                if (full || !hash_add(h_key, h_val, &s_fill, key, ww[u])) {
                    const int32_t p = ne - 1 - atomicAdd(&s_ovf, 1);
                    keys[y0 + p] = key;
                    vals[y0 + p] = ww[u];
                }
            } else {
                keys[e] = key;
                vals[e] = ww[u];
            }
            if (a == b) {
                const int32_t gg = gid ? gid[r] : 0;
                if (gg != g_cur) {
                    if (g_cur >= 0 && s) atomicAdd(&sigma_in[g_cur], s);
                    g_cur = gg;
                    s = 0;
                }
                s += (unsigned long long)ww[u];
            }
        }
    }
    if constexpr (SUM) {
    __syncthreads();
    // distinct keys out: one LDS atomic per wavefront reserves its positions
    for (int t0 = 0; t0 < AG_HS; t0 += TILE_BS) {
        const int t = t0 + threadIdx.x;
        const uint64_t k = h_key[t];
        const bool has = k != AG_EMPTY;
        const uint64_t mk = __ballot(has);
        int32_t wbase = 0;
        if (lane_id() == 0 && mk) wbase = atomicAdd(&s_cnt, __popcll(mk));
        wbase = __shfl(wbase, 0);
        if (has) {
            const int32_t pos = wbase + __popcll(mk & ((1ull << lane_id()) - 1ull));
            keys[y0 + pos] = k;
            vals[y0 + pos] = h_val[t];
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int64_t T = gridDim.x, b = blockIdx.x;
        meta[b] = s_cnt + s_ovf;  // keys the tile contributes
        meta[T + b] = (int32_t)y0;
        meta[2 * T + b] = s_cnt;
        meta[3 * T + b] = ne;
    }
    }
    const bool valid = g_cur >= 0 && s != 0;
    wave_grouped_add<unsigned long long, unsigned long long>(sigma_in, valid ? g_cur : 0, s, valid);
}

// Pack the tiles' keys densely: tile b's distinct keys [y0, y0 + c) and
// unplaced entries [y0 + ne - o, y0 + ne), o = total - c, go to pos[b] on.
__global__ __launch_bounds__(256) void k_compact_tiles(const uint64_t* keys, const int32_t* vals, const int32_t* meta,
                                                       const int32_t* pos, uint64_t* keys2, int32_t* vals2)
{
    const int64_t T = gridDim.x, b = blockIdx.x;
    const int32_t tot = meta[b], from = meta[T + b], c = meta[2 * T + b], ne = meta[3 * T + b];
    const int32_t to = pos[blockIdx.x];
    for (int32_t q = threadIdx.x; q < tot; q += 256) {
        const int32_t src = q < c ? from + q : from + ne - (tot - q);
        keys2[to + q] = keys[src];
        vals2[to + q] = vals[src];
    }
}

__global__ void k_segment_heads(const uint64_t* keys, int64_t n, int32_t* head)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        head[e] = (e == 0 || keys[e] != keys[e - 1]) ? 1 : 0;
}

// Sum the weights of each run of equal keys.  A workgroup stages its tile of
// 256 * SR_IT keys and weights in LDS (coalesced loads, plus the keys just
// before and after the tile); thread t then owns SR_IT consecutive entries.
// A run wholly inside one thread is stored directly, a run crossing a thread
// boundary is added atomically, one atomic per distinct run per wavefront.
// pos = exclusive scan of the head flags (output slot of a run).  Keys use at
// most 62 bits, so all-ones marks "no key".
constexpr int SR_IT = 8;
constexpr int SR_TILE = 256 * SR_IT;
__global__ __launch_bounds__(256) void k_segment_reduce(const uint64_t* keys, const int32_t* vals, const int32_t* pos,
                                                        int64_t n, int colbits, int32_t* idx2, int32_t* w2,
                                                        uint64_t* keys2)
{
    __shared__ uint64_t s_k[SR_TILE + 2];  // s_k[q + 1] = key of tile entry q
    __shared__ int32_t s_v[SR_TILE];
    const uint64_t cmask = (1ull << colbits) - 1ull;
    const uint64_t NONE = ~0ull;
    const int64_t tile0 = (int64_t)blockIdx.x * SR_TILE;
    const int32_t cnt = (int32_t)(n - tile0 < SR_TILE ? n - tile0 : SR_TILE);
    for (int32_t q = threadIdx.x; q < cnt; q += 256) {
        s_k[q + 1] = keys[tile0 + q];
        s_v[q] = vals[tile0 + q];
    }
    if (threadIdx.x == 0) s_k[0] = tile0 > 0 ? keys[tile0 - 1] : NONE;
    if (threadIdx.x == 1) s_k[cnt + 1] = tile0 + cnt < n ? keys[tile0 + cnt] : NONE;
    __syncthreads();
    const int32_t q0 = threadIdx.x * SR_IT;
    const int32_t q1 = q0 + SR_IT < cnt ? q0 + SR_IT : cnt;
    int64_t o_first = 0, o_last = 0;
    int32_t s_first = 0, s_last = 0;
    bool a_first = false, a_last = false;
    for (int32_t q = q0; q < q1;) {
        const uint64_t key = s_k[q + 1];
        const bool head = s_k[q] != key;
        int32_t sum = 0;
        int32_t q2 = q;
        while (q2 < q1 && s_k[q2 + 1] == key) { sum += s_v[q2]; ++q2; }
        const int64_t o = (int64_t)pos[tile0 + q] + (head ? 1 : 0) - 1;
        if (head) { idx2[o] = (int32_t)(key & cmask); keys2[o] = key; }
        const bool cont_next = q2 == q1 && s_k[q1 + 1] == key;
        if (head && !cont_next) {
            w2[o] = sum;
        } else if (!head) {  // continues from the previous thread (only the first run can)
            a_first = true; o_first = o; s_first = sum;
        } else {             // starts here and continues into the next thread
            a_last = true; o_last = o; s_last = sum;
        }
        q = q2;
    }
    wave_grouped_add<int32_t, int32_t>(w2, o_first, s_first, a_first);
    wave_grouped_add<int32_t, int32_t>(w2, o_last, s_last, a_last);
}

// off2[r] = first coarse entry of row r (keys2 sorted, row in the high bits)
// Graph construction from an undirected edge list (Section II-A: an edge set
// of unordered pairs, loops allowed).  Edge t = (u, v, w) becomes the keys
// u:v and v:u with weight w (one key u:u for a loop, none for a dropped loop);
// unused slots get the all-ones key of 2*cb bits, which sorts last.  Per
// workgroup: stats[0] += kept entries, stats[1] += their volume (a loop's
// weight counted twice, as the weighted degree does); err |= 2 for an
// endpoint outside [0, n), 4 for a weight < 1.
__global__ __launch_bounds__(256) void k_edge_keys(int64_t m, const int32_t* src, const int32_t* dst, const int32_t* w,
                                                   int32_t n, int cb, int drop_loops, uint64_t* keys, int32_t* vals,
                                                   unsigned long long* stats, int32_t* err)
{
    __shared__ unsigned long long red[256 / WAVE];
    const uint64_t none = (1ull << (2 * cb)) - 1ull;
    unsigned long long ne = 0, vol = 0;
    int32_t bad = 0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t u = src[t], v = dst[t], x = w ? w[t] : 1;
        uint64_t k0 = none, k1 = none;
        if (u < 0 || u >= n || v < 0 || v >= n) {
            bad |= 2;
        } else if (x < 1) {
            bad |= 4;
        } else if (u != v) {
            k0 = ((uint64_t)u << cb) | (uint64_t)v;
            k1 = ((uint64_t)v << cb) | (uint64_t)u;
            ne += 2;
            vol += 2ull * (unsigned long long)x;
        } else if (!drop_loops) {
            k0 = ((uint64_t)u << cb) | (uint64_t)u;
            ne += 1;
            vol += 2ull * (unsigned long long)x;
        }
        keys[2 * t] = k0;
        keys[2 * t + 1] = k1;
        vals[2 * t] = x;
        vals[2 * t + 1] = x;
    }
    if (bad) atomicOr(err, bad);
    ne = block_sum<256>(ne, red);
    vol = block_sum<256>(vol, red);
    if (threadIdx.x == 0 && ne) {
        atomicAdd(&stats[0], ne);
        atomicAdd(&stats[1], vol);
    }
}

// Stored loops are doubled (A_vv = 2w); the caller's convention carries w.
__global__ void k_halve_diagonal(const uint64_t* keys2, int64_t e2, int cb, int32_t* w2)
{
    const uint64_t lo = (1ull << cb) - 1ull;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < e2; e += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t k = keys2[e];
        if ((k >> cb) == (k & lo)) w2[e] /= 2;
    }
}

__global__ void k_row_offsets(const uint64_t* keys2, int64_t e2, int32_t n2, int colbits, int32_t* off2)
{
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r <= n2; r += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t key = (uint64_t)r << colbits;
        int64_t lo = 0, hi = e2;
        while (lo < hi) {
            const int64_t mid = (lo + hi) / 2;
            if (keys2[mid] < key) lo = mid + 1; else hi = mid;
        }
        off2[r] = (int32_t)lo;
    }
}

// Compose final labels of packed original vertices with one level's labels:
// for a vertex of original graph g that takes part at slot c = slot[g] >= 0
// (vertex base vbase[c], label base nbase[c] in the level's packed graph):
// fin = labels[vbase + fin] - nbase.  gid0 null: one graph at slot 0, bases 0.
__global__ void k_compose(int32_t n0, int32_t* fin, const int32_t* labels, const int32_t* gid0, const int32_t* slot,
                          const int32_t* vbase, const int32_t* nbase)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n0; v += (int64_t)gridDim.x * blockDim.x) {
        if (!gid0) { fin[v] = labels[fin[v]]; continue; }
        const int32_t c = slot[gid0[v]];
        if (c < 0) continue;
        fin[v] = labels[vbase[c] + fin[v]] - nbase[c];
    }
}

// Copy CSR segments into one packed CSR.  Segment q takes vertices
// [src_vb, src_vb + n) of its source CSR (their entries are contiguous and
// only point inside the segment) to vertices [dst_vb, dst_vb + n) and
// entries from dst_eb; indices are shifted accordingly; weights default to 1
// and degrees are copied; gid of the new vertices = q; orig (if not null)
// gets each new vertex's id: its segment's first id plus its id within the
// segment (src_orig, else its position).
__global__ void k_repack_vertices(const RepackSeg* seg, int32_t nseg, int32_t n_out, int32_t* off, int32_t* k,
                                  int32_t* gid, int32_t* orig, int64_t nnz_out)
{
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n_out; u += (int64_t)gridDim.x * blockDim.x) {
        int32_t lo = 0, hi = nseg;  // last segment with dst_vb <= u
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) / 2;
            if (seg[mid].dst_vb <= u) lo = mid; else hi = mid;
        }
        const RepackSeg& q = seg[lo];
        const int64_t x = u - q.dst_vb;
        const int64_t src_e0 = q.src_off[q.src_vb];
        off[u] = (int32_t)(q.src_off[q.src_vb + x] - src_e0 + q.dst_eb);
        k[u] = q.src_k[q.src_vb + x];
        if (gid) gid[u] = lo;
        if (orig) orig[u] = q.dst_vb + (q.src_orig ? q.src_orig[q.src_vb + x] - q.src_vb : (int32_t)x);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) off[n_out] = (int32_t)nnz_out;
}
__global__ void k_repack_entries(const RepackSeg* seg, int32_t nseg, int64_t nnz_out, int32_t* idx, int32_t* w)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz_out; e += (int64_t)gridDim.x * blockDim.x) {
        int32_t lo = 0, hi = nseg;  // last segment with dst_eb <= e
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) / 2;
            if (seg[mid].dst_eb <= e) lo = mid; else hi = mid;
        }
        const RepackSeg& q = seg[lo];
        const int64_t se = q.src_off[q.src_vb] + (e - q.dst_eb);
        idx[e] = q.src_idx[se] - q.src_vb + q.dst_vb;
        w[e] = q.src_w ? q.src_w[se] : 1;
    }
}

// out[v] = labels[v] - base[gid[v]] (labels numbered from 0 within each graph)
__global__ void k_local_labels(int32_t n, const int32_t* labels, const int32_t* gid, const int32_t* base, int32_t* out)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        out[v] = labels[v] - (gid ? base[gid[v]] : 0);
}

}  // namespace

hipError_t launch_local_labels(int32_t n, const int32_t* labels, const int32_t* gid, const int32_t* base, int32_t* out,
                               hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_local_labels<<<LV_GRID(n)>>>(n, labels, gid, base, out);
    return hipGetLastError();
}

hipError_t launch_renumber(int32_t n, const int32_t* comm, const int32_t* orig, int32_t* minv, int32_t* flag,
                           int32_t* pos, int32_t* labels, int32_t* n_out, void* tmp, size_t tb, hipStream_t s)
{
    if (n <= 0) return hipMemsetAsync(n_out, 0, sizeof(int32_t), s);
    hipError_t e = launch_fill_i32(minv, INT32_MAX, n, s);
    if (e != hipSuccess) return e;
    k_minv<<<LV_GRID(n)>>>(n, comm, orig, minv);
    k_first_flag<<<LV_GRID(n)>>>(n, comm, orig, minv, flag);
    e = scan_exclusive_i32(flag, pos, n, n_out, tmp, tb, s);
    if (e != hipSuccess) return e;
    k_label<<<LV_GRID(n)>>>(n, comm, minv, pos, labels);
    return hipGetLastError();
}
hipError_t launch_coarse_degree(int32_t n, const int32_t* comm, const int32_t* labels, const int32_t* sigma,
                                const int32_t* gid, int32_t* k2, int32_t* gid2, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_coarse_degree<<<LV_GRID(n)>>>(n, comm, labels, sigma, gid, k2, gid2);
    return hipGetLastError();
}
unsigned build_keys_tiles(int32_t n, int64_t nnz)
{
    const int64_t t = ((int64_t)n + nnz + AG_T - 1) / AG_T;
    return (unsigned)(t > 0 ? t : 1);
}
hipError_t launch_build_keys(bool agg, int32_t n, const int32_t* off, const int32_t* idx, const int32_t* w, int64_t nnz,
                             const int32_t* labels, int colbits, uint64_t* keys, int32_t* vals, int32_t* meta,
                             const int32_t* gid, int64_t* sigma_in, hipStream_t s)
{
    if (agg)
        k_tile_keys<true><<<build_keys_tiles(n, nnz), TILE_BS, 0, s>>>(n, off, idx, w, nnz, labels, colbits, keys, vals,
                                                                        meta, gid, (unsigned long long*)sigma_in);
    else if (nnz > 0)
        k_tile_keys<false><<<build_keys_tiles(n, nnz), TILE_BS, 0, s>>>(n, off, idx, w, nnz, labels, colbits, keys,
                                                                         vals, meta, gid, (unsigned long long*)sigma_in);
    return hipGetLastError();
}
hipError_t launch_compact_tiles(const uint64_t* keys, const int32_t* vals, const int32_t* meta, const int32_t* pos,
                                unsigned tiles, uint64_t* keys2, int32_t* vals2, hipStream_t s)
{
    k_compact_tiles<<<tiles, 256, 0, s>>>(keys, vals, meta, pos, keys2, vals2);
    return hipGetLastError();
}
hipError_t launch_repack(const RepackSeg* seg, int32_t nseg, int32_t n_out, int64_t nnz_out, int32_t* off, int32_t* idx,
                         int32_t* w, int32_t* k, int32_t* gid, int32_t* orig, hipStream_t s)
{
    if (nseg <= 0) return hipSuccess;
    k_repack_vertices<<<LV_GRID((int64_t)n_out + 1)>>>(seg, nseg, n_out, off, k, gid, orig, nnz_out);
    if (nnz_out > 0) k_repack_entries<<<LV_GRID(nnz_out)>>>(seg, nseg, nnz_out, idx, w);
    return hipGetLastError();
}
hipError_t launch_segment_heads(const uint64_t* keys, int64_t n, int32_t* head, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_segment_heads<<<LV_GRID(n)>>>(keys, n, head);
    return hipGetLastError();
}
hipError_t launch_segment_reduce(const uint64_t* keys, const int32_t* vals, const int32_t* pos, int64_t n, int colbits,
                                 int32_t* idx2, int32_t* w2, uint64_t* keys2, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_segment_reduce<<<(unsigned)((n + SR_TILE - 1) / SR_TILE), 256, 0, s>>>(keys, vals, pos, n, colbits,
                                                                                       idx2, w2, keys2);
    return hipGetLastError();
}
hipError_t launch_edge_keys(int64_t m, const int32_t* src, const int32_t* dst, const int32_t* w, int32_t n, int cb,
                            bool drop_loops, uint64_t* keys, int32_t* vals, int64_t* stats, int32_t* err, hipStream_t s)
{
    if (m <= 0) return hipSuccess;
    k_edge_keys<<<LV_GRID(m)>>>(m, src, dst, w, n, cb, drop_loops ? 1 : 0, keys, vals, (unsigned long long*)stats, err);
    return hipGetLastError();
}
hipError_t launch_halve_diagonal(const uint64_t* keys2, int64_t e2, int cb, int32_t* w2, hipStream_t s)
{
    if (e2 <= 0) return hipSuccess;
    k_halve_diagonal<<<LV_GRID(e2)>>>(keys2, e2, cb, w2);
    return hipGetLastError();
}
hipError_t launch_row_offsets(const uint64_t* keys2, int64_t e2, int32_t n2, int colbits, int32_t* off2, hipStream_t s)
{
    k_row_offsets<<<LV_GRID((int64_t)n2 + 1)>>>(keys2, e2, n2, colbits, off2);
    return hipGetLastError();
}
hipError_t launch_compose(int32_t n0, int32_t* fin, const int32_t* labels, const int32_t* gid0, const int32_t* slot,
                          const int32_t* vbase, const int32_t* nbase, hipStream_t s)
{
    if (n0 <= 0) return hipSuccess;
    k_compose<<<LV_GRID(n0)>>>(n0, fin, labels, gid0, slot, vbase, nbase);
    return hipGetLastError();
}

}  // namespace lv
