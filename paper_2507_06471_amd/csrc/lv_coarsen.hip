// Renumbering and aggregation (Algorithm 3 of arXiv 2507.06471) on gfx950.
//
// Renumber (K9): a community's new id is the rank of its smallest member
// vertex.  Aggregation (K10/K11): every CSR entry (i, j, A_ij) becomes the key
// (label(i), label(j)) with weight A_ij; keys are radix-sorted and equal keys
// merged with their weights summed, giving the coarse CSR A' = S^T A S with
// sorted columns.  The community's internal weight lands on the diagonal,
// already in the doubled-loop convention, so degrees and M carry over.
#include "lv_device.h"

namespace lv {

using namespace dev;

namespace {

__global__ void k_minv(int32_t n, const int32_t* comm, int32_t* minv)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t c = comm[i];
        if (minv[c] > (int32_t)i) atomicMin(&minv[c], (int32_t)i);  // read first: skips most contended atomics
    }
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
// coarse degree of community P = its volume Sigma_tot (written by its smallest member)
__global__ void k_coarse_degree(int32_t n, const int32_t* comm, const int32_t* flag, const int32_t* labels,
                                const int32_t* sigma, int32_t* k2)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (flag[i]) k2[labels[i]] = sigma[comm[i]];
}

// keys/vals per entry; sigma_in += weight of entries inside one community
__global__ __launch_bounds__(TILE_BS) void k_build_keys(int32_t n, const int32_t* off, const int32_t* idx,
                                                         const int32_t* w, int64_t nnz, const int32_t* labels,
                                                         int colbits, uint64_t* keys, int32_t* vals,
                                                         unsigned long long* sigma_in)
{
    __shared__ unsigned long long red[TILE_BS / WAVE];
    unsigned long long s = 0;
    for_tile_entries<TILE_BS, TILE_IT>(off, n, nnz, [&](int32_t r, int64_t e) {
        const uint32_t a = (uint32_t)labels[r], b = (uint32_t)labels[idx[e]];
        const int32_t wv = w ? w[e] : 1;
        keys[e] = ((uint64_t)a << colbits) | (uint64_t)b;
        vals[e] = wv;
        if (a == b) s += (unsigned long long)wv;
    });
    s = block_sum<TILE_BS>(s, red);
    if (threadIdx.x == 0 && s) atomicAdd(sigma_in, s);
}

__global__ void k_segment_heads(const uint64_t* keys, int64_t n, int32_t* head)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        head[e] = (e == 0 || keys[e] != keys[e - 1]) ? 1 : 0;
}

// Sum the weights of each run of equal keys.  Thread t owns SR_IT consecutive
// entries; a run wholly inside one thread is stored directly, a run crossing
// a thread boundary is added atomically, one atomic per distinct run per
// wavefront.  pos = exclusive scan of the head flags (output slot of a run).
constexpr int SR_IT = 8;
__global__ __launch_bounds__(256) void k_segment_reduce(const uint64_t* keys, const int32_t* vals, const int32_t* pos,
                                                        int64_t n, int colbits, int32_t* idx2, int32_t* w2,
                                                        uint64_t* keys2)
{
    const uint64_t cmask = (1ull << colbits) - 1ull;
    const int64_t base = ((int64_t)blockIdx.x * 256 + threadIdx.x) * SR_IT;
    const int64_t end = base + SR_IT < n ? base + SR_IT : n;
    int64_t o_first = 0, o_last = 0;
    int32_t s_first = 0, s_last = 0;
    bool a_first = false, a_last = false;
    for (int64_t e = base; e < end;) {
        const uint64_t key = keys[e];
        const bool head = e == 0 || keys[e - 1] != key;
        const int64_t o = (int64_t)pos[e] + (head ? 1 : 0) - 1;
        int32_t sum = 0;
        int64_t e2 = e;
        while (e2 < end && keys[e2] == key) { sum += vals[e2]; ++e2; }
        if (head) { idx2[o] = (int32_t)(key & cmask); keys2[o] = key; }
        const bool cont_next = e2 == end && end < n && keys[end] == key;
        if (head && !cont_next) {
            w2[o] = sum;
        } else if (!head) {  // continues from the previous thread (only the first run can)
            a_first = true; o_first = o; s_first = sum;
        } else {             // starts here and continues into the next thread
            a_last = true; o_last = o; s_last = sum;
        }
        e = e2;
    }
    wave_grouped_add<int32_t, int32_t>(w2, o_first, s_first, a_first);
    wave_grouped_add<int32_t, int32_t>(w2, o_last, s_last, a_last);
}

// off2[r] = first coarse entry of row r (keys2 sorted, row in the high bits)
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

__global__ void k_compose(int32_t n0, int32_t* fin, const int32_t* labels)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n0; v += (int64_t)gridDim.x * blockDim.x)
        fin[v] = labels[fin[v]];
}

}  // namespace

hipError_t launch_renumber(int32_t n, const int32_t* comm, int32_t* minv, int32_t* flag, int32_t* pos, int32_t* labels,
                           int32_t* n_out, void* tmp, size_t tb, hipStream_t s)
{
    if (n <= 0) return hipMemsetAsync(n_out, 0, sizeof(int32_t), s);
    hipError_t e = launch_fill_i32(minv, INT32_MAX, n, s);
    if (e != hipSuccess) return e;
    k_minv<<<LV_GRID(n)>>>(n, comm, minv);
    k_first_flag<<<LV_GRID(n)>>>(n, comm, minv, flag);
    e = scan_exclusive_i32(flag, pos, n, n_out, tmp, tb, s);
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
                             const int32_t* labels, int colbits, uint64_t* keys, int32_t* vals, int64_t* sigma_in,
                             hipStream_t s)
{
    if (nnz <= 0) return hipSuccess;
    k_build_keys<<<tiles_for(n, nnz), TILE_BS, 0, s>>>(n, off, idx, w, nnz, labels, colbits, keys, vals,
                                                        (unsigned long long*)sigma_in);
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
    k_segment_reduce<<<(unsigned)((n + 256 * SR_IT - 1) / (256 * SR_IT)), 256, 0, s>>>(keys, vals, pos, n, colbits,
                                                                                       idx2, w2, keys2);
    return hipGetLastError();
}
hipError_t launch_row_offsets(const uint64_t* keys2, int64_t e2, int32_t n2, int colbits, int32_t* off2, hipStream_t s)
{
    k_row_offsets<<<LV_GRID((int64_t)n2 + 1)>>>(keys2, e2, n2, colbits, off2);
    return hipGetLastError();
}
hipError_t launch_compose(int32_t n0, int32_t* fin, const int32_t* labels, hipStream_t s)
{
    if (n0 <= 0) return hipSuccess;
    k_compose<<<LV_GRID(n0)>>>(n0, fin, labels);
    return hipGetLastError();
}

}  // namespace lv
