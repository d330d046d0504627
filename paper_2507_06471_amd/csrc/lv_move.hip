// Move step of local moving (Algorithm 2 of arXiv 2507.06471; Algorithm 1's
// PLPMove in LPA mode) on gfx950.
//
// Every vertex i sums its edge weights per neighbouring community,
// W_i(C) = cut_w(i, C \ {i}), then takes the best community by the exact
// integer score M*W_i(C) - k_i*Sigma_tot(C) (Louvain; Equation 1's gain is
// 2*(score - stay)/M^2) or W_i(C) (LPA), ties to the smallest id, and records
// a move if it beats staying and lies in the sweep's direction.  All reads are
// of the previous sweep's state.  Each vertex's decision (target community or
// -1) is written to its slot of the class-sorted vertex list; k_apply then
// commits the moves.
//
// Scheduling by the vertex's number of CSR entries L (degree classes): about
// one lane per four entries, so that a lane keeps four loads in flight and a
// compute unit holds many vertices.  Claim tables (8-byte slots: community
// and weight sum; the claimer scores with the volume that came with its
// entry) let every class run 8 wavefronts a SIMD: at most 20 KiB per
// 256-thread, 40 KiB per 512-thread and 80 KiB per 1024-thread workgroup.
// Sizes that are not a power of two hash by a multiply-high reduction; keys
// probe by double hashing; a row of L entries uses about 3L of the slots
// (table_pct), at least L + 1, so a table never fills.
//   L <= 4      later sweeps: one lane per vertex, no table (k_move_reg);
//               first sweep: 4 lanes per vertex
//   L <= 8      4 lanes, 32 slots
//   L <= 32     8 lanes, 64 slots
//   L <= 128    32 lanes, 312 slots
//   L <= 256    a wavefront, 624 slots
//   L <= 512    128 lanes, 1248 slots
//   L <= 1024   a 256-thread workgroup, 2496 slots
//   L <= 2048   a 512-thread workgroup, 5056 slots
//   L <= 3072   a 512-thread workgroup, 5056 slots
//   L <= 8192   a 1024-thread workgroup, 10112 slots (79 KiB, two
//               workgroups a CU)
//   L >  8192   P = ceil(L / part_keys) workgroups per vertex;
//               workgroup p aggregates the communities of hash partition p in
//               an LDS table; partial results are merged per vertex, and all P
//               workgroups of a vertex run on one XCD (shared L2).  Two modes:
//               compact tables of up to 16384 slots, each workgroup re-reading
//               the vertex's entries and keeping its partition's; or (with
//               P > 1) a scatter pass that reads the entries once, sums them
//               per community within chunks of 1024-4096 entries, and appends each
//               (community, volume, weight) to its partition's bucket, and
//               256-thread workgroups with 2048-slot tables fed from the
//               buckets.  If a partition's bucket or table ever fills up,
//               that vertex is redone with a global-memory table (it keeps
//               every input exact and finite).
// In the first sweep of a level every community is a single vertex and CSR
// columns are unique, so W_i(j) = A_ij and entries are scored directly.
//
// Memory traffic: a neighbour's community and that community's volume are
// read together as one 8-byte pair cs[j] = (comm[j], Sigma_tot(comm[j]))
// (refreshed after every commit), so an entry costs one random gather and the
// volume is kept in the LDS slot beside the summed weight.  Compact tables (8
// bytes a slot, twice the slots per workgroup) instead gather the volume once
// per distinct community.  CSR indices and weights are streamed with
// non-temporal loads so they do not evict the frequently gathered pairs from
// L2.
#include "lv_device.h"

namespace lv {

using namespace dev;

namespace {

struct Bounds { int32_t b[NUM_CLS]; };

__global__ void k_classify(int32_t n, const int32_t* off, Bounds bd, uint32_t* cls, int32_t* vert)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t L = off[i + 1] - off[i];
        uint32_t c = CLS_NONE;
        if (L > 0) {
            c = CLS_HUB;
            for (int q = CLS_L4; q < CLS_HUB; ++q)
                if (L <= bd.b[q]) { c = (uint32_t)q; break; }
        }
        cls[i] = c;
        vert[i] = (int32_t)i;
    }
}

__global__ void k_class_starts(const uint32_t* cls, int32_t n, int32_t* start)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        if (t == 0 || cls[t] != cls[t - 1]) start[cls[t]] = (int32_t)t;
}

__global__ __launch_bounds__(256) void k_class_entries(const int32_t* verts, int32_t lo, int32_t hi, const int32_t* off,
                                                       unsigned long long* out)
{
    __shared__ unsigned long long red[4];
    unsigned long long s = 0;
    for (int64_t t = lo + (int64_t)blockIdx.x * 256 + threadIdx.x; t < hi; t += (int64_t)gridDim.x * 256) {
        const int32_t v = verts[t];
        s += (unsigned long long)(off[v + 1] - off[v]);
    }
    s = block_sum<256>(s, red);
    if (threadIdx.x == 0 && s) atomicAdd(out, s);
}

__global__ void k_row_descriptors(const int32_t* verts, int32_t m, const int32_t* off, const int32_t* k, int4* rows)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = verts[t];
        rows[t] = make_int4(v, off[v], off[v + 1], k[v]);
    }
}

__global__ void k_gather_rows(const int32_t* verts, int32_t m, const int32_t* off, int32_t* beg, int32_t* len)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = verts[t];
        beg[t] = off[v];
        len[t] = off[v + 1] - off[v];
    }
}

constexpr int UNROLL = 4;

// Sweep direction from the device-side sweep counter: sweeps 1, 3, ... move
// down, sweeps 2, 4, ... up.
__device__ __forceinline__ int sweep_dir(const SweepCtl* c) { return (c->sweep % 2 == 0) ? DIR_DOWN : DIR_UP; }

// Total volume of the graph vertex i belongs to (graphs packed in one CSR
// each keep their own M), and whether that graph has stopped this level.
__device__ __forceinline__ int64_t vertex_M(const MoveArgs& a, int32_t i) { return a.Mg ? a.Mg[a.gid[i]] : a.M; }
__device__ __forceinline__ bool vertex_frozen(const MoveArgs& a, int32_t i)
{
    return a.gdone && a.gdone[a.gid ? a.gid[i] : 0];
}

// Active-vertex pruning (Alg. 1's V_active, Alg. 2's needCheck) for
// synchronous sweeps: sweep s evaluates every vertex while s <= 2, afterwards
// only a vertex that, or one of whose neighbours, changed community in sweep
// s-1 or s-2.  mark[i] holds the last such sweep (0 at the level's start).
__device__ __forceinline__ bool vertex_skipped(const MoveArgs& a, int32_t i)
{
    if (!a.mark) return false;
    const int32_t s = a.ctl->sweep + 1;
    return s > a.prune_back && a.mark[i] < s - a.prune_back;
}

// Asynchronous mode (Alg. 2 as written: labels and community volumes change
// in place while the sweep runs).  Label and (label, volume) of vertex j as
// they stand now, or from the sweep's snapshot in synchronous mode.
__device__ __forceinline__ int32_t comm_now(const MoveArgs& a, int32_t j)
{
    return a.live_comm ? a.live_comm[j] : a.cs[j].x;
}
__device__ __forceinline__ int2 pair_now(const MoveArgs& a, int32_t j)
{
    if (!a.live_comm) return a.cs[j];
    const int32_t c = a.live_comm[j];
    return make_int2(c, a.live_sigma[c]);
}
// Graph-major index into gmoves of vertex i's graph for the current sweep.
__device__ __forceinline__ int64_t move_slot(const MoveArgs& a, int32_t i)
{
    return (a.gid ? (int64_t)a.gid[i] * a.max_sweeps : 0) + a.ctl->sweep;
}

// Louvain's integer score M*W - k_i*Sigma (Eq. 1 up to the factor 2/M^2).
// Every factor lies in [0, 2^31): weights and volumes are non-negative and
// the library rejects a total volume of 2^31 or more.  So each product is one
// 32 x 32 -> 64-bit multiply, exact, where int64 operands would cost a full
// 64-bit one.
__device__ __forceinline__ int64_t louvain_score(int64_t M, int64_t W, int64_t ki, int64_t vol)
{
    return (int64_t)((uint64_t)(uint32_t)M * (uint32_t)W) - (int64_t)((uint64_t)(uint32_t)ki * (uint32_t)vol);
}

// Asynchronous decision of vertex i (own community A read when its table was
// built; only i changes its own label): against the live volume of A, move
// at once if the best community beats staying (no direction gate), updating
// both volumes atomically and the label in place.  Returns whether i moved.
__device__ __forceinline__ bool decide_apply(const MoveArgs& a, int64_t pos, int32_t i, int32_t A, int64_t ki,
                                             int64_t M, int64_t best_s, int32_t best_c, int32_t w_own)
{
    bool mover = false;
    if (best_c != INT32_MAX) {
        const bool louvain = a.mode == MODE_LOUVAIN;
        const int64_t sA = louvain ? (int64_t)a.live_sigma[A] : 0;
        const int64_t stay = louvain ? louvain_score(M, w_own, ki, sA - ki) : (int64_t)w_own;
        mover = best_s > stay;
    }
    if (mover) {
        atomicAdd(&a.live_sigma[A], -(int32_t)ki);
        atomicAdd(&a.live_sigma[best_c], (int32_t)ki);
        a.live_comm[i] = best_c;
    }
    a.dec[pos] = mover ? best_c : -1;
    return mover;
}

// Decision of vertex-list slot `pos`: the best community if it beats staying
// and lies in the sweep's direction, else -1.
__device__ __forceinline__ void decide_store(const MoveArgs& a, int64_t pos, int32_t A, int32_t sA, int64_t ki,
                                             int64_t M, int64_t best_s, int32_t best_c, int32_t w_own)
{
    bool mover = false;
    if (best_c != INT32_MAX) {
        const bool louvain = a.mode == MODE_LOUVAIN;
        const int64_t stay = louvain ? louvain_score(M, w_own, ki, (int64_t)sA - ki) : (int64_t)w_own;
        const bool dir_ok = sweep_dir(a.ctl) == DIR_DOWN ? best_c < A : best_c > A;
        mover = best_s > stay && dir_ok;
    }
    a.dec[pos] = mover ? best_c : -1;
}

// Entry cache access: 8-byte streaming load / store of entry e's pair.
__device__ __forceinline__ int2 ce_load(const int2* ce, int64_t e)
{
    const long long v = __builtin_nontemporal_load((const long long*)ce + e);
    return make_int2((int32_t)(uint32_t)(unsigned long long)v, (int32_t)((unsigned long long)v >> 32));
}
__device__ __forceinline__ void ce_store(int2* ce, int64_t e, int2 p)
{
    const unsigned long long v = ((unsigned long long)(uint32_t)p.y << 32) | (uint32_t)p.x;
    __builtin_nontemporal_store((long long)v, (long long*)ce + e);
}
// How this sweep's kernels get the entries' pairs (EC_GATHER without a cache).
__device__ __forceinline__ int entry_mode(const MoveArgs& a) { return a.ce ? a.ctl->ec_mode : EC_GATHER; }

// Score every entry of [e_beg, e_end) as its own community (first sweep of a level).
template <int STRIDE>
__device__ __forceinline__ void score_entries_singleton(const MoveArgs& a, int32_t i, int64_t ki, int64_t M,
                                                        int32_t e_beg, int32_t e_end, int64_t& best_s, int32_t& best_c)
{
    const bool louvain = a.mode == MODE_LOUVAIN;
    for (int32_t e0 = e_beg; e0 < e_end; e0 += STRIDE * UNROLL) {
        int32_t jj[UNROLL], ww[UNROLL];
        int2 cc[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int32_t e = e0 + u * STRIDE;
            const bool ok = e < e_end;
            jj[u] = ok ? __builtin_nontemporal_load(&a.idx[e]) : i;
            ww[u] = (ok && a.w) ? __builtin_nontemporal_load(&a.w[e]) : 1;
        }
        // A singleton neighbour's community is its vertex id, which differs
        // from its storage position when rows are kept in degree order.
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) cc[u] = jj[u] != i ? a.cs[jj[u]] : make_int2(0, 0);
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            if (jj[u] == i) continue;
            const int64_t s = louvain ? louvain_score(M, ww[u], ki, cc[u].y) : (int64_t)ww[u];
            if (better(s, cc[u].x, best_s, best_c)) { best_s = s; best_c = cc[u].x; }
        }
    }
}

// As lds_insert, but gives up (returns false) after probing every slot.
template <bool SIG>
__device__ __forceinline__ bool lds_insert_bounded(int32_t* key, int32_t* val, int32_t* sig, uint32_t mask, int32_t C,
                                                   int32_t W, int32_t S)
{
    Probe p = probe_start<false>(C, mask);  // power of two: every slot within mask + 1 probes
    for (uint32_t probes = 0; probes <= mask; ++probes) {
        const int32_t prev = atomicCAS(&key[p.h], EMPTY_KEY, C);
        if constexpr (SIG) if (prev == EMPTY_KEY) sig[p.h] = S;
        if (prev == EMPTY_KEY || prev == C) { atomicAdd(&val[p.h], W); return true; }
        probe_next<false>(p, mask);
    }
    return false;
}

// Aggregate the entries [e_beg, e_end) (stride STRIDE from the caller's lane)
// of vertex i into an LDS table, optionally only communities of partition
// `part` of P.  Returns false if the bounded table had no room (only
// possible with P > 1).
// ecm: EC_READ takes each entry's pair from the entry cache, EC_FILL gathers
// it and also stores it there, EC_GATHER gathers it.
template <int STRIDE, bool BOUNDED, bool SIG, int U = UNROLL, bool MOD = false>
__device__ __forceinline__ bool aggregate_entries(const MoveArgs& a, int32_t i, int32_t e_beg, int32_t e_end,
                                                  int32_t* key, int32_t* val, int32_t* sig, uint32_t mask, uint32_t P,
                                                  uint32_t part, int ecm)
{
    bool ok_all = true;
    for (int32_t e0 = e_beg; e0 < e_end; e0 += STRIDE * U) {
        int32_t ww[U];
        int2 cc[U];
        if (ecm == EC_READ) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t e = e0 + u * STRIDE;
                const bool ok = e < e_end;
                cc[u] = ok ? ce_load(a.ce, e) : make_int2(EMPTY_KEY, 0);
                ww[u] = (ok && a.w) ? __builtin_nontemporal_load(&a.w[e]) : 1;
            }
        } else {
            int32_t jj[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t e = e0 + u * STRIDE;
                const bool ok = e < e_end;
                jj[u] = ok ? __builtin_nontemporal_load(&a.idx[e]) : i;
                ww[u] = (ok && a.w) ? __builtin_nontemporal_load(&a.w[e]) : 1;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (SIG || ecm == EC_FILL) cc[u] = jj[u] != i ? a.cs[jj[u]] : make_int2(EMPTY_KEY, 0);
                else cc[u] = make_int2(jj[u] != i ? a.comm[jj[u]] : EMPTY_KEY, 0);
            }
            if (ecm == EC_FILL) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int32_t e = e0 + u * STRIDE;
                    if (e < e_end) ce_store(a.ce, e, cc[u]);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t C = cc[u].x;
            if (C == EMPTY_KEY) continue;
            if constexpr (BOUNDED) {
                if (P > 1 && part_of(C, P) != part) continue;
                if (!lds_insert_bounded<SIG>(key, val, sig, mask, C, ww[u], cc[u].y)) ok_all = false;
            } else {
                lds_insert<SIG, MOD>(key, val, sig, mask, C, ww[u], cc[u].y);
            }
        }
    }
    return ok_all;
}

// Aggregate bucket entries [t0, cnt) (stride STRIDE) into a bounded LDS table.
template <int STRIDE>
__device__ __forceinline__ bool aggregate_bucket(const int2* src, const int32_t* src_w, int32_t t0, int32_t cnt,
                                                 int32_t* key, int32_t* val, int32_t* sig, uint32_t mask)
{
    bool ok_all = true;
    for (int32_t b0 = t0; b0 < cnt; b0 += STRIDE * UNROLL) {
        int2 cc[UNROLL];
        int32_t ww[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int32_t t = b0 + u * STRIDE;
            const bool ok = t < cnt;
            cc[u] = ok ? src[t] : make_int2(EMPTY_KEY, 0);
            ww[u] = (ok && src_w) ? src_w[t] : 1;
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
            if (cc[u].x != EMPTY_KEY && !lds_insert_bounded<true>(key, val, sig, mask, cc[u].x, ww[u], cc[u].y))
                ok_all = false;
    }
    return ok_all;
}

// Scan a table's slots [t0, T) step STRIDE: own-community weight and best candidate.
template <int STRIDE, bool SIG>
__device__ __forceinline__ void scan_table(const MoveArgs& a, const int32_t* key, const int32_t* val,
                                           const int32_t* sig, uint32_t t0, uint32_t T, int32_t A, int64_t ki,
                                           int64_t M, int64_t& best_s, int32_t& best_c, int32_t& w_own)
{
    const bool louvain = a.mode == MODE_LOUVAIN;
    if constexpr (SIG) {
        for (uint32_t t = t0; t < T; t += STRIDE) {
            const int32_t C = key[t];
            if (C == EMPTY_KEY) continue;
            const int32_t W = val[t];
            if (C == A) { w_own = W; continue; }
            const int64_t s = louvain ? louvain_score(M, W, ki, sig[t]) : (int64_t)W;
            if (better(s, C, best_s, best_c)) { best_s = s; best_c = C; }
        }
    } else {
        // volumes gathered from global memory: issue SU gathers before using any
        constexpr int SU = 8;
        for (uint32_t tb = t0; tb < T; tb += STRIDE * SU) {
            int32_t Cs[SU], Ws[SU], Ss[SU];
#pragma unroll
            for (int u = 0; u < SU; ++u) {
                const uint32_t t = tb + u * STRIDE;
                Cs[u] = t < T ? key[t] : EMPTY_KEY;
                Ws[u] = t < T ? val[t] : 0;
            }
#pragma unroll
            for (int u = 0; u < SU; ++u) Ss[u] = (louvain && Cs[u] != EMPTY_KEY && Cs[u] != A) ? a.sigma[Cs[u]] : 0;
#pragma unroll
            for (int u = 0; u < SU; ++u) {
                if (Cs[u] == EMPTY_KEY) continue;
                if (Cs[u] == A) { w_own = Ws[u]; continue; }
                const int64_t s = louvain ? louvain_score(M, Ws[u], ki, Ss[u]) : (int64_t)Ws[u];
                if (better(s, Cs[u], best_s, best_c)) { best_s = s; best_c = Cs[u]; }
            }
        }
    }
}

// Pairs of the ME entries e_first + u*STRIDE (u < ME) of vertex i's row
// ending at e_end, by the sweep's entry mode (out of range or a loop: EMPTY_KEY).
template <int STRIDE, int ME>
__device__ __forceinline__ void load_pairs(const MoveArgs& a, int32_t i, int32_t e_first, int32_t e_end, int ecm,
                                           int2 (&cc)[ME], int32_t (&ww)[ME])
{
    if (ecm == EC_READ) {
#pragma unroll
        for (int u = 0; u < ME; ++u) {
            const int32_t e = e_first + u * STRIDE;
            const bool ok = e < e_end;
            cc[u] = ok ? ce_load(a.ce, e) : make_int2(EMPTY_KEY, 0);
            ww[u] = (ok && a.w) ? __builtin_nontemporal_load(&a.w[e]) : 1;
        }
        return;
    }
    int32_t jj[ME];
#pragma unroll
    for (int u = 0; u < ME; ++u) {
        const int32_t e = e_first + u * STRIDE;
        const bool ok = e < e_end;
        jj[u] = ok ? __builtin_nontemporal_load(&a.idx[e]) : i;
        ww[u] = (ok && a.w) ? __builtin_nontemporal_load(&a.w[e]) : 1;
    }
#pragma unroll
    for (int u = 0; u < ME; ++u) cc[u] = jj[u] != i ? a.cs[jj[u]] : make_int2(EMPTY_KEY, 0);
    if (ecm == EC_FILL) {
#pragma unroll
        for (int u = 0; u < ME; ++u) {
            const int32_t e = e_first + u * STRIDE;
            if (e < e_end) ce_store(a.ce, e, cc[u]);
        }
    }
}

// Claim-or-add of (C, W) in an LDS table of packed 64-bit slots (community
// in the high word, weight sum in the low word; EMPTY_SLOT when free) that
// has room for every key.  Returns the slot if this call claimed it (the
// claimer later scores the community), else -1 after adding W to the
// community's sum.  mask: slots - 1 (a power of two), or with MOD the slot
// count, hashed by a multiply-high reduction.
constexpr unsigned long long EMPTY_SLOT = 0xFFFFFFFF00000000ull;

template <bool MOD>
__device__ __forceinline__ int32_t claim_or_add(unsigned long long* tab, uint32_t mask, int32_t C, int32_t W)
{
    const unsigned long long mine = ((unsigned long long)(uint32_t)C << 32) | (uint32_t)W;
    Probe p = probe_start<MOD>(C, mask);
    // one exit test per probe (an empty slot or the key), the add after the
    // loop: the loop body stays free of nested branches
    unsigned long long prev;
    for (;;) {
        prev = atomicCAS(&tab[p.h], EMPTY_SLOT, mine);
        if (prev == EMPTY_SLOT || (int32_t)(prev >> 32) == C) break;
        probe_next<MOD>(p, mask);
    }
    if (prev == EMPTY_SLOT) return (int32_t)p.h;
    atomicAdd(&tab[p.h], (unsigned long long)(uint32_t)W);
    return -1;
}

// Kinds of the generic move kernel: the first sweep of a level (every
// community a single vertex: entries scored directly) and an asynchronous
// sweep (compact table; volumes read live at scan time).  Later synchronous
// sweeps run k_move_claim.
constexpr int MK_FIRST = 0, MK_ASYNC = 2;

// One group of G lanes per vertex (G <= BS); LDS table of up to SLOTS slots.
// (CLS only names the instantiation, so each degree class has its own kernel symbol)
template <int CLS, int BS, int G, int SLOTS, int KIND>
__global__ __launch_bounds__(BS) void k_move(MoveArgs a)
{
    constexpr int NG = BS / G;
    constexpr int TBL = KIND == MK_FIRST ? 1 : NG * SLOTS;
    constexpr bool ASYNC = KIND == MK_ASYNC;
    __shared__ int32_t s_key[ASYNC ? TBL : 1];
    __shared__ int32_t s_val[ASYNC ? TBL : 1];
    __shared__ int64_t rs[BS / WAVE];
    __shared__ int32_t rc[BS / WAVE], rw[BS / WAVE];

    if (a.ctl->all_done) return;
    const int g = threadIdx.x / G, lane = threadIdx.x % G;
    const int64_t vi = (int64_t)blockIdx.x * NG + g;
    const bool has = vi < a.nverts;
    const int4 row = has ? a.rows[vi] : make_int4(0, 0, 0, 0);
    const int32_t i = row.x;
    const bool live = has && !vertex_frozen(a, i) && !vertex_skipped(a, i);
    const int32_t beg = live ? row.y : 0, end = live ? row.z : 0;
    const int2 self = live ? (ASYNC ? make_int2(a.live_comm[i], 0) : a.cs[i]) : make_int2(0, 0);
    const int32_t A = self.x;
    const int64_t ki = live ? row.w : 0;
    const int64_t M = live ? vertex_M(a, i) : 0;
    int64_t best_s = INT64_MIN;
    int32_t best_c = INT32_MAX, w_own = 0;
    // a table of up to SLOTS slots sized to the row (a power of two when
    // SLOTS is one, else 2L + 1 with multiply-high hashing); SLOTS exceeds
    // every row of the class, so the table never fills
    constexpr bool POW2 = (SLOTS & (SLOTS - 1)) == 0;
    const uint32_t T = POW2 ? min((uint32_t)SLOTS, pow2_at_least(2u * (uint32_t)(end - beg)))
                            : min((uint32_t)SLOTS, 2u * (uint32_t)(end - beg) + 1u);

    if constexpr (KIND == MK_FIRST) {
        score_entries_singleton<G>(a, i, ki, M, beg + lane, end, best_s, best_c);
    } else {
        int32_t* key = s_key + g * SLOTS;
        int32_t* val = s_val + g * SLOTS;
        for (uint32_t t = lane; t < T; t += G) { key[t] = EMPTY_KEY; val[t] = 0; }
        group_sync<G>();
        aggregate_entries<G, false, false, (G >= 1024 ? 8 : UNROLL), !POW2>(a, i, beg + lane, end, key, val, key,
                                                                           POW2 ? T - 1u : T, 1u, 0u, EC_GATHER);
        group_sync<G>();
        scan_table<G, false>(a, key, val, key, lane, T, A, ki, M, best_s, best_c, w_own);
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
    bool moved = false;
    if (has && lane == 0) {
        if (!live) a.dec[vi] = -1;
        else if constexpr (ASYNC) moved = decide_apply(a, vi, i, A, ki, M, best_s, best_c, w_own);
        else decide_store(a, vi, A, self.y, ki, M, best_s, best_c, w_own);
    }
    if constexpr (ASYNC) block_flush_sums<BS, uint32_t>(a.gmoves, moved ? move_slot(a, i) : -1, moved ? 1u : 0u);
}

// Later synchronous sweeps: one group of G lanes per vertex (a block of BS
// threads holds BS/G groups; group g takes listed row vi_first + g if it is
// below vi_end), an LDS table of up to SLOTS packed slots per group at
// tab + g*SLOTS, each community scored by the lane that claimed its slot with
// the volume that came with the entry's pair (no scan of the table, no volume
// array).  rs/rc/rw: BS/64 entries for the reduction across wavefronts.
// Every thread of the block calls it with the same arguments.
template <int CLS, int BS, int G, int SLOTS>
__device__ __forceinline__ void claim_rows(const MoveArgs& a, int ecm, int64_t vi_first, int64_t vi_end,
                                           unsigned long long* s_tab, int64_t* rs, int32_t* rc, int32_t* rw)
{
    constexpr int ME = (CLS_CAP[CLS] + G - 1) / G;  // entries per lane (rows of the class have <= CLS_CAP entries)
    static_assert(ME >= 1 && ME <= 8, "entries per lane");
    constexpr bool POW2 = (SLOTS & (SLOTS - 1)) == 0;
    const int g = threadIdx.x / G, lane = threadIdx.x % G;
    const int64_t vi = vi_first + g;
    const bool has = vi < vi_end;
    const int4 row = has ? a.rows[vi] : make_int4(0, 0, 0, 0);
    const int32_t i = row.x;
    const bool live = has && !vertex_frozen(a, i) && !vertex_skipped(a, i);
    const int32_t beg = live ? row.y : 0, end = live ? row.z : 0;
    const int2 self = live ? a.cs[i] : make_int2(0, 0);
    const int32_t A = self.x;
    const int64_t ki = live ? row.w : 0;
    const int64_t M = live ? vertex_M(a, i) : 0;
    // a table of about L * table_pct / 100 + 1 slots, at least L + 1 (a power
    // of two when SLOTS is one), at most SLOTS, which exceeds every row of the
    // class: it never fills
    const uint32_t L = (uint32_t)(end - beg);
    const uint32_t want = max(L + 1u, (uint32_t)(((uint64_t)L * (uint32_t)a.table_pct) / 100u) + (POW2 ? 0u : 1u));
    const uint32_t T = POW2 ? min((uint32_t)SLOTS, pow2_at_least(want)) : min((uint32_t)SLOTS, want);
    unsigned long long* tab = s_tab + g * SLOTS;
    {  // cleared two slots a store: every group's table starts 16-byte aligned (SLOTS is even), and
       // ceil(T / 2) pairs stay within its SLOTS (T < SLOTS, or T == SLOTS and even)
        static_assert(SLOTS % 2 == 0, "claim tables are cleared in pairs of slots");
        ulonglong2* tab2 = reinterpret_cast<ulonglong2*>(tab);
        const ulonglong2 empty2 = make_ulonglong2(EMPTY_SLOT, EMPTY_SLOT);
        for (uint32_t t = lane; t < (T + 1u) / 2u; t += G) tab2[t] = empty2;
    }
    int2 cc[ME];
    int32_t ww[ME], slot[ME];
    load_pairs<G, ME>(a, i, beg + lane, end, ecm, cc, ww);
    group_sync<G>();
    // LPA gathers a row's entries into few labels once they spread: in a
    // group of a whole wavefront or more, the lanes holding the first lane's
    // label sum their weights and make one table add (Louvain's communities
    // at a vertex are mostly distinct, so it adds entry by entry)
    const bool merge = G >= WAVE && a.mode == MODE_LPA;
#pragma unroll
    for (int u = 0; u < ME; ++u) {
        const int32_t C = cc[u].x;
        if (merge) {
            const uint64_t live_m = __ballot(C != EMPTY_KEY);
            const int leader = live_m ? __ffsll((unsigned long long)live_m) - 1 : 0;
            const int32_t lk = __shfl(C, leader);
            const bool same = live_m && C != EMPTY_KEY && C == lk;
            int32_t sw = same ? ww[u] : 0;
#pragma unroll
            for (int d = WAVE / 2; d >= 1; d >>= 1) sw += __shfl_xor(sw, d);
            if (C == EMPTY_KEY) slot[u] = -1;
            else if (same) slot[u] = (int)lane_id() == leader ? claim_or_add<!POW2>(tab, POW2 ? T - 1u : T, C, sw) : -1;
            else slot[u] = claim_or_add<!POW2>(tab, POW2 ? T - 1u : T, C, ww[u]);
        } else {
            slot[u] = C == EMPTY_KEY ? -1 : claim_or_add<!POW2>(tab, POW2 ? T - 1u : T, C, ww[u]);
        }
    }
    group_sync<G>();
    const bool louvain = a.mode == MODE_LOUVAIN;
    int64_t best_s = INT64_MIN;
    int32_t best_c = INT32_MAX, w_own = 0;
#pragma unroll
    for (int u = 0; u < ME; ++u) {
        if (slot[u] < 0) continue;
        const int32_t W = (int32_t)(uint32_t)tab[slot[u]];
        const int32_t C = cc[u].x;
        if (C == A) { w_own = W; continue; }
        const int64_t sc = louvain ? louvain_score(M, W, ki, cc[u].y) : (int64_t)W;
        if (better(sc, C, best_s, best_c)) { best_s = sc; best_c = C; }
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
    if (has && lane == 0) {
        if (!live) a.dec[vi] = -1;
        else decide_store(a, vi, A, self.y, ki, M, best_s, best_c, w_own);
    }
}

template <int CLS, int BS, int G, int SLOTS>
__global__ __launch_bounds__(BS) void k_move_claim(MoveArgs a)
{
    __shared__ __align__(16) unsigned long long s_tab[(BS / G) * SLOTS];
    __shared__ int64_t rs[BS / WAVE];
    __shared__ int32_t rc[BS / WAVE], rw[BS / WAVE];
    if (a.ctl->all_done) return;
    claim_rows<CLS, BS, G, SLOTS>(a, entry_mode(a), (int64_t)blockIdx.x * (BS / G), a.nverts, s_tab, rs, rc, rw);
}

// Persistent fused sweep kernel (later synchronous sweeps, every class
// below the hub class in one launch).  Work items are blocks of rows of one
// class, numbered class by class (item_first[q] is class q's first);
// 1024-thread workgroups take FUSED_CHUNK items at a time from the counter
// ctl->work_next until none is left, each item laid out as its class's
// kernel lays out its block
// (BS/G groups of G lanes), with its tables carved from one LDS array sized
// for the largest class.  The counter is reset by k_sweep_end.
constexpr int FUSED_BS = 1024;
constexpr int FUSED_SLOTS = L8K_SLOTS;  // the largest (BS/G) * SLOTS of the classes at 1024 threads
constexpr int FUSED_CHUNK = 16;         // work items a workgroup takes per atomic
__global__ __launch_bounds__(FUSED_BS) void k_move_fused(MoveArgs a, FusedMap fm, SweepCtl* ctl)
{
    __shared__ __align__(16) unsigned long long s_tab[FUSED_SLOTS];
    __shared__ int64_t rs[FUSED_BS / WAVE];
    __shared__ int32_t rc[FUSED_BS / WAVE], rw[FUSED_BS / WAVE];
    __shared__ int32_t s_item;
    if (ctl->all_done) return;
    const int ecm = entry_mode(a);
    const int32_t total = fm.item_first[fm.nclass];
    int32_t item = 0, chunk_end = 0;
    for (;;) {
        if (item >= chunk_end) {  // take the next FUSED_CHUNK items
            __syncthreads();      // every thread has read s_item
            if (threadIdx.x == 0) s_item = atomicAdd(&ctl->work_next, FUSED_CHUNK);
            __syncthreads();
            item = s_item;
            chunk_end = item + FUSED_CHUNK;
        } else {
            __syncthreads();  // the previous item is done with the tables
        }
        if (item >= total) break;
        int q = 0;
        while (q + 1 < fm.nclass && fm.item_first[q + 1] <= item) ++q;
        const int32_t k = item - fm.item_first[q];
        const int64_t r0 = fm.row_first[q], r1 = fm.row_end[q];
#define LV_FUSED_CASE(C, G, SL)                                                                                    \
    case C:                                                                                                        \
        static_assert((FUSED_BS / G) * SL <= FUSED_SLOTS, "the fused kernel's LDS holds every class's tables");    \
        claim_rows<C, FUSED_BS, G, SL>(a, ecm, r0 + (int64_t)k * (FUSED_BS / G), r1, s_tab, rs, rc, rw);            \
        break;
        switch (fm.cls[q]) {
            LV_FUSED_CASE(CLS_L4, 4, L4_SLOTS)
            LV_FUSED_CASE(CLS_L8, 4, L8_SLOTS)
            LV_FUSED_CASE(CLS_L32, 8, L32_SLOTS)
            LV_FUSED_CASE(CLS_L128, 32, L128_SLOTS)
            LV_FUSED_CASE(CLS_L256, 64, L256_SLOTS)
            LV_FUSED_CASE(CLS_L512, 128, L512_SLOTS)
            LV_FUSED_CASE(CLS_L1K, 256, L1K_SLOTS)
            LV_FUSED_CASE(CLS_L2K, 512, L2K_SLOTS)
            LV_FUSED_CASE(CLS_L3K, 512, L3K_SLOTS)
            LV_FUSED_CASE(CLS_L8K, 1024, L8K_SLOTS)
            default: break;
        }
#undef LV_FUSED_CASE
        ++item;
    }
}

// Later synchronous sweeps of the class of at most ME = 4 entries: one
// lane per row and no table.  The lane holds its row's pairs in
// registers; entry u sums the weights of every entry of the row with its
// community, and the first entry of each community scores it.
constexpr int REG_BS = 256;
template <int CLS>
__global__ __launch_bounds__(REG_BS) void k_move_reg(MoveArgs a)
{
    constexpr int ME = CLS_CAP[CLS];
    static_assert(ME >= 1 && ME <= 4, "rows held in registers");
    if (a.ctl->all_done) return;
    const int64_t vi = (int64_t)blockIdx.x * REG_BS + threadIdx.x;
    if (vi >= a.nverts) return;
    const int4 row = a.rows[vi];
    const int32_t i = row.x;
    if (vertex_frozen(a, i) || vertex_skipped(a, i)) {
        a.dec[vi] = -1;
        return;
    }
    const int2 self = a.cs[i];
    const int32_t A = self.x;
    const int64_t ki = row.w;
    const int64_t M = vertex_M(a, i);
    int2 cc[ME];
    int32_t ww[ME];
    load_pairs<1, ME>(a, i, row.y, row.z, entry_mode(a), cc, ww);
    const bool louvain = a.mode == MODE_LOUVAIN;
    int64_t best_s = INT64_MIN;
    int32_t best_c = INT32_MAX, w_own = 0;
#pragma unroll
    for (int u = 0; u < ME; ++u) {
        const int32_t C = cc[u].x;
        bool first = C != EMPTY_KEY;
        int32_t W = 0;
#pragma unroll
        for (int v = 0; v < ME; ++v) {
            if (cc[v].x == C) W += ww[v];
            if (v < u && cc[v].x == C) first = false;
        }
        if (!first) continue;
        if (C == A) { w_own = W; continue; }
        const int64_t sc = louvain ? louvain_score(M, W, ki, cc[u].y) : (int64_t)W;
        if (better(sc, C, best_s, best_c)) { best_s = sc; best_c = C; }
    }
    decide_store(a, vi, A, self.y, ki, M, best_s, best_c, w_own);
}

template <int CLS, int BS, int G, int SLOTS>
hipError_t launch_move_t(bool singleton, bool async, const MoveArgs& a, hipStream_t s)
{
    static_assert(SLOTS > CLS_CAP[CLS], "a class's table must hold every distinct community of its longest row");
    if (a.nverts <= 0) return hipSuccess;
    constexpr int NG = BS / G;
    const unsigned grid = (unsigned)((a.nverts + NG - 1) / NG);
    if (async) k_move<CLS, BS, G, SLOTS, MK_ASYNC><<<grid, BS, 0, s>>>(a);
    else if (singleton) k_move<CLS, BS, G, SLOTS, MK_FIRST><<<grid, BS, 0, s>>>(a);
    else if constexpr (CLS_CAP[CLS] <= 4)  // the 8-entry class was slower this way on graphs of short rows
        k_move_reg<CLS><<<(unsigned)((a.nverts + REG_BS - 1) / REG_BS), REG_BS, 0, s>>>(a);
    else k_move_claim<CLS, BS, G, SLOTS><<<grid, BS, 0, s>>>(a);
    return hipGetLastError();
}

// ------------------------------------------------------------------ partitioned path (L > block_max)
constexpr int PBS = 1024;               // compact partition workgroups and the scatter pass
constexpr int PSLOTS_COMPACT = 16384;  // 8-byte slots (key, weight): 128 KiB
constexpr int BBS = 256;               // bucketed partition workgroups
constexpr int BSLOTS = 2048;           // 12-byte slots (key, weight, volume): 24 KiB, six workgroups a CU

// Workgroups are dispatched to the 8 XCDs round-robin; renumber them so that
// consecutive logical ids run on one XCD (and share its L2).
__device__ __forceinline__ int32_t xcd_logical(int32_t b, int32_t nblk)
{
    const int32_t x = b & 7, k = b >> 3, q = nblk >> 3, r = nblk & 7;
    return x * q + min(x, r) + k;
}

// One workgroup per (vertex, partition): aggregate the partition's
// communities in LDS (or, in the first sweep, score a contiguous 1/P of the
// entries directly) and write the partial best.
template <bool SINGLETON, bool SIG, int BS, int SLOTS>
__global__ __launch_bounds__(BS) void k_hub_part(MoveArgs a, HubArgs h)
{
    __shared__ int32_t s_key[SINGLETON ? 1 : SLOTS];
    __shared__ int32_t s_val[SINGLETON ? 1 : SLOTS];
    __shared__ int32_t s_sig[(SINGLETON || !SIG) ? 1 : SLOTS];
    __shared__ int64_t rs[BS / WAVE];
    __shared__ int32_t rc[BS / WAVE], rw[BS / WAVE];
    __shared__ int32_t s_over;
    if (a.ctl->all_done) return;
    const int32_t b = xcd_logical((int32_t)blockIdx.x, h.nblk);
    const int32_t hh = h.blk_hub[b];
    const uint32_t part = (uint32_t)h.blk_part[b], P = (uint32_t)h.hub_parts[hh];
    const int32_t i = h.hub_vert[hh];
    if (vertex_frozen(a, i) || vertex_skipped(a, i)) {
        if (threadIdx.x == 0) { h.part_score[b] = INT64_MIN; h.part_comm[b] = INT32_MAX; h.part_wown[b] = 0; h.part_flag[b] = 0; }
        return;
    }
    const int32_t beg = a.off[i], end = a.off[i + 1];
    const int32_t A = comm_now(a, i);
    const int64_t ki = a.k[i];
    const int64_t M = vertex_M(a, i);
    int64_t best_s = INT64_MIN;
    int32_t best_c = INT32_MAX, w_own = 0;
    int32_t over = 0;
    if constexpr (SINGLETON) {
        const int64_t L = end - beg;
        const int32_t cb = beg + (int32_t)(L * part / P), ce = beg + (int32_t)(L * (part + 1) / P);
        score_entries_singleton<BS>(a, i, ki, M, cb + (int32_t)threadIdx.x, ce, best_s, best_c);
    } else {
        const uint32_t T = h.part_mask + 1u;
        // bucketed: this partition's communities were scattered to its bucket;
        // a bucket offered more than it holds sends the vertex to the
        // global-table fallback
        const int32_t cnt = (SIG && h.bucketed && P > 1) ? h.bucket_cnt[b] : -1;
        for (uint32_t t = threadIdx.x; t < T; t += BS) { s_key[t] = EMPTY_KEY; s_val[t] = 0; }
        if (threadIdx.x == 0) s_over = 0;
        __syncthreads();
        if (cnt >= 0 && threadIdx.x == 0) h.bucket_cnt[b] = 0;  // every thread has read it
        bool ok;
        if (cnt > h.bucket_cap) {
            ok = false;
        } else if (cnt >= 0) {
            const size_t at = (size_t)b * (size_t)h.bucket_cap;
            ok = aggregate_bucket<BS>(h.bucket + at, h.bucket_w + at, (int32_t)threadIdx.x, cnt, s_key, s_val, s_sig,
                                      h.part_mask);
        } else {
            // every partition reads the whole row; partition 0 fills the cache
            const int ecm = entry_mode(a);
            ok = aggregate_entries<BS, true, SIG>(a, i, beg + (int32_t)threadIdx.x, end, s_key, s_val, s_sig,
                                                  h.part_mask, P, part,
                                                  (ecm == EC_FILL && part != 0) ? EC_GATHER : ecm);
        }
        if (!ok) s_over = 1;
        __syncthreads();
        over = s_over;
        if (!over) scan_table<BS, SIG>(a, s_key, s_val, s_sig, threadIdx.x, T, A, ki, M, best_s, best_c, w_own);
    }
    block_reduce_best<BS>(best_s, best_c, w_own, rs, rc, rw);
    if (threadIdx.x == 0) {
        h.part_score[b] = best_s;
        h.part_comm[b] = best_c;
        h.part_wown[b] = w_own;
        h.part_flag[b] = over;
    }
}

// As claim_or_add, but gives up (ok = false) after probing every slot.
__device__ __forceinline__ int32_t claim_or_add_bounded(unsigned long long* tab, uint32_t mask, int32_t C, int32_t W,
                                                        bool& ok)
{
    const unsigned long long mine = ((unsigned long long)(uint32_t)C << 32) | (uint32_t)W;
    Probe p = probe_start<false>(C, mask);  // a power-of-two table: odd stride, every slot within mask + 1 probes
    unsigned long long prev = 0;
    bool placed = false;
    for (uint32_t probes = 0; probes <= mask; ++probes) {
        prev = atomicCAS(&tab[p.h], EMPTY_SLOT, mine);
        placed = prev == EMPTY_SLOT || (int32_t)(prev >> 32) == C;
        if (placed) break;
        probe_next<false>(p, mask);
    }
    if (!placed) {
        ok = false;
        return -1;
    }
    if (prev == EMPTY_SLOT) return (int32_t)p.h;
    atomicAdd(&tab[p.h], (unsigned long long)(uint32_t)W);
    return -1;
}

// Later sweeps of the bucketed partition path: one workgroup per (hub,
// partition).  Its communities come from the partition's bucket (hubs with
// P > 1) or, for a hub of one partition, from the row itself; each is summed
// in a packed LDS table and scored by the thread that claimed its slot, with
// the volume that came with it.  A bucket offered more than it holds, or a
// table without room, sends the hub to the global-table fallback.
template <int BS, int SLOTS>
__global__ __launch_bounds__(BS) void k_hub_part_claim(MoveArgs a, HubArgs h)
{
    constexpr int ME = SLOTS / BS;  // records per thread: a bucket holds at most SLOTS, a row of one partition fewer
    __shared__ unsigned long long s_tab[SLOTS];
    __shared__ int64_t rs[BS / WAVE];
    __shared__ int32_t rc[BS / WAVE], rw[BS / WAVE];
    __shared__ int32_t s_over;
    if (a.ctl->all_done) return;
    const int32_t b = xcd_logical((int32_t)blockIdx.x, h.nblk);
    const int32_t hh = h.blk_hub[b];
    const uint32_t P = (uint32_t)h.hub_parts[hh];
    const int32_t i = h.hub_vert[hh];
    if (vertex_frozen(a, i) || vertex_skipped(a, i)) {
        if (threadIdx.x == 0) { h.part_score[b] = INT64_MIN; h.part_comm[b] = INT32_MAX; h.part_wown[b] = 0; h.part_flag[b] = 0; }
        return;
    }
    const int32_t A = a.cs[i].x;
    const int64_t ki = a.k[i];
    const int64_t M = vertex_M(a, i);
    const uint32_t T = h.part_mask + 1u;
    const int32_t cnt = P > 1 ? h.bucket_cnt[b] : -1;
    for (uint32_t t = threadIdx.x; t < T; t += BS) s_tab[t] = EMPTY_SLOT;
    if (threadIdx.x == 0) s_over = 0;
    int2 cc[ME];
    int32_t ww[ME], slot[ME];
    bool ok = cnt <= h.bucket_cap;
    if (cnt >= 0) {
        const size_t at = (size_t)b * (size_t)h.bucket_cap;
        const int32_t n = ok ? cnt : 0;
#pragma unroll
        for (int u = 0; u < ME; ++u) {
            const int32_t t = (int32_t)threadIdx.x + u * BS;
            cc[u] = t < n ? h.bucket[at + t] : make_int2(EMPTY_KEY, 0);
            ww[u] = t < n ? h.bucket_w[at + t] : 0;
        }
    } else {
        // one partition: the row has at most part_keys <= 3/4 SLOTS entries
        load_pairs<BS, ME>(a, i, a.off[i] + (int32_t)threadIdx.x, a.off[i + 1], entry_mode(a), cc, ww);
    }
    __syncthreads();
    if (cnt >= 0 && threadIdx.x == 0) h.bucket_cnt[b] = 0;  // every thread has read it
#pragma unroll
    for (int u = 0; u < ME; ++u)
        slot[u] = cc[u].x == EMPTY_KEY ? -1 : claim_or_add_bounded(s_tab, T - 1u, cc[u].x, ww[u], ok);
    if (!ok) s_over = 1;
    __syncthreads();
    const int32_t over = s_over;
    int64_t best_s = INT64_MIN;
    int32_t best_c = INT32_MAX, w_own = 0;
    if (!over) {
        const bool louvain = a.mode == MODE_LOUVAIN;
#pragma unroll
        for (int u = 0; u < ME; ++u) {
            if (slot[u] < 0) continue;
            const int32_t W = (int32_t)(uint32_t)s_tab[slot[u]];
            const int32_t C = cc[u].x;
            if (C == A) { w_own = W; continue; }
            const int64_t sc = louvain ? louvain_score(M, W, ki, cc[u].y) : (int64_t)W;
            if (better(sc, C, best_s, best_c)) { best_s = sc; best_c = C; }
        }
    }
    block_reduce_best<BS>(best_s, best_c, w_own, rs, rc, rw);
    if (threadIdx.x == 0) {
        h.part_score[b] = best_s;
        h.part_comm[b] = best_c;
        h.part_wown[b] = w_own;
        h.part_flag[b] = over;
    }
}

// One wavefront per hub: merge the partitions' partial results, decide.
__global__ __launch_bounds__(256) void k_hub_finalize(MoveArgs a, HubArgs h)
{
    if (a.ctl->all_done) return;
    const int64_t hh64 = (int64_t)blockIdx.x * (256 / WAVE) + threadIdx.x / WAVE;
    const bool has = hh64 < h.nhubs;
    const int32_t hh = has ? (int32_t)hh64 : 0;
    int64_t best_s = INT64_MIN;
    int32_t best_c = INT32_MAX, w_own = 0, i = 0, A = 0, sA = 0, flag = 0;
    int64_t ki = 0;
    if (has) {
        i = h.hub_vert[hh];
        const int2 self = pair_now(a, i);
        A = self.x;
        sA = self.y;
        ki = a.k[i];
        for (int32_t p = h.hub_first_blk[hh] + (int32_t)lane_id(); p < h.hub_first_blk[hh + 1]; p += WAVE) {
            if (better(h.part_score[p], h.part_comm[p], best_s, best_c)) { best_s = h.part_score[p]; best_c = h.part_comm[p]; }
            w_own = max(w_own, h.part_wown[p]);
            flag |= h.part_flag[p];
        }
    }
    group_reduce<WAVE>(best_s, best_c, w_own);
    const bool overflowed = __ballot(flag != 0) != 0;
    if (has && overflowed && lane_id() == 0) h.fb_flag[hh] = 1;
    if (has && !overflowed && lane_id() == 0) {
        if (a.live_comm) {
            if (decide_apply(a, hh, i, A, ki, vertex_M(a, i), best_s, best_c, w_own)) atomicAdd(&a.gmoves[move_slot(a, i)], 1u);
        } else {
            decide_store(a, hh, A, sA, ki, vertex_M(a, i), best_s, best_c, w_own);
        }
    }
}

// Scatter the entries of hubs with P > 1 into their partitions' buckets.  A
// workgroup takes a chunk of a row in NCH passes of SBS * EPT entries; each
// pass sums its entries per community in a packed LDS table (so a community
// shared by many neighbours costs one bucket entry per pass) and the thread
// that claimed a community's slot keeps (community, volume, weight sum) in
// registers.  After the last pass the workgroup takes its room in each
// partition's bucket with one atomic per partition and writes its records.
// Positions inside a bucket depend on timing; the sums a partition workgroup
// forms from them do not.
template <int SBS, int EPT, int NCH, int PMAX>
__global__ __launch_bounds__(SBS) void k_hub_scatter(MoveArgs a, HubArgs h)
{
    constexpr int SC_SLOTS = 2 * SBS * EPT;  // at most SBS * EPT keys a pass: always room
    constexpr int R = EPT * NCH;              // records a thread may hold
    __shared__ unsigned long long t_tab[SC_SLOTS];
    __shared__ int32_t s_cnt[PMAX];  // per-partition counts, then bucket bases (P <= PMAX)
    if (a.ctl->all_done) return;
    const int b = blockIdx.x;
    const int32_t hh = h.sc_hub[b];
    const int32_t i = h.hub_vert[hh];
    if (vertex_frozen(a, i) || vertex_skipped(a, i)) return;
    const uint32_t P = (uint32_t)h.hub_parts[hh];
    const int32_t c0 = h.sc_beg[b], c1 = h.sc_end[b];
    for (uint32_t t = threadIdx.x; t < P; t += SBS) s_cnt[t] = 0;
    const int ecm = entry_mode(a);
    int32_t ww[R], rk[R];
    uint32_t pp[R];
    int2 cc[R];
#pragma unroll
    for (int q = 0; q < NCH; ++q) {
        const int32_t e0 = c0 + q * SBS * EPT, e1 = c1;
        for (uint32_t t = threadIdx.x; t < (uint32_t)SC_SLOTS; t += SBS) t_tab[t] = EMPTY_SLOT;
        int32_t slot[EPT];
        if (ecm == EC_READ) {
#pragma unroll
            for (int u = 0; u < EPT; ++u) {
                const int32_t e = e0 + u * SBS + (int32_t)threadIdx.x;
                const bool ok = e < e1;
                cc[q * EPT + u] = ok ? ce_load(a.ce, e) : make_int2(EMPTY_KEY, 0);
                ww[q * EPT + u] = (ok && a.w) ? __builtin_nontemporal_load(&a.w[e]) : 1;
            }
        } else {
            int32_t jj[EPT];
#pragma unroll
            for (int u = 0; u < EPT; ++u) {
                const int32_t e = e0 + u * SBS + (int32_t)threadIdx.x;
                const bool ok = e < e1;
                jj[u] = ok ? __builtin_nontemporal_load(&a.idx[e]) : i;
                ww[q * EPT + u] = (ok && a.w) ? __builtin_nontemporal_load(&a.w[e]) : 1;
            }
#pragma unroll
            for (int u = 0; u < EPT; ++u) cc[q * EPT + u] = jj[u] != i ? pair_now(a, jj[u]) : make_int2(EMPTY_KEY, 0);
            if (ecm == EC_FILL) {
#pragma unroll
                for (int u = 0; u < EPT; ++u) {
                    const int32_t e = e0 + u * SBS + (int32_t)threadIdx.x;
                    if (e < e1) ce_store(a.ce, e, cc[q * EPT + u]);
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < EPT; ++u)
            slot[u] = cc[q * EPT + u].x == EMPTY_KEY ? -1
                                                     : claim_or_add<false>(t_tab, SC_SLOTS - 1, cc[q * EPT + u].x,
                                                                           ww[q * EPT + u]);
        __syncthreads();
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            const int r = q * EPT + u;
            rk[r] = -1;
            if (slot[u] < 0) continue;
            ww[r] = (int32_t)(uint32_t)t_tab[slot[u]];  // the community's weight sum in this pass
            pp[r] = part_of(cc[r].x, P);
            rk[r] = atomicAdd(&s_cnt[pp[r]], 1);
        }
        __syncthreads();  // the table is cleared by the next pass
    }
    int32_t* cnt = h.bucket_cnt + h.hub_first_blk[hh];
    for (uint32_t t = threadIdx.x; t < P; t += SBS) {
        const int32_t c = s_cnt[t];
        s_cnt[t] = c ? atomicAdd(&cnt[t], c) : 0;
    }
    __syncthreads();
    const size_t cap = (size_t)h.bucket_cap;
    const size_t first = (size_t)h.hub_first_blk[hh];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (rk[r] < 0) continue;
        const int32_t pos = s_cnt[pp[r]] + rk[r];
        if (pos >= h.bucket_cap) continue;  // the partition's workgroup flags the overflow
        const size_t at = (first + pp[r]) * cap + (size_t)pos;
        h.bucket[at] = cc[r];
        h.bucket_w[at] = ww[r];
    }
}

// ---- global-table fallback for hubs whose partition tables overflowed
constexpr int FBS = 256;

__global__ __launch_bounds__(FBS) void k_fb_insert(MoveArgs a, HubArgs h)
{
    if (a.ctl->all_done) return;
    const int b = blockIdx.x;
    const int32_t hh = h.ins_hub[b];
    if (!h.fb_flag[hh]) return;
    const int32_t i = h.hub_vert[hh];
    const uint32_t mask = (uint32_t)h.tab_cap[hh] - 1u;
    int32_t* tab = h.table + 2 * h.tab_off[hh];
    for (int32_t e = h.ins_beg[b] + threadIdx.x; e < h.ins_end[b]; e += FBS) {
        const int32_t j = a.idx[e];
        if (j == i) continue;
        const int32_t C = comm_now(a, j);
        const int32_t W = a.w ? a.w[e] : 1;
        uint32_t slot = mix32(C) & mask;
        for (;;) {
            const int32_t prev = atomicCAS(&tab[2 * slot], EMPTY_KEY, C);
            if (prev == EMPTY_KEY || prev == C) { atomicAdd(&tab[2 * slot + 1], W); break; }
            slot = (slot + 1) & mask;
        }
    }
}

__global__ __launch_bounds__(FBS) void k_fb_scan(MoveArgs a, HubArgs h)
{
    __shared__ int64_t rs[FBS / WAVE];
    __shared__ int32_t rc[FBS / WAVE], rw[FBS / WAVE];
    if (a.ctl->all_done) return;
    const int b = blockIdx.x;
    const int32_t hh = h.scan_hub[b];
    if (!h.fb_flag[hh]) return;
    const int32_t i = h.hub_vert[hh];
    const int32_t A = comm_now(a, i);
    const int64_t ki = a.k[i];
    const bool louvain = a.mode == MODE_LOUVAIN;
    int32_t* tab = h.table + 2 * h.tab_off[hh];
    int64_t best_s = INT64_MIN;
    int32_t best_c = INT32_MAX, w_own = 0;
    for (int32_t t = h.scan_beg[b] + threadIdx.x; t < h.scan_end[b]; t += FBS) {
        const int32_t C = tab[2 * t];
        if (C == EMPTY_KEY) continue;
        const int32_t W = tab[2 * t + 1];
        tab[2 * t] = EMPTY_KEY;
        tab[2 * t + 1] = 0;
        if (C == A) { w_own = W; continue; }
        const int64_t s = louvain ? louvain_score(vertex_M(a, i), W, ki, a.sigma[C]) : (int64_t)W;
        if (better(s, C, best_s, best_c)) { best_s = s; best_c = C; }
    }
    block_reduce_best<FBS>(best_s, best_c, w_own, rs, rc, rw);
    if (threadIdx.x == 0) { h.fpart_score[b] = best_s; h.fpart_comm[b] = best_c; h.fpart_wown[b] = w_own; }
}

__global__ __launch_bounds__(256) void k_fb_finalize(MoveArgs a, HubArgs h)
{
    if (a.ctl->all_done) return;
    const int64_t hh64 = (int64_t)blockIdx.x * (256 / WAVE) + threadIdx.x / WAVE;
    const bool has = hh64 < h.nhubs && h.fb_flag[hh64];
    const int32_t hh = has ? (int32_t)hh64 : 0;
    int64_t best_s = INT64_MIN;
    int32_t best_c = INT32_MAX, w_own = 0, i = 0, A = 0, sA = 0;
    int64_t ki = 0;
    if (has) {
        i = h.hub_vert[hh];
        const int2 self = pair_now(a, i);
        A = self.x;
        sA = self.y;
        ki = a.k[i];
        for (int32_t p = h.fpart_first[hh] + (int32_t)lane_id(); p < h.fpart_first[hh + 1]; p += WAVE) {
            if (better(h.fpart_score[p], h.fpart_comm[p], best_s, best_c)) { best_s = h.fpart_score[p]; best_c = h.fpart_comm[p]; }
            w_own = max(w_own, h.fpart_wown[p]);
        }
    }
    group_reduce<WAVE>(best_s, best_c, w_own);
    if (has && lane_id() == 0) {
        if (a.live_comm) {
            if (decide_apply(a, hh, i, A, ki, vertex_M(a, i), best_s, best_c, w_own)) atomicAdd(&a.gmoves[move_slot(a, i)], 1u);
        } else {
            decide_store(a, hh, A, sA, ki, vertex_M(a, i), best_s, best_c, w_own);
        }
        h.fb_flag[hh] = 0;
    }
}

// ------------------------------------------------------------------ pruning marks
// After the decisions of sweep s: mark[v] = s for every mover v and every
// neighbour of one.  One wavefront per 64 listed vertices walks its movers'
// rows one after another (rows below the hub class hold at most 8192 entries).
// mark[idx[e]] = s for e in [e0, e1), `step` lanes apart from this lane's
// first entry; four index loads are in flight before their stores.
__device__ __forceinline__ void mark_entries(const int32_t* __restrict__ idx, int32_t* __restrict__ mark, int32_t e0,
                                             int32_t e1, int32_t step, int32_t s)
{
    constexpr int U = 4;
    for (int32_t e = e0; e < e1; e += U * step) {
        int32_t j[U];
#pragma unroll
        for (int u = 0; u < U; ++u) j[u] = e + u * step < e1 ? __builtin_nontemporal_load(&idx[e + u * step]) : -1;
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (j[u] >= 0) mark[j[u]] = s;
    }
}

// After the decisions of sweep s: mark[v] = s for every mover v and every
// neighbour of one.  One wavefront per 64 listed vertices walks its movers'
// rows one after another (rows below the hub class hold at most 8192 entries).
__global__ __launch_bounds__(256) void k_mark_movers(const int4* __restrict__ rows, const int32_t* __restrict__ dec,
                                                     int32_t m, const int32_t* __restrict__ idx,
                                                     int32_t* __restrict__ mark, const SweepCtl* ctl)
{
    if (ctl->all_done) return;
    const int32_t s = ctl->sweep + 1;
    const int64_t w0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) / WAVE * WAVE;
    const int lane = (int)lane_id();
    const bool mover = w0 + lane < m && dec[w0 + lane] >= 0;
    uint64_t todo = __ballot(mover);
    while (todo) {
        const int b = __builtin_ctzll(todo);
        todo &= todo - 1;
        const int4 r = rows[w0 + b];
        if (lane == 0) mark[r.x] = s;
        mark_entries(idx, mark, r.y + lane, r.z, WAVE, s);
    }
}

// The same for the hubs: workgroup b marks one chunk of a moving hub's row.
__global__ __launch_bounds__(256) void k_hub_mark(MoveArgs a, HubArgs h, int32_t* __restrict__ mark)
{
    if (a.ctl->all_done) return;
    const int32_t hh = h.mk_hub[blockIdx.x];
    if (a.dec[hh] < 0) return;
    const int32_t s = a.ctl->sweep + 1;
    if (threadIdx.x == 0) mark[h.hub_vert[hh]] = s;
    mark_entries(a.idx, mark, h.mk_beg[blockIdx.x] + (int32_t)threadIdx.x, h.mk_end[blockIdx.x], 256, s);
}

// ------------------------------------------------------------------ commit (K7)
// Apply the decisions of the m listed vertices: labels and community
// volumes (LPA's modularity reads the volumes too).  Every mover adds its
// volume change for the community it leaves and the one it joins into the
// workgroup's LDS table (integer sums, so order is irrelevant; see
// peeled_apply); the table is added into the volumes once at the end, so a
// community that many movers leave or join costs one global atomic per
// workgroup.  A change that finds no table slot within APPLY_PROBE probes,
// or is for a community not yet in the table once it holds APPLY_FILL
// communities (a workgroup whose movers touch many communities gains nothing
// from more), is added globally at once.  The movers of graph g in this sweep
// are counted in gmoves[g * max_sweeps + sweep].
constexpr int APPLY_SLOTS = 4096;
constexpr int APPLY_PROBE = 16;
constexpr int APPLY_FILL = APPLY_SLOTS * 3 / 4;

__device__ __forceinline__ void apply_add(int32_t* key, int32_t* val, int32_t* fill, int32_t* sigma, int32_t C,
                                          int32_t d)
{
    // a community already in the table always adds there; a new one takes
    // a slot only while the table holds fewer than APPLY_FILL communities
    constexpr uint32_t AMASK = (uint32_t)(APPLY_SLOTS - 1);
    Probe pr = probe_start<false>(C, AMASK);
    for (int p = 0; p < APPLY_PROBE; ++p) {
        const int32_t k = *(volatile int32_t*)&key[pr.h];
        if (k == C) { atomicAdd(&val[pr.h], d); return; }
        if (k == EMPTY_KEY) {
            if (*(volatile int32_t*)fill >= APPLY_FILL) break;
            const int32_t prev = atomicCAS(&key[pr.h], EMPTY_KEY, C);
            if (prev == EMPTY_KEY) atomicAdd(fill, 1);
            if (prev == EMPTY_KEY || prev == C) { atomicAdd(&val[pr.h], d); return; }
        }
        probe_next<false>(pr, AMASK);
    }
    atomicAdd(&sigma[C], d);
}

// Add d to community C for every valid lane: the lanes that share the first
// valid lane's community are summed into one add (movers crowding into one
// large community), every other lane adds on its own (the LDS atomics sort
// out any further collisions).  Reached by all lanes of the wavefront.
__device__ __forceinline__ void peeled_apply(int32_t* key, int32_t* val, int32_t* fill, int32_t* sigma, int32_t C,
                                             int32_t d, bool valid)
{
    const uint64_t any = __ballot(valid);
    if (!any) return;
    const int leader = __ffsll((unsigned long long)any) - 1;
    const int32_t lc = __shfl(C, leader);
    const bool mine = valid && C == lc;
    int32_t c = mine ? d : 0;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) c += __shfl_xor(c, m);
    if ((int)lane_id() == leader && c) apply_add(key, val, fill, sigma, lc, c);
    if (valid && !mine && d) apply_add(key, val, fill, sigma, C, d);
}

// Commit of one synchronous sweep: every mover takes its new community, and
// (sigma not null) the community volumes follow.  LPA passes no volumes: its
// scores never read them, and they are summed once from the final labels
// (k_volumes).
__global__ __launch_bounds__(256) void k_apply(const int32_t* verts, const int32_t* dec, int32_t m, const int32_t* k,
                                               const int32_t* gid, int32_t* comm, int32_t* sigma, const SweepCtl* ctl,
                                               uint32_t* gmoves, int32_t max_sweeps)
{
    __shared__ int32_t t_key[APPLY_SLOTS];
    __shared__ int32_t t_val[APPLY_SLOTS];
    __shared__ int32_t t_fill;
    if (ctl->all_done) return;
    if (threadIdx.x == 0) t_fill = 0;
    for (int t = threadIdx.x; t < APPLY_SLOTS; t += 256) { t_key[t] = EMPTY_KEY; t_val[t] = 0; }
    __syncthreads();
    uint32_t* moves = gmoves + ctl->sweep;
    int64_t my_g = -1;  // this thread's running mover count, for graph my_g
    uint32_t my_n = 0;
    for (int64_t base = (int64_t)blockIdx.x * 256; base < m; base += (int64_t)gridDim.x * 256) {
        const int64_t t = base + threadIdx.x;
        const int32_t C = t < m ? dec[t] : -1;
        const bool valid = C >= 0;
        int32_t A = 0, kv = 0;
        if (valid) {
            const int32_t v = verts[t];
            A = comm[v];
            kv = k[v];
            const int64_t gv = gid ? (int64_t)gid[v] * max_sweeps : 0;
            if (gv != my_g) {
                if (my_n) atomicAdd(&moves[my_g], my_n);
                my_g = gv;
                my_n = 0;
            }
            ++my_n;
            comm[v] = C;
        }
        if (sigma && __ballot(valid)) {
            peeled_apply(t_key, t_val, &t_fill, sigma, C, kv, valid);
            peeled_apply(t_key, t_val, &t_fill, sigma, A, -kv, valid);
        }
    }
    __syncthreads();
    if (sigma)
        for (int t = threadIdx.x; t < APPLY_SLOTS; t += 256)
            if (t_key[t] != EMPTY_KEY && t_val[t] != 0) atomicAdd(&sigma[t_key[t]], t_val[t]);
    block_flush_sums<256, uint32_t>(moves, my_n ? my_g : -1, my_n);
}

// sigma[comm[v]] += k[v] over the listed vertices verts[0..m) (sigma cleared
// by the caller), summed per workgroup in the same LDS table as the commit.
__global__ __launch_bounds__(256) void k_volumes(const int32_t* verts, int32_t m, const int32_t* k,
                                                 const int32_t* comm, int32_t* sigma)
{
    __shared__ int32_t t_key[APPLY_SLOTS];
    __shared__ int32_t t_val[APPLY_SLOTS];
    __shared__ int32_t t_fill;
    if (threadIdx.x == 0) t_fill = 0;
    for (int t = threadIdx.x; t < APPLY_SLOTS; t += 256) { t_key[t] = EMPTY_KEY; t_val[t] = 0; }
    __syncthreads();
    for (int64_t base = (int64_t)blockIdx.x * 256; base < m; base += (int64_t)gridDim.x * 256) {
        const int64_t t = base + threadIdx.x;
        const bool valid = t < m;
        int32_t C = 0, kv = 0;
        if (valid) {
            const int32_t v = verts[t];
            C = comm[v];
            kv = k[v];
        }
        peeled_apply(t_key, t_val, &t_fill, sigma, C, kv, valid);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < APPLY_SLOTS; t += 256)
        if (t_key[t] != EMPTY_KEY && t_val[t] != 0) atomicAdd(&sigma[t_key[t]], t_val[t]);
}

// After sweep s (1-based): a running graph stops when s >= 2 and its last two
// sweeps moved at most theta vertices each, or when s == max_sweeps.  Sets
// all_done when no graph runs any more, so later sweeps' kernels exit early.
// With the entry cache (ec_read_max >= 0) it also chooses how the next sweep
// gets its pairs: from the cache if the cache holds this sweep's pairs and at
// most ec_read_max entries saw their pair change in this commit (the refresh
// that follows rewrites them), else by gathering, filling the cache on the way
// if at most ec_fill_max entries changed (a later sweep may then read it).
__global__ __launch_bounds__(256) void k_sweep_end(SweepCtl* ctl, int32_t G, int32_t* gdone, int32_t* gsweeps,
                                                   const uint32_t* gmoves, int32_t max_sweeps, int64_t theta,
                                                   int32_t consecutive, int64_t ec_read_max, int64_t ec_fill_max)
{
    __shared__ int32_t red[4];
    if (ctl->all_done) return;
    const int32_t s = ctl->sweep + 1;
    int32_t running = 0;
    for (int32_t g = threadIdx.x; g < G; g += 256) {
        if (gdone[g]) continue;
        const uint32_t* mv = gmoves + (int64_t)g * max_sweeps;
        bool quiet = s >= consecutive;
        for (int32_t q = 1; q <= consecutive && quiet; ++q) quiet = (int64_t)mv[s - q] <= theta;
        const bool stop = quiet || s >= max_sweeps;
        if (stop) { gdone[g] = 1; gsweeps[g] = s; } else ++running;
    }
    running = block_sum<256>(running, red);
    if (threadIdx.x == 0) {
        ctl->sweep = s;
        ctl->all_done = running == 0 ? 1 : 0;
        ctl->work_next = 0;
        if (ec_read_max >= 0) {
            ctl->ec_last = ctl->ec_mode;
            const unsigned long long chg = ctl->chg_entries;
            const bool filled = ctl->ec_mode != EC_GATHER;
            int32_t next = EC_GATHER;
            if (filled && chg <= (unsigned long long)ec_read_max) next = EC_READ;
            else if (chg <= (unsigned long long)ec_fill_max) next = EC_FILL;
            ctl->ec_mode = next;
            if (next == EC_READ && running > 0) {
                ctl->ec_reads += 1;
                ctl->refreshed += chg;
            }
            ctl->chg_entries = 0;
        }
    }
}

__global__ void k_ctl_init(SweepCtl* ctl, int32_t G, const int32_t* gactive, int32_t* gdone, int32_t* gsweeps,
                           uint32_t* gmoves, int32_t max_sweeps)
{
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = t0; t < (int64_t)G * max_sweeps; t += stride) gmoves[t] = 0;
    for (int64_t g = t0; g < G; g += stride) {
        gdone[g] = gactive && !gactive[g] ? 1 : 0;
        gsweeps[g] = 0;
    }
    if (t0 == 0) {
        ctl->sweep = 0;
        ctl->all_done = 0;
        ctl->ec_mode = EC_GATHER;
        ctl->ec_last = EC_GATHER;
        ctl->ec_reads = 0;
        ctl->work_next = 0;
        ctl->chg_entries = 0;
        ctl->refreshed = 0;
    }
}

// cs[v] = (comm[v], Sigma_tot(comm[v])): the pair a move kernel gathers per
// CSR entry, for the listed vertices (verts null: v < n).  Only vertices with
// entries need it: nobody gathers an isolated vertex's pair.
__global__ void k_pairs(int32_t n, const int32_t* verts, const int32_t* comm, const int32_t* sigma, int2* cs,
                        const SweepCtl* ctl)
{
    if (ctl && ctl->all_done) return;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = verts ? verts[t] : (int32_t)t;
        const int32_t c = comm[v];
        cs[v] = make_int2(c, sigma[c]);
    }
}

// As k_pairs over the listed vertices (class order), recording whether each
// slot's pair changed (LPA, whose scores ignore volumes: its label) and the
// entries of the changed rows.  Each 256-slot tile also lists its changed
// rows below the hub class, (row begin, length, new pair), at the tile's
// own place in `list`, with their number in cnt[tile]: the refresh reads
// only those.
// The vertex of slot t is verts[t]; its row bounds are read only if its
// pair changed.
__global__ __launch_bounds__(256) void k_pairs_changed(int32_t m, int32_t nonhub, const int32_t* __restrict__ verts,
                                                       const int32_t* __restrict__ off, const int32_t* comm,
                                                       const int32_t* sigma, int2* cs, uint8_t* chg, int4* list,
                                                       int32_t* cnt, int mode, SweepCtl* ctl)
{
    __shared__ unsigned long long red[4];
    __shared__ int32_t w_cnt[4];
    if (ctl->all_done) return;
    unsigned long long tot = 0;
    for (int64_t base = (int64_t)blockIdx.x * 256; base < m; base += (int64_t)gridDim.x * 256) {
        const int64_t t = base + threadIdx.x;
        bool ch = false;
        int4 rec = make_int4(0, 0, 0, 0);
        if (t < m) {
            const int32_t v = verts[t];
            const int32_t c = comm[v];
            const int2 nw = make_int2(c, sigma[c]);
            const int2 old = cs[v];
            const bool lab = nw.x != old.x, pair = lab || nw.y != old.y;
            if (pair) cs[v] = nw;
            ch = mode == MODE_LOUVAIN ? pair : lab;
            if (ch) {
                const int32_t b0 = off[v], b1 = off[v + 1];
                tot += (unsigned long long)(b1 - b0);
                rec = make_int4(b0, b1 - b0, nw.x, nw.y);
            }
            chg[t] = ch ? 1 : 0;
        }
        const bool listed = ch && t < nonhub;
        const uint64_t bal = __ballot(listed);
        const int wid = (int)(threadIdx.x / WAVE);
        if (lane_id() == 0) w_cnt[wid] = __popcll(bal);
        __syncthreads();
        int32_t at = 0;
        for (int w = 0; w < wid; ++w) at += w_cnt[w];
        const int64_t tile = base / 256;
        if (listed) list[base + at + (int32_t)lane_rank(bal)] = rec;
        if (threadIdx.x == 0) cnt[tile] = w_cnt[0] + w_cnt[1] + w_cnt[2] + w_cnt[3];
        __syncthreads();  // w_cnt is reused by the next tile
    }
    tot = block_sum<256>(tot, red);
    if (threadIdx.x == 0 && tot) atomicAdd(&ctl->chg_entries, tot);
}

constexpr int32_t REFRESH_GRID = 8192;  // four rounds of resident 256-thread workgroups

// Entry-cache refresh (only when the next sweep reads the cache): for every
// listed vertex v whose pair changed, rewrite the cache entry of each of its
// neighbours u that refers to v (the reverse of v's entry for u; a loop is
// its own reverse and keeps its empty entry).  A workgroup takes a tile's
// list of changed rows (k_pairs_changed), sums their lengths and spreads
// their entries over its lanes, so that no lane waits on an unchanged row.
__global__ __launch_bounds__(256) void k_cache_refresh(int32_t tiles, const int4* __restrict__ list,
                                                       const int32_t* __restrict__ cnt,
                                                       const int32_t* __restrict__ rev, int2* __restrict__ ce,
                                                       const SweepCtl* ctl)
{
    __shared__ int32_t s_off[257];
    __shared__ int4 s_row[256];
    __shared__ int32_t w_sum[4];
    if (ctl->all_done || ctl->ec_mode != EC_READ) return;
    for (int32_t tile = (int32_t)blockIdx.x; tile < tiles; tile += (int32_t)gridDim.x) {
        const int32_t c = cnt[tile];
        if (c == 0) continue;  // the same for every thread of the workgroup
        int32_t len = 0;
        if ((int32_t)threadIdx.x < c) {
            const int4 r = list[(int64_t)tile * 256 + threadIdx.x];
            s_row[threadIdx.x] = r;
            len = r.y;
        }
        // inclusive scan of the lengths: within each wavefront, then across the four
        int32_t x = len;
#pragma unroll
        for (int d = 1; d < WAVE; d <<= 1) {
            const int32_t y = __shfl_up(x, d);
            if ((int)lane_id() >= d) x += y;
        }
        const int wid = (int)(threadIdx.x / WAVE);
        if (lane_id() == WAVE - 1) w_sum[wid] = x;
        __syncthreads();
        for (int w = 0; w < wid; ++w) x += w_sum[w];
        s_off[threadIdx.x + 1] = x;
        if (threadIdx.x == 0) s_off[0] = 0;
        __syncthreads();
        const int32_t total = s_off[c];
        // RU entries a thread per round: their rows found, then all their
        // reverse-map loads in flight, then their writes
        constexpr int RU = 4;
        for (int32_t f0 = (int32_t)threadIdx.x; f0 < total; f0 += 256 * RU) {
            int32_t e[RU], re[RU];
            int2 pr[RU];
#pragma unroll
            for (int u = 0; u < RU; ++u) {
                const int32_t f = f0 + u * 256;
                e[u] = -1;
                if (f >= total) continue;
                int32_t lo = 0, hi = c - 1;  // the row q with s_off[q] <= f < s_off[q + 1]
                while (lo < hi) {
                    const int32_t mid = (lo + hi + 1) >> 1;
                    if (s_off[mid] <= f) lo = mid; else hi = mid - 1;
                }
                const int4 r = s_row[lo];
                e[u] = r.x + (f - s_off[lo]);
                pr[u] = make_int2(r.z, r.w);
            }
#pragma unroll
            for (int u = 0; u < RU; ++u) re[u] = e[u] >= 0 ? __builtin_nontemporal_load(&rev[e[u]]) : -1;
#pragma unroll
            for (int u = 0; u < RU; ++u)
                if (e[u] >= 0 && re[u] != e[u]) ce[re[u]] = pr[u];
        }
        __syncthreads();  // s_row and s_off are reused by the next tile
    }
}

// The same for the hubs: workgroup b takes one 4096-entry chunk of a hub's row.
__global__ __launch_bounds__(256) void k_hub_cache_refresh(MoveArgs a, HubArgs h, const uint8_t* chg_hub,
                                                           const int32_t* __restrict__ rev)
{
    if (a.ctl->all_done || a.ctl->ec_mode != EC_READ) return;
    const int32_t hh = h.mk_hub[blockIdx.x];
    if (!chg_hub[hh]) return;
    const int32_t v = h.hub_vert[hh];
    const int2 p = a.cs[v];
    for (int32_t e = h.mk_beg[blockIdx.x] + (int32_t)threadIdx.x; e < h.mk_end[blockIdx.x]; e += 256) {
        const int32_t re = __builtin_nontemporal_load(&rev[e]);
        if (re != e) a.ce[re] = p;
    }
}

}  // namespace

hipError_t launch_pairs_changed(int32_t m, int32_t nonhub, const int32_t* verts, const int32_t* off,
                                const int32_t* comm, const int32_t* sigma, int2* cs, uint8_t* chg, int4* list,
                                int32_t* cnt, int mode, SweepCtl* ctl, hipStream_t s)
{
    if (m <= 0) return hipSuccess;
    k_pairs_changed<<<grid_for(m, 256, 8192), 256, 0, s>>>(m, nonhub, verts, off, comm, sigma, cs, chg, list, cnt,
                                                           mode, ctl);
    return hipGetLastError();
}
hipError_t launch_cache_refresh(int32_t m, const int4* list, const int32_t* cnt, const int32_t* rev, int2* ce,
                                SweepCtl* ctl, hipStream_t s)
{
    const int32_t tiles = (int32_t)(((int64_t)m + 255) / 256);
    if (tiles <= 0) return hipSuccess;
    k_cache_refresh<<<(unsigned)std::min(tiles, REFRESH_GRID), 256, 0, s>>>(tiles, list, cnt, rev, ce, ctl);
    return hipGetLastError();
}
hipError_t launch_hub_cache_refresh(const MoveArgs& a, const HubArgs& h, const uint8_t* chg_hub, const int32_t* rev,
                                    hipStream_t s)
{
    if (h.nmk <= 0) return hipSuccess;
    k_hub_cache_refresh<<<(unsigned)h.nmk, 256, 0, s>>>(a, h, chg_hub, rev);
    return hipGetLastError();
}

hipError_t launch_mark_movers(const int4* rows, const int32_t* dec, int32_t m, const int32_t* idx, int32_t* mark,
                              const SweepCtl* ctl, hipStream_t s)
{
    if (m <= 0) return hipSuccess;
    k_mark_movers<<<(unsigned)(((int64_t)m + 255) / 256), 256, 0, s>>>(rows, dec, m, idx, mark, ctl);
    return hipGetLastError();
}

hipError_t launch_hub_mark(const MoveArgs& a, const HubArgs& h, int32_t* mark, hipStream_t s)
{
    if (h.nmk <= 0) return hipSuccess;
    k_hub_mark<<<(unsigned)h.nmk, 256, 0, s>>>(a, h, mark);
    return hipGetLastError();
}

hipError_t launch_pairs(int32_t n, const int32_t* verts, const int32_t* comm, const int32_t* sigma, int2* cs,
                        const SweepCtl* ctl, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_pairs<<<LV_GRID(n)>>>(n, verts, comm, sigma, cs, ctl);
    return hipGetLastError();
}
hipError_t launch_ctl_init(SweepCtl* ctl, int32_t G, const int32_t* gactive, int32_t* gdone, int32_t* gsweeps,
                           uint32_t* gmoves, int32_t max_sweeps, hipStream_t s)
{
    k_ctl_init<<<grid_for((int64_t)G * max_sweeps + 1, 256, 4096), 256, 0, s>>>(ctl, G, gactive, gdone, gsweeps,
                                                                             gmoves, max_sweeps);
    return hipGetLastError();
}
hipError_t launch_sweep_end(SweepCtl* ctl, int32_t G, int32_t* gdone, int32_t* gsweeps, const uint32_t* gmoves,
                            int32_t max_sweeps, int64_t theta, int32_t consecutive, int64_t ec_read_max,
                            int64_t ec_fill_max, hipStream_t s)
{
    k_sweep_end<<<1, 256, 0, s>>>(ctl, G, gdone, gsweeps, gmoves, max_sweeps, theta, consecutive, ec_read_max,
                                  ec_fill_max);
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
hipError_t launch_class_starts(const uint32_t* cls_sorted, int32_t n, int32_t* start, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_class_starts<<<LV_GRID(n)>>>(cls_sorted, n, start);
    return hipGetLastError();
}
hipError_t launch_class_entries(const int32_t* verts_sorted, const int32_t* start, const int32_t* off, int64_t* out,
                                hipStream_t s)
{
    for (int c = CLS_L4; c < NUM_CLS; ++c) {
        const int32_t lo = start[c], hi = start[c + 1];
        if (hi <= lo) continue;
        k_class_entries<<<grid_for(hi - lo, 256, 4096), 256, 0, s>>>(verts_sorted, lo, hi, off,
                                                                     (unsigned long long*)(out + c));
    }
    return hipGetLastError();
}
hipError_t launch_row_descriptors(const int32_t* verts, int32_t m, const int32_t* off, const int32_t* k, int4* rows,
                                  hipStream_t s)
{
    if (m <= 0) return hipSuccess;
    k_row_descriptors<<<LV_GRID(m)>>>(verts, m, off, k, rows);
    return hipGetLastError();
}
hipError_t launch_gather_rows(const int32_t* verts, int32_t m, const int32_t* off, int32_t* beg, int32_t* len,
                              hipStream_t s)
{
    if (m <= 0) return hipSuccess;
    k_gather_rows<<<LV_GRID(m)>>>(verts, m, off, beg, len);
    return hipGetLastError();
}

hipError_t launch_move_fused(const MoveArgs& a, const FusedMap& fm, SweepCtl* ctl, hipStream_t s)
{
    if (fm.nclass <= 0 || fm.item_first[fm.nclass] <= 0) return hipSuccess;
    // two workgroups fit a CU (LDS of the largest class's table)
    const int32_t items = fm.item_first[fm.nclass];
    k_move_fused<<<(unsigned)(items < 512 ? items : 512), FUSED_BS, 0, s>>>(a, fm, ctl);
    return hipGetLastError();
}

hipError_t launch_move_class(int cls, bool singleton, bool async, const MoveArgs& a, hipStream_t s)
{
    switch (cls) {
    case CLS_L4: return launch_move_t<CLS_L4, 256, 4, L4_SLOTS>(singleton, async, a, s);
    case CLS_L8: return launch_move_t<CLS_L8, 256, 4, L8_SLOTS>(singleton, async, a, s);
    case CLS_L32: return launch_move_t<CLS_L32, 256, 8, L32_SLOTS>(singleton, async, a, s);
    case CLS_L128: return launch_move_t<CLS_L128, 256, 32, L128_SLOTS>(singleton, async, a, s);
    case CLS_L256: return launch_move_t<CLS_L256, 256, 64, L256_SLOTS>(singleton, async, a, s);
    case CLS_L512: return launch_move_t<CLS_L512, 256, 128, L512_SLOTS>(singleton, async, a, s);
    case CLS_L1K: return launch_move_t<CLS_L1K, 256, 256, L1K_SLOTS>(singleton, async, a, s);
    case CLS_L2K: return launch_move_t<CLS_L2K, 512, 512, L2K_SLOTS>(singleton, async, a, s);
    case CLS_L3K: return launch_move_t<CLS_L3K, 512, 512, L3K_SLOTS>(singleton, async, a, s);
    case CLS_L8K: return launch_move_t<CLS_L8K, 1024, 1024, L8K_SLOTS>(singleton, async, a, s);
    default: return hipErrorInvalidValue;
    }
}

// Expands per-hub workgroup counts into a per-workgroup list: workgroup b
// (of first[nhubs]) belongs to the hub h with first[h] <= b < first[h+1] (the
// last such h: hubs without workgroups have first[h] == first[h+1]) and is
// its chunk k = b - first[h], covering [base[h] + k*chunk, min(base[h] +
// (k+1)*chunk, base[h] + len[h])) (base null: 0).  o_end may be null.
__global__ __launch_bounds__(256) void k_chunk_list(const int32_t* __restrict__ first, int32_t nhubs, int32_t total,
                                                    const int32_t* __restrict__ base, const int32_t* __restrict__ len,
                                                    int32_t chunk, int32_t* __restrict__ o_hub,
                                                    int32_t* __restrict__ o_beg, int32_t* __restrict__ o_end)
{
    const int32_t b = (int32_t)(blockIdx.x * 256 + threadIdx.x);
    if (b >= total) return;
    int32_t lo = 0, hi = nhubs - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (first[mid] <= b) lo = mid; else hi = mid - 1;
    }
    const int64_t b0 = base ? (int64_t)base[lo] : 0;
    const int64_t e0 = b0 + (int64_t)(b - first[lo]) * chunk;
    o_hub[b] = lo;
    o_beg[b] = (int32_t)e0;
    if (o_end) o_end[b] = (int32_t)min(e0 + chunk, b0 + (int64_t)len[lo]);
}
hipError_t launch_chunk_list(const int32_t* first, int32_t nhubs, int32_t total, const int32_t* base,
                             const int32_t* len, int32_t chunk, int32_t* o_hub, int32_t* o_beg, int32_t* o_end,
                             hipStream_t s)
{
    if (total <= 0 || nhubs <= 0) return hipSuccess;
    k_chunk_list<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(first, nhubs, total, base, len, chunk, o_hub, o_beg,
                                                                  o_end);
    return hipGetLastError();
}

__global__ void k_hub_clear(int32_t* table, int64_t slots)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < slots; t += (int64_t)gridDim.x * blockDim.x) {
        table[2 * t] = EMPTY_KEY;
        table[2 * t + 1] = 0;
    }
}
hipError_t launch_hub_clear(int32_t* table, int64_t slots, hipStream_t s)
{
    if (slots <= 0) return hipSuccess;
    k_hub_clear<<<LV_GRID(slots)>>>(table, slots);
    return hipGetLastError();
}

hipError_t launch_hub_scatter(const MoveArgs& a, const HubArgs& h, hipStream_t s)
{
    if (h.nhubs <= 0 || !h.bucketed || h.nsc <= 0) return hipSuccess;
    // hubs of at most HUB_PSMALL partitions: a 4 KiB count array, so that
    // eight workgroups fit a CU's LDS instead of five
    const bool small = h.max_parts <= HUB_PSMALL;
    if (h.sc_chunk == 1024) {
        if (small) k_hub_scatter<256, 4, 1, HUB_PSMALL><<<(unsigned)h.nsc, 256, 0, s>>>(a, h);
        else k_hub_scatter<256, 4, 1, HUB_PMAX><<<(unsigned)h.nsc, 256, 0, s>>>(a, h);
    } else if (h.sc_chunk == 2048) {
        if (small) k_hub_scatter<256, 4, 2, HUB_PSMALL><<<(unsigned)h.nsc, 256, 0, s>>>(a, h);
        else k_hub_scatter<256, 4, 2, HUB_PMAX><<<(unsigned)h.nsc, 256, 0, s>>>(a, h);
    } else {
        if (small) k_hub_scatter<256, 4, 4, HUB_PSMALL><<<(unsigned)h.nsc, 256, 0, s>>>(a, h);
        else k_hub_scatter<256, 4, 4, HUB_PMAX><<<(unsigned)h.nsc, 256, 0, s>>>(a, h);
    }
    return hipGetLastError();
}

hipError_t launch_hub_sweep(bool singleton, const MoveArgs& a, const HubArgs& h, hipStream_t s)
{
    if (h.nhubs <= 0) return hipSuccess;
    if (h.bucketed) {
        if (singleton) k_hub_part<true, false, BBS, 1><<<(unsigned)h.nblk, BBS, 0, s>>>(a, h);
        else if (!a.live_comm) k_hub_part_claim<BBS, BSLOTS><<<(unsigned)h.nblk, BBS, 0, s>>>(a, h);
        else k_hub_part<false, true, BBS, BSLOTS><<<(unsigned)h.nblk, BBS, 0, s>>>(a, h);
    } else if (singleton) {
        k_hub_part<true, false, PBS, 1><<<(unsigned)h.nblk, PBS, 0, s>>>(a, h);
    } else {
        k_hub_part<false, false, PBS, PSLOTS_COMPACT><<<(unsigned)h.nblk, PBS, 0, s>>>(a, h);
    }
    const unsigned fin = (unsigned)((h.nhubs + 3) / 4);
    k_hub_finalize<<<fin, 256, 0, s>>>(a, h);
    if (!singleton && h.nins > 0) {
        k_fb_insert<<<(unsigned)h.nins, FBS, 0, s>>>(a, h);
        k_fb_scan<<<(unsigned)h.nscan, FBS, 0, s>>>(a, h);
        k_fb_finalize<<<fin, 256, 0, s>>>(a, h);
    }
    return hipGetLastError();
}

hipError_t launch_apply(const int32_t* verts, const int32_t* dec, int32_t m, const int32_t* k, const int32_t* gid,
                        int32_t* comm, int32_t* sigma, const SweepCtl* ctl, uint32_t* gmoves, int32_t max_sweeps,
                        hipStream_t s)
{
    if (m <= 0) return hipSuccess;
    k_apply<<<grid_for(m, 256, 2048), 256, 0, s>>>(verts, dec, m, k, gid, comm, sigma, ctl, gmoves, max_sweeps);
    return hipGetLastError();
}
hipError_t launch_volumes(const int32_t* verts, int32_t m, const int32_t* k, const int32_t* comm, int32_t* sigma,
                          hipStream_t s)
{
    if (m <= 0) return hipSuccess;
    k_volumes<<<grid_for(m, 256, 2048), 256, 0, s>>>(verts, m, k, comm, sigma);
    return hipGetLastError();
}

}  // namespace lv
