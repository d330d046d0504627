// Internal declarations shared by the kernel and host translation units of
// the Louvain library.  Everything here is gfx950 / HIP only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lv {

constexpr int32_t EMPTY_KEY = -1;
constexpr int MODE_LOUVAIN = 0;
constexpr int MODE_LPA = 1;
constexpr int DIR_DOWN = 0;
constexpr int DIR_UP = 1;

// Degree classes of the move step.  A vertex with L CSR entries goes to the
// first class whose bound is >= L (L = 0 never moves and is skipped).
enum MoveClass : int {
    CLS_NONE = 0,  // isolated
    CLS_L4,        // L <= 4:     first sweep 4 lanes per vertex; later sweeps one lane, no table
    CLS_L8,        // L <= 8:     4 lanes
    CLS_L32,       // L <= 32:    8 lanes
    CLS_L128,      // L <= 128:   32 lanes
    CLS_L256,      // L <= 256:   one wavefront
    CLS_L512,      // L <= 512:   128 lanes
    CLS_L1K,       // L <= 1024:  one 256-thread workgroup
    CLS_L2K,       // L <= 2048:  one 512-thread workgroup
    CLS_L3K,       // L <= 3072:  one 512-thread workgroup
    CLS_L8K,       // L <= 8192:  one 1024-thread workgroup (two workgroups a CU)
    CLS_HUB,       // several partition workgroups per vertex
    NUM_CLS
};

// row-length caps of the classes (a vertex takes the first class whose cap is
// at least its number of entries L)
constexpr int32_t CLS_CAP[NUM_CLS] = {0, 4, 8, 32, 128, 256, 512, 1024, 2048, 3072, 8192, INT32_MAX};
// classes of groups narrower than a wavefront, of one wavefront, of workgroups
constexpr int CLS_FIRST_WAVE = CLS_L256, CLS_FIRST_BLOCK = CLS_L512;
// Claim-table slots per row of each class (8-byte slots: key and weight
// sum), sized so that a CU still holds eight wavefronts a SIMD: at most
// 20 KiB of tables per 256-thread workgroup, 40 KiB per 512-thread one,
// 80 KiB per 1024-thread one (two workgroups of the 8192-entry class share a
// CU's 160 KiB).  Every class's table exceeds its longest row.
constexpr int32_t L4_SLOTS = 16, L8_SLOTS = 32, L32_SLOTS = 64, L128_SLOTS = 312, L256_SLOTS = 624,
                  L512_SLOTS = 1248, L1K_SLOTS = 2496, L2K_SLOTS = 5056, L3K_SLOTS = 5056;
constexpr int32_t L8K_SLOTS = 10112;

// Device-side sweep control of one level: completed sweeps and whether every
// graph of the level has stopped (kernels of later sweeps then exit early).
struct SweepCtl {
    int32_t sweep;
    int32_t all_done;
    // Entry cache (see MoveArgs::ce): how the current sweep's move kernels
    // get each entry's (community, volume) pair: EC_GATHER from cs[idx[e]],
    // EC_FILL the same and also storing it into ce[e], EC_READ from ce[e].
    int32_t ec_mode;
    int32_t ec_reads;                 // sweeps of this level that read the cache
    unsigned long long chg_entries;   // entries whose pair the last commit changed
    unsigned long long refreshed;     // entries rewritten by cache refreshes this level
    int32_t work_next;                // next work item of the fused sweep kernel
    int32_t ec_last;                  // how the last completed sweep got its pairs
};
constexpr int32_t EC_GATHER = 0, EC_FILL = 1, EC_READ = 2;

// Arguments shared by every move kernel.
struct MoveArgs {
    const int32_t* off;
    const int32_t* idx;
    const int32_t* w;       // null = unit weights
    const int32_t* k;       // weighted degree, < 2^31
    const int32_t* comm;    // labels of the previous sweep
    const int32_t* sigma;   // community volumes of the previous sweep, < 2^31
    const int2* cs;         // per vertex (comm[v], sigma[comm[v]]) of the previous sweep
    int64_t M;              // total volume (one graph)
    const int64_t* Mg;      // per-graph total volume when several graphs are packed (else null)
    const int32_t* gid;     // graph of each vertex (null for one graph)
    const int32_t* gdone;   // per graph: 1 = stopped for the rest of this level
    const SweepCtl* ctl;    // sweep counter / early exit
    const int32_t* verts;   // vertices of this class
    const int4* rows;       // per listed vertex: (vertex, row begin, row end, degree)
    int32_t nverts;
    int32_t mode;           // MODE_LOUVAIN / MODE_LPA
    int32_t* dec;           // decision per listed vertex: target community or -1
    const int32_t* mark;    // active-vertex pruning: per vertex, the last sweep in which it or a
                            // neighbour changed community (null: every vertex is evaluated)
    int32_t prune_back;     // pruning looks this many sweeps back (2 synchronous, 1 asynchronous)
    // asynchronous mode (null: synchronous): labels and community volumes read
    // and updated in place during the sweep; moves counted into
    // gmoves[graph * max_sweeps + sweep]
    int32_t* live_comm;
    int32_t* live_sigma;
    uint32_t* gmoves;
    int32_t max_sweeps;
    // Entry cache (null: off).  ce[e] holds the (community, volume) pair of
    // entry e's neighbour as of the previous sweep ((EMPTY_KEY, 0) for a loop
    // entry), so a sweep that reads it streams 8 bytes per entry instead of
    // gathering cs[idx[e]] at random.  Kept current by rewriting, after every
    // commit, the entries that point at a vertex whose pair changed (through
    // the reverse-entry map).
    int2* ce;
    int32_t table_pct;      // later sweeps' LDS table: about L * table_pct / 100 + 1 slots for L entries
};

// One segment of a packed CSR rebuild (see launch_repack).
struct RepackSeg {
    const int32_t* src_off;
    const int32_t* src_idx;
    const int32_t* src_w;   // null = unit weights
    const int32_t* src_k;
    const int32_t* src_orig; // vertex id of each source position (null: the position)
    int32_t src_vb;         // first source vertex
    int32_t n;              // vertices
    int32_t dst_vb;         // first destination vertex
    int32_t pad;
    int64_t dst_eb;         // first destination entry
};

// Vertices above the workgroup classes: P partitions per vertex, each a
// 1024-thread workgroup with an LDS table; a global-table fallback per vertex
// for partitions that overflow.  Layout built on the host once per level.
struct HubArgs {
    int32_t nhubs;
    uint32_t part_mask;            // LDS slots of a partition workgroup - 1
    int32_t bucketed;              // 1: partition tables with volumes, fed from per-partition buckets
    const int32_t* hub_vert;       // [nhubs]
    const int32_t* hub_parts;      // [nhubs] P
    const int32_t* hub_first_blk;  // [nhubs+1] first partition workgroup of each hub
    const int32_t* blk_hub;        // [nblk]
    const int32_t* blk_part;       // [nblk]
    int32_t nblk;
    int64_t* part_score;           // [nblk] partial results
    int32_t* part_comm;
    int32_t* part_wown;
    int32_t* part_flag;            // 1 = the partition's table overflowed
    int32_t* fb_flag;              // [nhubs] hub needs the global-table fallback
    // buckets (bucketed mode, hubs with P > 1): bucket b belongs to partition
    // workgroup b and holds up to bucket_cap (community, volume) pairs with
    // their weight sums, per chunk of the hub's row, of the communities in
    // that partition; bucket_cnt[b] counts the pairs offered (more than
    // bucket_cap: the hub takes the global-table fallback)
    int32_t bucket_cap;
    int32_t* bucket_cnt;           // [nblk], zero between sweeps
    int2* bucket;                  // [nblk * bucket_cap]
    int32_t* bucket_w;             // [nblk * bucket_cap] weight sums
    int32_t sc_chunk;              // entries per scatter workgroup: 1024, 2048 or 4096
    int32_t max_parts;             // the largest P among the hubs the scatter pass takes
    const int32_t* sc_hub;         // scatter workgroup b: entries [sc_beg, sc_end) of hub sc_hub
    const int32_t* sc_beg;
    const int32_t* sc_end;
    int32_t nsc;
    const int32_t* mk_hub;         // pruning marks, workgroup b: entries [mk_beg, mk_end) of hub mk_hub
    const int32_t* mk_beg;
    const int32_t* mk_end;
    int32_t nmk;
    // fallback: global open-addressing tables (2 ints per slot: key, value)
    const int64_t* tab_off;        // [nhubs] slot offset of the hub's table
    const int32_t* tab_cap;        // [nhubs] slots (power of two, 0 if P == 1)
    int32_t* table;
    const int32_t* ins_hub;        // insert workgroup b: entries [ins_beg, ins_end) of hub ins_hub
    const int32_t* ins_beg;
    const int32_t* ins_end;
    int32_t nins;
    const int32_t* scan_hub;       // scan workgroup b: slots [scan_beg, scan_end) of hub scan_hub
    const int32_t* scan_beg;
    const int32_t* scan_end;
    int32_t nscan;
    int64_t* fpart_score;          // [nscan]
    int32_t* fpart_comm;
    int32_t* fpart_wown;
    const int32_t* fpart_first;    // [nhubs+1] scan-workgroup range of each hub
};

// partitions per hub in bucketed mode are limited by the scatter kernel's LDS histogram
constexpr int32_t HUB_PMAX = 4096;
constexpr int32_t HUB_PSMALL = 1024;  // the scatter pass's per-partition counts fit a smaller LDS array up to here


// ---- launchers (lv_kernels.hip) ----
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
hipError_t launch_iota(int32_t* p, int32_t n, hipStream_t s);
hipError_t launch_copy_i32(int32_t* dst, const int32_t* src, int64_t n, hipStream_t s);
// dst[t] = src[idx[t]] (dst may alias idx)
hipError_t launch_gather_i32(const int32_t* src, const int32_t* idx, int32_t m, int32_t* dst, hipStream_t s);
// out[v] = labels[v] - base[gid[v]] (gid null: copy)
hipError_t launch_local_labels(int32_t n, const int32_t* labels, const int32_t* gid, const int32_t* base, int32_t* out,
                               hipStream_t s);

// exclusive scans; `total` (device, may be null) receives the sum
hipError_t scan_exclusive_i32(const int32_t* in, int32_t* out, int64_t n, int32_t* total, void* tmp,
                              size_t tmp_bytes, hipStream_t s);
hipError_t scan_exclusive_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* total, void* tmp,
                              size_t tmp_bytes, hipStream_t s);
size_t scan_tmp_bytes(int64_t n, size_t elem);

// stable LSD radix sort of (key, value) pairs on key bits [0, bits)
size_t radix_tmp_bytes(int64_t n);
hipError_t radix_sort_u64(uint64_t* keys, int32_t* vals, uint64_t* keys_alt, int32_t* vals_alt, int64_t n,
                          int bits, void* tmp, size_t tmp_bytes, bool* result_in_alt, hipStream_t s);
hipError_t radix_sort_u32(uint32_t* keys, int32_t* vals, uint32_t* keys_alt, int32_t* vals_alt, int64_t n,
                          int bits, void* tmp, size_t tmp_bytes, bool* result_in_alt, hipStream_t s);

// graph preparation / validation; err bits: 1 offsets, 2 indices, 4 weights,
// 8 asymmetric, 16 overflow
hipError_t launch_check_offsets(int32_t n, const int32_t* off, int64_t nnz, int32_t* err, hipStream_t s);
hipError_t launch_check_entries(int32_t n, const int32_t* off, const int32_t* idx, const int32_t* w,
                                int64_t nnz, int32_t* err, hipStream_t s);
hipError_t launch_check_symmetric(int32_t n, const int32_t* off, const int32_t* idx, const int32_t* w,
                                  int64_t nnz, int32_t* err, hipStream_t s);
hipError_t launch_diag_scan(int32_t n, const int32_t* off, const int32_t* idx, int32_t* diag_pos,
                            int32_t* any_diag, hipStream_t s);
hipError_t launch_adjacency_weights(int32_t n, const int32_t* w_in, const int32_t* diag_pos, int64_t nnz,
                                    int32_t* w_out, int32_t* err, hipStream_t s);
// k = row sums (int32), k64 scratch [n], *total += sum (caller zeroes total)
hipError_t launch_row_sums(int32_t n, const int32_t* off, const int32_t* w, int64_t nnz, int32_t* k,
                           int64_t* k64, int64_t* total, hipStream_t s);
hipError_t launch_degree_unit(int32_t n, const int32_t* off, int32_t* k, hipStream_t s);
// per graph g (gid null: one graph): out[g] += sum of v^2 / trace (caller zeroes out)
hipError_t launch_sum_sq(const int32_t* v, int64_t n, const int32_t* gid, int64_t* out, hipStream_t s);
hipError_t launch_trace(int32_t n, const int32_t* off, const int32_t* idx, const int32_t* w, int64_t nnz,
                        const int32_t* gid, int64_t* out, hipStream_t s);
hipError_t launch_seg_sum(const int32_t* v, int64_t n, const int32_t* gid, int64_t* out, hipStream_t s);
hipError_t launch_fill_gid(const int32_t* voff, int32_t G, int32_t n, int32_t* gid, hipStream_t s);
// out[g] += Sigma_in of labels within graph g
hipError_t launch_sigma_in(int32_t n, const int32_t* off, const int32_t* idx, const int32_t* w, int64_t nnz,
                           const int32_t* labels, const int32_t* gid, int64_t* out, hipStream_t s);
// The same for one graph from an entry cache that holds every entry's
// neighbour label of `labels` (a loop entry holds EMPTY_KEY): *out += the
// weight of the non-loop entries inside communities; the caller adds the trace.
hipError_t launch_sigma_in_cached(int32_t n, const int32_t* off, const int2* ce, const int32_t* w, int64_t nnz,
                                  const int32_t* labels, int64_t* out, hipStream_t s);

// classes
hipError_t launch_classify(int32_t n, const int32_t* off, const int32_t* bounds, uint32_t* cls,
                           int32_t* vert, hipStream_t s);

hipError_t launch_class_starts(const uint32_t* cls_sorted, int32_t n, int32_t* start, hipStream_t s);
// rows[t] = (v, off[v], off[v+1], k[v]) for v = verts[t], t < m
hipError_t launch_row_descriptors(const int32_t* verts, int32_t m, const int32_t* off, const int32_t* k, int4* rows,
                                  hipStream_t s);
hipError_t launch_gather_rows(const int32_t* verts, int32_t m, const int32_t* off, int32_t* beg, int32_t* len,
                              hipStream_t s);

// out[c] += CSR entries of class c; start = host array [NUM_CLS+1] of class bounds
hipError_t launch_class_entries(const int32_t* verts_sorted, const int32_t* start, const int32_t* off,
                                int64_t* out, hipStream_t s);

// sweep
hipError_t launch_move_class(int cls, bool singleton, bool async, const MoveArgs& a, hipStream_t s);
// Later synchronous sweeps of every class below the hub class in one
// persistent launch (k_move_fused).  Per class q that has rows, in order of
// decreasing row length: its class id, its first work item (item_first[nclass]
// = items in all; an item is one block of 1024 threads laid out as the
// class's own kernel lays out a block) and its listed rows [row_first,
// row_end) in the MoveArgs' rows/dec arrays.
struct FusedMap {
    int32_t nclass;
    int32_t cls[NUM_CLS];
    int32_t item_first[NUM_CLS + 1];
    int32_t row_first[NUM_CLS];
    int32_t row_end[NUM_CLS];
};
hipError_t launch_move_fused(const MoveArgs& a, const FusedMap& fm, SweepCtl* ctl, hipStream_t s);
hipError_t launch_hub_clear(int32_t* table, int64_t slots, hipStream_t s);
hipError_t launch_chunk_list(const int32_t* first, int32_t nhubs, int32_t total, const int32_t* base,
                             const int32_t* len, int32_t chunk, int32_t* o_hub, int32_t* o_beg, int32_t* o_end,
                             hipStream_t s);
// bucketed mode, sweeps after the first: scatter the hubs' entries to the partition buckets
hipError_t launch_hub_scatter(const MoveArgs& a, const HubArgs& h, hipStream_t s);
// partition workgroups, merge and decision, global-table fallback
hipError_t launch_hub_sweep(bool singleton, const MoveArgs& a, const HubArgs& h, hipStream_t s);
// Active-vertex pruning: after the decisions of a sweep, record the sweep
// number for every mover and every neighbour of a mover (rows: the m listed
// vertices below the hub class; the hubs through their mark chunks).
// Gather probe (see lv_probe_gather): stream idx[0, nnz) and gather tab[idx[e]].
// dst[0..n) = src[0..n) with 16-byte accesses (src, dst 16-byte aligned)
hipError_t launch_probe_copy(const int32_t* src, int32_t* dst, int64_t n, hipStream_t s);
hipError_t launch_probe_gather(const int32_t* idx, const int2* tab, int64_t nnz, unsigned long long* sink, hipStream_t s);
hipError_t launch_mark_movers(const int4* rows, const int32_t* dec, int32_t m, const int32_t* idx, int32_t* mark,
                              const SweepCtl* ctl, hipStream_t s);
hipError_t launch_hub_mark(const MoveArgs& a, const HubArgs& h, int32_t* mark, hipStream_t s);
hipError_t launch_pairs(int32_t n, const int32_t* verts, const int32_t* comm, const int32_t* sigma, int2* cs,
                        const SweepCtl* ctl, hipStream_t s);
// As launch_pairs over the m listed vertices verts[0..m) (class order), also
// recording in chg[t] whether slot t's pair changed (LPA: its label) and
// adding the changed rows' entries to ctl->chg_entries.  The changed rows of
// slots below `nonhub` are listed per 256-slot tile: (row begin, length, new
// pair) at list[tile * 256 + i] for i < cnt[tile].
hipError_t launch_pairs_changed(int32_t m, int32_t nonhub, const int32_t* verts, const int32_t* off,
                                const int32_t* comm, const int32_t* sigma, int2* cs, uint8_t* chg, int4* list,
                                int32_t* cnt, int mode, SweepCtl* ctl, hipStream_t s);
// Entry-cache refresh when the next sweep reads the cache: for every listed
// changed row (list/cnt of launch_pairs_changed over m slots), ce[rev[e]] =
// its new pair for each non-loop entry e of the row.  Hubs: through their
// 4096-entry chunks (launch_hub_cache_refresh, from chg).
hipError_t launch_cache_refresh(int32_t m, const int4* list, const int32_t* cnt, const int32_t* rev, int2* ce,
                                SweepCtl* ctl, hipStream_t s);
hipError_t launch_hub_cache_refresh(const MoveArgs& a, const HubArgs& h, const uint8_t* chg_hub, const int32_t* rev,
                                    hipStream_t s);
// Reverse-entry map of a CSR whose rows are sorted: rank[e] = position of
// entry e's reverse (j, i) within row j.  err |= 32 if some entry has no
// reverse (an asymmetric graph).
hipError_t launch_reverse_rank(int32_t n, const int32_t* off, const int32_t* idx, int64_t nnz, int32_t* rank,
                               int32_t* err, hipStream_t s);
// rev[e] = off[idx[e]] + rank[e] (rows kept in place)
hipError_t launch_reverse_from_rank(int32_t n, const int32_t* off, const int32_t* idx, int64_t nnz,
                                    const int32_t* rank, int32_t* rev, hipStream_t s);
// commit the decisions dec[0..m) of vertices verts[0..m); per-graph movers into
// gmoves; sigma null: labels only (LPA)
hipError_t launch_apply(const int32_t* verts, const int32_t* dec, int32_t m, const int32_t* k, const int32_t* gid,
                        int32_t* comm, int32_t* sigma, const SweepCtl* ctl, uint32_t* gmoves, int32_t max_sweeps,
                        hipStream_t s);
// sigma[comm[v]] += k[v] for the vertices verts[0..m) (the caller clears sigma)
hipError_t launch_volumes(const int32_t* verts, int32_t m, const int32_t* k, const int32_t* comm, int32_t* sigma,
                          hipStream_t s);
// level start: sweep counter 0; gdone[g] = !gactive[g] (gactive null = all run); moves zeroed
hipError_t launch_ctl_init(SweepCtl* ctl, int32_t G, const int32_t* gactive, int32_t* gdone, int32_t* gsweeps,
                           uint32_t* gmoves, int32_t max_sweeps, hipStream_t s);
// ec_read_max / ec_fill_max: the next sweep reads the entry cache if it was
// filled and at most ec_read_max entries changed, else fills it if at most
// ec_fill_max changed (-1: no cache)
hipError_t launch_sweep_end(SweepCtl* ctl, int32_t G, int32_t* gdone, int32_t* gsweeps, const uint32_t* gmoves,
                            int32_t max_sweeps, int64_t theta, int32_t consecutive, int64_t ec_read_max,
                            int64_t ec_fill_max, hipStream_t s);

// renumber + aggregation
hipError_t launch_renumber(int32_t n, const int32_t* comm, const int32_t* orig, int32_t* minv, int32_t* flag,
                           int32_t* pos, int32_t* labels, int32_t* n_out, void* tmp, size_t tb, hipStream_t s);
hipError_t launch_coarse_degree(int32_t n, const int32_t* comm, const int32_t* labels, const int32_t* sigma,
                                const int32_t* gid, int32_t* k2, int32_t* gid2, hipStream_t s);
// Storage order by descending degree (within each packed graph): keys for
// the sort, the inverse map, the permuted row lengths and rows.
hipError_t launch_degree_keys(int32_t n, const int32_t* off, const int32_t* gid, int32_t maxdeg, int db, uint64_t* keys,
                              int32_t* vals, hipStream_t s);
hipError_t launch_max_degree(int32_t n, const int32_t* off, int32_t* out, hipStream_t s);
hipError_t launch_inverse(const int32_t* perm, int32_t n, int32_t* inv, hipStream_t s);
hipError_t launch_perm_lengths(const int32_t* perm, int32_t n, const int32_t* off, int32_t* len, hipStream_t s);
// rank (may be null): the reverse-entry ranks of the old rows (launch_reverse_rank);
// then rev_new receives the reverse-entry map of the permuted CSR
hipError_t launch_perm_rows(int32_t n, const int32_t* off_new, int64_t nnz, const int32_t* perm, const int32_t* off,
                            const int32_t* idx, const int32_t* w, const int32_t* inv, int32_t* idx_new, int32_t* w_new,
                            const int32_t* rank, int32_t* rev_new, hipStream_t s);
// dst[idx[t]] = src[t]
hipError_t launch_scatter_i32(const int32_t* src, const int32_t* idx, int32_t m, int32_t* dst, hipStream_t s);
// keys = (label(i) << colbits) | label(j); sigma_in[g] += weight inside communities (caller zeroes it)
// Aggregation keys.  agg = false: one key per entry at the entry's index.
// agg = true: summed per tile (build_keys_tiles(n, nnz) = T tiles), tile b
// leaving meta[b + k T], k = 0..3 = {keys, first entry, distinct keys,
// entries}; pack them with launch_compact_tiles (pos = exclusive scan of
// meta[0..T)).
unsigned build_keys_tiles(int32_t n, int64_t nnz);
hipError_t launch_build_keys(bool agg, int32_t n, const int32_t* off, const int32_t* idx, const int32_t* w, int64_t nnz,
                             const int32_t* labels, int colbits, uint64_t* keys, int32_t* vals, int32_t* meta,
                             const int32_t* gid, int64_t* sigma_in, hipStream_t s);
hipError_t launch_compact_tiles(const uint64_t* keys, const int32_t* vals, const int32_t* meta, const int32_t* pos,
                                unsigned tiles, uint64_t* keys2, int32_t* vals2, hipStream_t s);
// rebuild a packed CSR (off[n_out+1], idx/w[nnz_out], k, gid) from device segment descriptors
hipError_t launch_repack(const RepackSeg* seg, int32_t nseg, int32_t n_out, int64_t nnz_out, int32_t* off, int32_t* idx,
                         int32_t* w, int32_t* k, int32_t* gid, int32_t* orig, hipStream_t s);
hipError_t launch_segment_heads(const uint64_t* keys, int64_t n, int32_t* head, hipStream_t s);
// w2 must be zeroed; writes idx2/w2/keys2 of each run of equal keys
hipError_t launch_segment_reduce(const uint64_t* keys, const int32_t* vals, const int32_t* pos, int64_t n,
                                 int colbits, int32_t* idx2, int32_t* w2, uint64_t* keys2, hipStream_t s);
// Edge list -> 2m keys/values (see lv_graph_create_edges); stats = {entries, volume}.
hipError_t launch_edge_keys(int64_t m, const int32_t* src, const int32_t* dst, const int32_t* w, int32_t n, int cb,
                            bool drop_loops, uint64_t* keys, int32_t* vals, int64_t* stats, int32_t* err, hipStream_t s);
hipError_t launch_halve_diagonal(const uint64_t* keys2, int64_t e2, int cb, int32_t* w2, hipStream_t s);
hipError_t launch_row_offsets(const uint64_t* keys2, int64_t e2, int32_t n2, int colbits, int32_t* off2,
                              hipStream_t s);
hipError_t launch_compose(int32_t n0, int32_t* final_labels, const int32_t* labels, const int32_t* gid0,
                          const int32_t* slot, const int32_t* vbase, const int32_t* nbase, hipStream_t s);
hipError_t launch_modularity_parts(int32_t n, const int32_t* off, const int32_t* idx, const int32_t* w,
                                   int64_t nnz, const int32_t* k, const int32_t* labels, int64_t* tot,
                                   int64_t* out2, hipStream_t s);

hipError_t launch_check_labels(const int32_t* labels, int32_t n, int32_t* err, hipStream_t s);

// ---- aggregation by community (lv_agg.hip)
// One degree class of coarse vertices: verts[0..m) are coarse vertices whose
// segments [seg[P], seg[P+1]) of (col, wt) (wt null: unit) are summed; the
// distinct pairs go to [seg[P], seg[P] + cnt[P]) of (col2, wt2);
// sigma_in[graph] += the weight of the pair (P, P).
struct AggArgs {
    const int32_t* verts;
    int32_t m;
    const int32_t* seg;
    const int32_t* col;
    const int32_t* wt;
    int32_t* col2;
    int32_t* wt2;
    int32_t* cnt;
    const int32_t* gid2;    // graph of each coarse vertex (null: one graph)
    int64_t* sigma_in;
};
hipError_t launch_member_lengths(int32_t n, const int32_t* mem, const int32_t* off, int32_t* dm, hipStream_t s);
hipError_t launch_segment_starts(int32_t n, const uint32_t* lab_sorted, const int32_t* voff, int32_t n2, int32_t nnz,
                                 int32_t* seg, hipStream_t s);
hipError_t launch_agg_class(int cls, const AggArgs& a, hipStream_t s);
hipError_t launch_long_lengths(int32_t nh, const int32_t* hv, const int32_t* seg, int32_t* hd, hipStream_t s);
hipError_t launch_long_keys(int32_t nh, const int32_t* hv, const int32_t* hoff, int64_t eh, const int32_t* seg,
                            const int32_t* col, const int32_t* wt, int colbits, uint64_t* keys, int32_t* vals,
                            hipStream_t s);
hipError_t launch_long_place(int64_t eu, const uint64_t* keys2, const int32_t* col_u, const int32_t* wt_u,
                             const int32_t* uoff, const int32_t* seg, int colbits, int32_t* col2, int32_t* wt2,
                             const int32_t* gid2, int64_t* sigma_in, hipStream_t s);
hipError_t launch_long_counts(int32_t nh, const int32_t* hv, const int32_t* uoff, int32_t* cnt, hipStream_t s);
hipError_t launch_pack_rows(int32_t n2, const int32_t* off2, int64_t e2, const int32_t* seg, const int32_t* col2,
                            const int32_t* wt2, int32_t* idx, int32_t* w, hipStream_t s);
// sort the columns of every row of a CSR in place (keys / vals: nnz items each, plus alternates)
hipError_t launch_row_keys(int32_t n, const int32_t* off, int64_t nnz, const int32_t* idx, const int32_t* w,
                           int colbits, uint64_t* keys, int32_t* vals, hipStream_t s);
hipError_t launch_unpack_keys(int64_t nnz, const uint64_t* keys, const int32_t* vals, int colbits, int32_t* idx,
                              int32_t* w, hipStream_t s);

}  // namespace lv
