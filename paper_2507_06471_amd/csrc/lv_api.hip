// C ABI of the Louvain library (declared in include/lv.h): argument checks,
// device workspace, and the host-side level driver of Algorithm 3 around the
// HIP kernels.
//
// One engine serves every entry point: a handle packs G >= 1 independent
// graphs into one CSR (vertex segments), and every level runs all of them in
// the same launches.  Each graph keeps its own total volume M, its own sweep
// count and stopping rule (kept on the device: no host round trip per sweep,
// so a level's sweep loop is replayed from a captured HIP graph), its own
// level acceptance, and leaves the packed graph once its run ends.  A single
// graph is the case G = 1.
#include "lv.h"
#include "lv_internal.h"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <initializer_list>
#include <vector>

using namespace lv;

namespace {

thread_local std::string g_last_error;

void set_error(const char* what, hipError_t e)
{
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    g_last_error = buf;
}
void set_error_msg(const std::string& m) { g_last_error = m; }

lv_status from_hip(hipError_t e) { return e == hipErrorOutOfMemory ? LV_E_NOMEM : LV_E_HIP; }

#define HIP_TRY(expr)                                                  \
    do {                                                               \
        hipError_t e_ = (expr);                                        \
        if (e_ != hipSuccess) {                                        \
            set_error(#expr, e_);                                      \
            return from_hip(e_);                                       \
        }                                                              \
    } while (0)

#define LV_TRY(expr)                                                   \
    do {                                                               \
        lv_status s_ = (expr);                                         \
        if (s_ != LV_OK) return s_;                                    \
    } while (0)

// Waits for the stream when it goes out of scope.  Declared after host
// buffers that are the source or target of asynchronous copies, it keeps
// every such copy from outliving its buffer when a later call fails and the
// function returns early (a pending copy into a freed vector or a popped
// stack slot would corrupt host memory).  Never used inside a captured region.
struct SyncOnExit {
    hipStream_t s;
    ~SyncOnExit() { (void)hipStreamSynchronize(s); }
};

// Allocation with optional fault injection for tests of the out-of-memory
// paths: with LV_FAULT_ALLOC_AT=k in the environment, the k-th device or
// pinned-host allocation made by one entry-point call on the calling thread
// fails with out-of-memory.  The variable is read at the start of every
// graph-creation, louvain, lpa and modularity call (FaultScope), so a test may
// change it between calls.
thread_local long t_alloc_count = 0;
thread_local long t_fail_at = 0;
struct FaultScope {
    FaultScope()
    {
        t_alloc_count = 0;
        const char* v = std::getenv("LV_FAULT_ALLOC_AT");
        t_fail_at = v ? std::atol(v) : 0L;
    }
};
bool fault_now()
{
    ++t_alloc_count;
    return t_fail_at > 0 && t_alloc_count == t_fail_at;
}
hipError_t dev_alloc(void** p, size_t bytes)
{
    if (fault_now()) { *p = nullptr; return hipErrorOutOfMemory; }
    return hipMalloc(p, bytes ? bytes : 1);
}

// Grow-only device buffer.
struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
    hipError_t ensure(size_t bytes)
    {
        bytes = (bytes + 255) & ~(size_t)255;
        if (bytes == 0) bytes = 256;
        if (cap >= bytes) return hipSuccess;
        release();
        hipError_t e = dev_alloc(&p, bytes);
        if (e == hipSuccess) cap = bytes; else p = nullptr;
        return e;
    }
    template <typename T> T* as() const { return (T*)p; }
    void swap(DevBuf& o)
    {
        std::swap(p, o.p);
        std::swap(cap, o.cap);
    }
};

struct Workspace {
    DevBuf comm, sigma, dec, cls, vert, cls_alt, vert_alt, minv, flag, pos, labels, tmp, small, cs;
    DevBuf keys, keys_alt, vals, vals_alt, head;
    DevBuf g_off[2], g_idx[2], g_w[2], g_k[2], g_gid[2];
    DevBuf hub_table, hub_meta, hub_part, hub_rows, hub_cnt, hub_bucket, hub_bucket_w;
    bool hub_table_clean = false;  // every slot of hub_table is empty
    DevBuf rows;  // per-level row descriptors of the class-sorted vertices
    DevBuf ce;    // entry cache: per CSR entry of the handle's input graph, its neighbour's pair
    DevBuf chg;   // per listed vertex: its pair changed in the last commit (uint8)
    DevBuf rlist, rcnt;  // per 256-slot tile: its changed rows below the hub class (int4) and their number
    DevBuf mark;  // active-vertex pruning: last sweep that changed the vertex's neighbourhood
    DevBuf tiles; // aggregation: per key tile its count, first entry and output position
    DevBuf p_off, p_idx, p_w, p_k, p_orig, p_inv;  // a coarse level stored by degree
    DevBuf k64;
    // aggregation by community: entry offsets in member order, segment starts,
    // distinct counts, long segments' offsets, their sort keys and results
    DevBuf a_voff, a_seg, a_cnt, a_hoff, a_uoff, h_keys, h_keys_alt, h_col, h_wt;
    // per-graph state of a level (G entries) and sweep control
    DevBuf ctl, gdone, gsweeps, gmoves, gactive, gsum, gsq, gmeta, segs;
};

struct Timer {
    bool on = false;
    hipStream_t s = nullptr;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    hipError_t mark(hipEvent_t* out)
    {
        if (used == pool.size()) {
            hipEvent_t ev;
            hipError_t e = hipEventCreate(&ev);
            if (e != hipSuccess) return e;
            pool.push_back(ev);
        }
        *out = pool[used++];
        return hipEventRecord(*out, s);
    }
    ~Timer()
    {
        for (auto ev : pool) (void)hipEventDestroy(ev);
    }
};

float elapsed(hipEvent_t a, hipEvent_t b)
{
    float ms = 0.f;
    if (!a || !b || hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.f;
    return ms;
}

int bits_for(int64_t x)
{
    int b = 1;
    while (b < 62 && (1LL << b) < x) ++b;
    return b;
}

uint64_t next_pow2(uint64_t x)
{
    uint64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

// Device buffers that results hold (level labels, final labels) come from a
// pool of the handle and go back to it when the result is destroyed, so that
// repeated calls neither allocate nor free (a free waits for the whole
// device).  A result may outlive its handle: a buffer whose pool is gone is
// freed.  The pool keeps what it holds until the handle is destroyed.
struct BufPool {
    std::mutex mu;
    std::vector<std::unique_ptr<DevBuf>> free;
};
struct PooledBuf {
    std::unique_ptr<DevBuf> buf;
    std::weak_ptr<BufPool> pool;
    PooledBuf() = default;
    PooledBuf(const PooledBuf&) = delete;
    PooledBuf& operator=(const PooledBuf&) = delete;
    ~PooledBuf() { give_back(); }
    void give_back()
    {
        if (buf && buf->p) {
            if (std::shared_ptr<BufPool> pl = pool.lock()) {
                std::lock_guard<std::mutex> lk(pl->mu);
                pl->free.push_back(std::move(buf));
            }
        }
        buf.reset();
    }
    int32_t* i32() const { return buf ? buf->as<int32_t>() : nullptr; }
};
// Take the pool's smallest buffer of at least `bytes` (else its largest,
// grown) into `out`.
hipError_t pool_take(const std::shared_ptr<BufPool>& pool, size_t bytes, PooledBuf& out)
{
    out.give_back();
    out.pool = pool;
    {
        std::lock_guard<std::mutex> lk(pool->mu);
        const size_t want = (std::max<size_t>(bytes, 1) + 255) & ~(size_t)255;
        int best = -1;
        for (int i = 0; i < (int)pool->free.size(); ++i) {
            const size_t c = pool->free[i]->cap;
            if (best < 0) { best = i; continue; }
            const size_t b = pool->free[best]->cap;
            const bool fits = c >= want, best_fits = b >= want;
            if (fits ? (!best_fits || c < b) : (!best_fits && c > b)) best = i;
        }
        if (best >= 0) {
            out.buf = std::move(pool->free[best]);
            pool->free.erase(pool->free.begin() + best);
        }
    }
    if (!out.buf) out.buf = std::make_unique<DevBuf>();
    return out.buf->ensure(std::max<size_t>(bytes, 1));
}

}  // namespace

struct lv_graph {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int32_t n = 0;          // packed vertices
    int64_t nnz = 0;        // packed entries
    int32_t G = 1;          // graphs
    DevBuf off, idx, w, k;
    bool weighted = false;  // false: every A entry is 1 (no weights, no loops)
    std::vector<int32_t> voff;   // [G+1] vertex offset of each graph
    std::vector<int64_t> eoff;   // [G+1] entry offset of each graph
    std::vector<int64_t> M;      // [G] total volume
    std::vector<int64_t> q0;     // [G] Q_int of singletons
    std::vector<int64_t> trace;  // [G] sum of the diagonal entries (loops, doubled)
    DevBuf d_gid, d_M;           // per vertex graph id, per graph M (G > 1)
    // Storage order: vertices are kept by descending degree within each
    // graph (unless LV_KEEP_ORDER); orig[p] = vertex id at position p,
    // inv[id] = its position.  Every segment of a packed handle keeps its
    // range, so graph ids by position and by id coincide.
    bool reordered = false;
    DevBuf orig, inv;
    // Reverse-entry map of the stored input graph: rev[e] = position of the
    // entry (j, i) for the entry e = (i, j) (a loop entry: itself).  Built at
    // creation unless LV_NO_ENTRY_CACHE; used to keep the entry cache current.
    DevBuf rev;
    bool has_rev = false;
    Workspace ws;
    int32_t* pinned = nullptr;   // host staging area
    size_t pinned_bytes = 0;
    bool has_tuned = false;      // LV_AUTOTUNE: the setting chosen on first use
    lv_tuning tuned{};
    // Set-up frees nothing while set (a free waits for the whole device, and
    // the server sets graphs up while another stream runs): buffers that set-up
    // would free are parked here until the handle is destroyed.
    bool keep_scratch = false;
    std::vector<std::unique_ptr<DevBuf>> parked;
    std::shared_ptr<BufPool> pool = std::make_shared<BufPool>();  // result buffers
    void release_or_park(DevBuf& b)
    {
        if (!b.p) return;
        if (!keep_scratch) { b.release(); return; }
        parked.push_back(std::make_unique<DevBuf>());
        parked.back()->swap(b);
    }
    ~lv_graph()
    {
        if (pinned) (void)hipHostFree(pinned);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
};

namespace {

// Labels of one packed level, shared by the graphs that took part in it.
struct LabelStore {
    PooledBuf labels;
    int32_t n = 0;
};

struct LevelRecord {
    lv_level_info info{};
    std::vector<int64_t> moves;
    std::shared_ptr<LabelStore> store;  // accepted levels: packed labels of the level
    int32_t vbase = 0, nbase = 0;       // this graph's slice: labels[vbase + x] - nbase
    std::shared_ptr<DevBuf> g_off, g_idx, g_w;  // coarse graph (one graph, LV_KEEP_GRAPHS)
    int64_t g_nnz = 0;
};

struct GraphResult {
    int32_t n0 = 0, fin_base = 0;
    int64_t M = 0, q_int = 0;
    int32_t accepted = 0;
    std::vector<LevelRecord> levels;
};

}  // namespace

struct lv_result {
    int32_t G = 1;
    int32_t n0 = 0;
    std::vector<GraphResult> graphs;
    PooledBuf final_labels;  // packed like the handle's vertices
};

namespace {

struct Tune {
    int32_t bounds[NUM_CLS];
    int32_t part_keys;  // expected distinct communities per partition workgroup
    int32_t part_slots; // LDS slots of a partition workgroup (power of two)
    int32_t bucketed;   // partition mode (see lv_tuning.hub_mode)
    int32_t fb_chunk;   // entries / slots per workgroup on the global-table fallback
    int32_t sc_chunk;   // entries per scatter workgroup (bucketed mode)
    int64_t order_min;  // coarse levels with at least this many entries are stored by degree
    int32_t agg_sort;   // 1: aggregation sorts every entry's key (else by community)
    int32_t fused;      // 1: later sweeps of the classes below the hub class in one persistent launch
    int32_t table_pct;  // later sweeps' LDS tables: about L * table_pct / 100 + 1 slots for L entries
    int32_t cache_read_pct;  // entry cache: read it after a commit that changed at most this % of the pairs
    int32_t cache_fill_pct;  // ... fill it during a sweep after a commit that changed at most this %
};

Tune make_tune(const lv_tuning* t)
{
    Tune u;
    for (int c = 0; c < NUM_CLS; ++c) u.bounds[c] = CLS_CAP[c];
    // default partition mode: bucketed, 1024 expected communities per 2048-slot table
    u.part_keys = 1024;
    u.part_slots = 2048;
    u.bucketed = 1;
    u.order_min = (int64_t)1 << 22;
    u.fb_chunk = 4096;
    u.sc_chunk = 2048;
    u.agg_sort = 0;
    u.cache_read_pct = 10;
    u.fused = 0;
    u.table_pct = 300;
    if (t) {
        // sub_max bounds the sub-wavefront classes, wave_max the wavefront
        // class, block_max the workgroup classes; each is clamped to the
        // class's cap, so no setting can overflow a table.
        auto cap = [&](int c, int32_t knob) { u.bounds[c] = std::min(CLS_CAP[c], knob); };
        if (t->sub_max > 0)
            for (int c = CLS_L4; c < CLS_FIRST_WAVE; ++c) cap(c, t->sub_max);
        if (t->wave_max > 0)
            for (int c = CLS_FIRST_WAVE; c < CLS_FIRST_BLOCK; ++c) cap(c, t->wave_max);
        if (t->block_max > 0)
            for (int c = CLS_FIRST_BLOCK; c < CLS_HUB; ++c) cap(c, t->block_max);
        if (t->hub_mode == 1) {
            u.bucketed = 0;
            u.part_slots = 16384;
            u.part_keys = 8192;
        }
        const uint64_t max_slots = u.bucketed ? 2048 : 16384;
        if (t->part_slots > 0)
            u.part_slots = (int32_t)std::min<uint64_t>(max_slots, std::max<uint64_t>(64, next_pow2((uint64_t)t->part_slots)));
        if (t->part_keys > 0) u.part_keys = std::max(32, t->part_keys);
        if (t->hub_chunk > 0) u.sc_chunk = t->hub_chunk <= 1024 ? 1024 : t->hub_chunk <= 2048 ? 2048 : 4096;
        if (t->order_min > 0) u.order_min = t->order_min;
        u.agg_sort = t->agg_sort == 1 ? 1 : 0;
        if (t->cache_pct > 0) u.cache_read_pct = std::min(100, t->cache_pct);
        u.fused = t->fused == 1 ? 1 : 0;
        if (t->table_pct > 0) u.table_pct = std::min(400, std::max(100, t->table_pct));
    }
    u.cache_fill_pct = std::max(u.cache_read_pct, std::min(100, 2 * u.cache_read_pct + 5));
    // a single partition must always fit: part_keys <= 3/4 of the slots
    u.part_keys = std::min(u.part_keys, u.part_slots / 4 * 3);
    // keep bounds non-decreasing
    for (int c = CLS_L8; c < CLS_HUB; ++c) u.bounds[c] = std::max(u.bounds[c], u.bounds[c - 1]);
    return u;
}

struct Params {
    int32_t max_sweeps = 20;
    int32_t max_levels = 32;
    int64_t lpa_threshold = 0;
    uint32_t flags = 0;
    Tune tune{};
};

lv_status read_params(const lv_params* p, Params& out)
{
    lv_params d;
    lv_params_default(&d);
    const lv_params* q = p ? p : &d;
    if (q->max_sweeps < 1 || q->max_sweeps > 1000 || q->max_levels < 1 || q->lpa_threshold < 0) {
        set_error_msg("lv_params: max_sweeps in [1,1000], max_levels >= 1, lpa_threshold >= 0");
        return LV_E_ARG;
    }
    out.max_sweeps = q->max_sweeps;
    out.max_levels = q->max_levels;
    out.lpa_threshold = q->lpa_threshold;
    out.flags = q->flags;
    out.tune = make_tune(q->tuning);
    return LV_OK;
}

// One level's packed graph (device pointers) and its graphs.
struct LevelGraph {
    int32_t n;
    int64_t nnz;
    const int32_t* off;
    const int32_t* idx;
    const int32_t* w;    // null = unit
    const int32_t* k;
    int32_t G;           // graphs packed in this level
    const int32_t* gid;  // per vertex graph (null when G == 1)
    const int64_t* Mg;   // per graph M, device (null when G == 1)
    int64_t M;           // M when G == 1
    std::vector<int32_t> voff;  // [G+1] vertex offsets (host)
    std::vector<int64_t> Mh;    // [G] total volume of each graph (host)
    const int32_t* orig = nullptr;  // vertex id at each position (null: the position)
    const int32_t* rev = nullptr;   // reverse-entry map (the handle's input graph only; null: none)
};

// timing slots after the 2 x 11 class slots: the bucketed scatter pass, the
// commit (labels, volumes, pairs, sweep control) and the entry-cache refresh
constexpr int SLOT_HUB_SCATTER = 22, SLOT_COMMIT = 23, SLOT_REFRESH = 24, SLOT_FUSED = 25;

struct SweepOut {
    std::vector<int32_t> sweeps;   // [G]
    std::vector<uint32_t> moves;   // [G * max_sweeps]
    int32_t executed = 0;          // sweeps with at least one running graph
    double move_ms = 0, sweep_ms = 0;
    int64_t launches = 0;
    int64_t bytes = 0;
    double kern_ms[LV_KERNEL_SLOTS] = {};
    int64_t kern_launches[LV_KERNEL_SLOTS] = {};
    int64_t kern_bytes[LV_KERNEL_SLOTS] = {};
    int32_t isolated = 0;          // vertices without entries
    int32_t cached_sweeps = 0;     // sweeps that read the entry cache
    int64_t refreshed = 0;         // cache entries rewritten after commits
    int32_t ec_last = EC_GATHER;   // how the last sweep got its pairs (EC_GATHER without a cache)
};

// Hub (partition) layout for one level.
struct HubPlan {
    int32_t nhubs = 0;
    HubArgs args{};
};

lv_status ensure_pinned(lv_graph* g, size_t bytes)
{
    if (g->pinned_bytes >= bytes) return LV_OK;
    if (g->pinned) (void)hipHostFree(g->pinned);
    g->pinned = nullptr;
    g->pinned_bytes = 0;
    if (fault_now()) { set_error_msg("hipHostMalloc: injected out-of-memory"); return LV_E_NOMEM; }
    HIP_TRY(hipHostMalloc((void**)&g->pinned, bytes, hipHostMallocDefault));
    g->pinned_bytes = bytes;
    return LV_OK;
}

// Read small device results back to host memory through the handle's pinned
// staging area, several in one wait.  Overwrites the staging area.
struct HostCopy {
    void* dst;
    const void* src;
    size_t bytes;
};
lv_status read_back(lv_graph* g, std::initializer_list<HostCopy> parts)
{
    auto padded = [](size_t b) { return (b + 15) & ~(size_t)15; };
    size_t total = 0;
    for (const HostCopy& p : parts) total += padded(p.bytes);
    LV_TRY(ensure_pinned(g, std::max<size_t>(total, 4096)));
    char* base = (char*)g->pinned;
    size_t at = 0;
    for (const HostCopy& p : parts) {
        if (p.bytes) HIP_TRY(hipMemcpyAsync(base + at, p.src, p.bytes, hipMemcpyDeviceToHost, g->stream));
        at += padded(p.bytes);
    }
    HIP_TRY(hipStreamSynchronize(g->stream));
    at = 0;
    for (const HostCopy& p : parts) {
        if (p.bytes) std::memcpy(p.dst, base + at, p.bytes);
        at += padded(p.bytes);
    }
    return LV_OK;
}

lv_status plan_hubs(lv_graph* g, const LevelGraph& G, const int32_t* hub_verts, int32_t nhubs, const Tune& tu_in,
                    HubPlan& plan)
{
    Tune tu = tu_in;
    Workspace& ws = g->ws;
    hipStream_t s = g->stream;
    plan.nhubs = nhubs;
    if (nhubs == 0) return LV_OK;
    // row starts and lengths of the hubs; the lengths are read back to size the layout
    HIP_TRY(ws.hub_rows.ensure(sizeof(int32_t) * 2 * (size_t)nhubs));
    int32_t* d_beg = ws.hub_rows.as<int32_t>();
    int32_t* d_len = d_beg + nhubs;
    HIP_TRY(launch_gather_rows(hub_verts, nhubs, G.off, d_beg, d_len, s));
    std::vector<int32_t> len(nhubs);
    LV_TRY(read_back(g, {{len.data(), d_len, sizeof(int32_t) * (size_t)nhubs}}));
    if (tu.bucketed) {
        // the scatter pass histograms at most HUB_PMAX partitions of a vertex:
        // a level with a longer row uses the compact mode instead
        const int32_t maxL = *std::max_element(len.begin(), len.end());
        if (((int64_t)maxL + tu.part_keys - 1) / tu.part_keys > HUB_PMAX) {
            tu.bucketed = 0;
            tu.part_slots = 16384;
            tu.part_keys = 8192;
        }
    }
    // Per hub: its partitions, its fallback table, and where its workgroups
    // start in each per-workgroup list (partition, scatter, fallback insert
    // and scan, pruning marks).  The lists themselves are expanded on the
    // device from these prefix counts (k_chunk_list), so the host work and the
    // upload stay proportional to the number of hubs.
    constexpr int64_t MARK_CHUNK = 4096;  // entries per pruning-mark workgroup
    std::vector<int32_t> parts(nhubs), tab_cap(nhubs);
    std::vector<int32_t> first_blk(nhubs + 1), first_sc(nhubs + 1), first_ins(nhubs + 1), first_scan(nhubs + 1),
        first_mk(nhubs + 1);
    std::vector<int64_t> tab_off(nhubs);
    int64_t slots = 0, nblk = 0, nsc = 0, nins = 0, nscan = 0, nmk = 0;
    auto chunks = [](int64_t n, int64_t c) { return (n + c - 1) / c; };
    for (int32_t h = 0; h < nhubs; ++h) {
        first_mk[h] = (int32_t)nmk;
        nmk += chunks(len[h], MARK_CHUNK);
        const int64_t P = std::max<int64_t>(1, chunks(len[h], tu.part_keys));
        parts[h] = (int32_t)P;
        first_blk[h] = (int32_t)nblk;
        nblk += P;
        first_sc[h] = (int32_t)nsc;
        first_ins[h] = (int32_t)nins;
        first_scan[h] = (int32_t)nscan;
        tab_off[h] = slots;
        tab_cap[h] = 0;
        if (P == 1) continue;  // one partition of <= part_keys keys always fits its LDS table
        if (tu.bucketed) nsc += chunks(len[h], tu.sc_chunk);
        const uint64_t cap = std::max<uint64_t>(64, next_pow2(2ull * (uint64_t)len[h]));
        if (cap > (uint64_t)INT32_MAX) { set_error_msg("hub table too large"); return LV_E_OVERFLOW; }
        tab_cap[h] = (int32_t)cap;
        slots += (int64_t)cap;
        nins += chunks(len[h], tu.fb_chunk);
        nscan += chunks((int64_t)cap, tu.fb_chunk);
    }
    if (std::max({nblk, nsc, nins, nscan, nmk}) > (int64_t)INT32_MAX) {
        set_error_msg("hub workgroup lists too long");
        return LV_E_OVERFLOW;
    }
    first_blk[nhubs] = (int32_t)nblk;
    first_sc[nhubs] = (int32_t)nsc;
    first_ins[nhubs] = (int32_t)nins;
    first_scan[nhubs] = (int32_t)nscan;
    first_mk[nhubs] = (int32_t)nmk;
    // device metadata: int64 tab_off, then the per-hub int32 arrays (uploaded
    // through the pinned staging area), then the per-workgroup lists
    const size_t H = (size_t)nhubs, H1 = H + 1;
    const size_t o_hv = 0, o_parts = o_hv + H, o_cap = o_parts + H, o_fb = o_cap + H, o_fsc = o_fb + H1,
                 o_fins = o_fsc + H1, o_ff = o_fins + H1, o_fmk = o_ff + H1, n_up = o_fmk + H1;
    const size_t o_bh = n_up, o_bp = o_bh + (size_t)nblk, o_ch = o_bp + (size_t)nblk, o_cb = o_ch + (size_t)nsc,
                 o_ce = o_cb + (size_t)nsc, o_ih = o_ce + (size_t)nsc, o_ib = o_ih + (size_t)nins,
                 o_ie = o_ib + (size_t)nins, o_sh = o_ie + (size_t)nins, o_sb = o_sh + (size_t)nscan,
                 o_se = o_sb + (size_t)nscan, o_mh = o_se + (size_t)nscan, o_mb = o_mh + (size_t)nmk,
                 o_me = o_mb + (size_t)nmk, n_all = o_me + (size_t)nmk;
    const size_t b64 = sizeof(int64_t) * H;
    const size_t up_bytes = b64 + sizeof(int32_t) * n_up;
    HIP_TRY(ws.hub_meta.ensure(b64 + sizeof(int32_t) * n_all + 64));
    char* base = ws.hub_meta.as<char>();
    int32_t* p32 = (int32_t*)(base + b64);
    LV_TRY(ensure_pinned(g, up_bytes));
    {
        char* st = (char*)g->pinned;
        int32_t* u32 = (int32_t*)(st + b64);
        std::memcpy(st, tab_off.data(), b64);
        std::memcpy(u32 + o_parts, parts.data(), sizeof(int32_t) * H);
        std::memcpy(u32 + o_cap, tab_cap.data(), sizeof(int32_t) * H);
        std::memcpy(u32 + o_fb, first_blk.data(), sizeof(int32_t) * H1);
        std::memcpy(u32 + o_fsc, first_sc.data(), sizeof(int32_t) * H1);
        std::memcpy(u32 + o_fins, first_ins.data(), sizeof(int32_t) * H1);
        std::memcpy(u32 + o_ff, first_scan.data(), sizeof(int32_t) * H1);
        std::memcpy(u32 + o_fmk, first_mk.data(), sizeof(int32_t) * H1);
    }
    // the staging area is reused by the next read-back only after the stream
    // has drained (every read-back synchronizes first), and this function
    // synchronizes before it returns
    HIP_TRY(hipMemcpyAsync(base, g->pinned, up_bytes, hipMemcpyHostToDevice, s));
    HIP_TRY(launch_copy_i32(p32 + o_hv, hub_verts, nhubs, s));
    HIP_TRY(launch_chunk_list(p32 + o_fb, nhubs, (int32_t)nblk, nullptr, p32 + o_parts, 1, p32 + o_bh, p32 + o_bp,
                              nullptr, s));
    HIP_TRY(launch_chunk_list(p32 + o_fsc, nhubs, (int32_t)nsc, d_beg, d_len, tu.sc_chunk, p32 + o_ch, p32 + o_cb,
                              p32 + o_ce, s));
    HIP_TRY(launch_chunk_list(p32 + o_fins, nhubs, (int32_t)nins, d_beg, d_len, tu.fb_chunk, p32 + o_ih, p32 + o_ib,
                              p32 + o_ie, s));
    HIP_TRY(launch_chunk_list(p32 + o_ff, nhubs, (int32_t)nscan, nullptr, p32 + o_cap, tu.fb_chunk, p32 + o_sh,
                              p32 + o_sb, p32 + o_se, s));
    HIP_TRY(launch_chunk_list(p32 + o_fmk, nhubs, (int32_t)nmk, d_beg, d_len, (int32_t)MARK_CHUNK, p32 + o_mh,
                              p32 + o_mb, p32 + o_me, s));
    // partial results + flags: [nblk] x (int64 score, int32 comm, wown, flag), [nhubs] fb_flag, [nscan] fallback partials
    const size_t part_bytes =
        (size_t)nblk * (8 + 4 * 3) + (size_t)nhubs * 4 + (size_t)std::max<int64_t>(nscan, 1) * (8 + 4 * 2);
    HIP_TRY(ws.hub_part.ensure(part_bytes + 64));
    char* pb = ws.hub_part.as<char>();
    HubArgs& a = plan.args;
    a = HubArgs{};
    a.nhubs = nhubs;
    a.part_mask = (uint32_t)tu.part_slots - 1u;
    a.bucketed = tu.bucketed;
    a.hub_vert = p32 + o_hv;
    a.hub_parts = p32 + o_parts;
    a.hub_first_blk = p32 + o_fb;
    a.blk_hub = p32 + o_bh;
    a.blk_part = p32 + o_bp;
    a.nblk = (int32_t)nblk;
    a.part_score = (int64_t*)pb;
    a.part_comm = (int32_t*)(a.part_score + nblk);
    a.part_wown = a.part_comm + nblk;
    a.part_flag = a.part_wown + nblk;
    a.fb_flag = a.part_flag + nblk;
    int64_t* fps = (int64_t*)(((uintptr_t)(a.fb_flag + nhubs) + 7) & ~(uintptr_t)7);
    a.fpart_score = fps;
    a.fpart_comm = (int32_t*)(fps + std::max<int64_t>(nscan, 1));
    a.fpart_wown = a.fpart_comm + std::max<int64_t>(nscan, 1);
    a.fpart_first = p32 + o_ff;
    a.tab_off = (const int64_t*)base;
    a.sc_hub = p32 + o_ch;
    a.sc_beg = p32 + o_cb;
    a.sc_end = p32 + o_ce;
    a.nsc = (int32_t)nsc;
    a.mk_hub = p32 + o_mh;
    a.mk_beg = p32 + o_mb;
    a.mk_end = p32 + o_me;
    a.nmk = (int32_t)nmk;
    a.sc_chunk = tu.sc_chunk;
    a.max_parts = 0;
    for (int32_t h = 0; h < nhubs; ++h) a.max_parts = std::max(a.max_parts, parts[h]);
    a.bucket_cap = tu.part_slots;
    if (tu.bucketed && nsc > 0) {
        const size_t nb = (size_t)nblk * (size_t)tu.part_slots;
        HIP_TRY(ws.hub_cnt.ensure(sizeof(int32_t) * (size_t)nblk));
        HIP_TRY(ws.hub_bucket.ensure(sizeof(int2) * nb));
        a.bucket_cnt = ws.hub_cnt.as<int32_t>();
        a.bucket = ws.hub_bucket.as<int2>();
        HIP_TRY(ws.hub_bucket_w.ensure(sizeof(int32_t) * nb));
        a.bucket_w = ws.hub_bucket_w.as<int32_t>();
        HIP_TRY(launch_fill_i32(a.bucket_cnt, 0, nblk, s));
    }
    a.tab_cap = p32 + o_cap;
    a.ins_hub = p32 + o_ih;
    a.ins_beg = p32 + o_ib;
    a.ins_end = p32 + o_ie;
    a.nins = (int32_t)nins;
    a.scan_hub = p32 + o_sh;
    a.scan_beg = p32 + o_sb;
    a.scan_end = p32 + o_se;
    a.nscan = (int32_t)nscan;
    HIP_TRY(launch_fill_i32(a.fb_flag, 0, nhubs, s));
    // The fallback tables: every slot starts empty, and the scan pass empties
    // each slot it reads, so a table that completed its sweeps is clean for
    // the next level; it is cleared here only when it is new or a level did
    // not complete (run_sweeps marks it clean at the end of a level).
    const size_t old_cap = ws.hub_table.cap;
    HIP_TRY(ws.hub_table.ensure(sizeof(int32_t) * 2 * (size_t)std::max<int64_t>(slots, 1)));
    a.table = ws.hub_table.as<int32_t>();
    if (!ws.hub_table_clean || ws.hub_table.cap != old_cap)
        HIP_TRY(launch_hub_clear(a.table, (int64_t)(ws.hub_table.cap / (2 * sizeof(int32_t))), s));
    ws.hub_table_clean = false;
    // the staging area is free again once the upload is done
    HIP_TRY(hipStreamSynchronize(s));
    return LV_OK;
}


// Synchronous local-moving sweeps of one level (Algorithm 2; Algorithm 1 in
// LPA mode) for every graph of G.  gactive (device, may be null) marks the
// graphs that take part.  On return ws.comm holds the labels and ws.sigma the
// community volumes; out holds per-graph sweep and move counts.
lv_status run_sweeps(lv_graph* g, const LevelGraph& G, int mode, const Params& p, const int32_t* gactive,
                     SweepOut& out)
{
    Workspace& ws = g->ws;
    hipStream_t s = g->stream;
    const int32_t n = G.n;
    const int32_t S = p.max_sweeps;
    const size_t nb = sizeof(int32_t) * (size_t)std::max(n, 1);
    HIP_TRY(ws.comm.ensure(nb));
    HIP_TRY(ws.sigma.ensure(nb));
    HIP_TRY(ws.cs.ensure(2 * nb));
    HIP_TRY(ws.dec.ensure(nb));
    HIP_TRY(ws.cls.ensure(nb));
    HIP_TRY(ws.vert.ensure(nb));
    HIP_TRY(ws.cls_alt.ensure(nb));
    HIP_TRY(ws.vert_alt.ensure(nb));
    HIP_TRY(ws.tmp.ensure(std::max(radix_tmp_bytes(n), scan_tmp_bytes(n, 8))));
    HIP_TRY(ws.small.ensure(4096));
    HIP_TRY(ws.ctl.ensure(sizeof(SweepCtl)));
    HIP_TRY(ws.gdone.ensure(sizeof(int32_t) * (size_t)G.G));
    HIP_TRY(ws.gsweeps.ensure(sizeof(int32_t) * (size_t)G.G));
    HIP_TRY(ws.gmoves.ensure(sizeof(uint32_t) * (size_t)G.G * (size_t)S));
    // pinned: the per-graph move and sweep counts and the control block read
    // back at the end, then (at poll_off) the early-exit flag the sweeps of a
    // large level copy out as they go
    const size_t poll_off = (((sizeof(int32_t) + sizeof(uint32_t) * S) * (size_t)G.G + 64 + sizeof(SweepCtl)) + 63) &
                            ~(size_t)63;
    LV_TRY(ensure_pinned(g, std::max<size_t>(4096, poll_off + 64)));

    // degree classes: classify, then one stable radix pass groups vertices by class
    HIP_TRY(launch_classify(n, G.off, p.tune.bounds, ws.cls.as<uint32_t>(), ws.vert.as<int32_t>(), s));
    bool in_alt = false;
    HIP_TRY(radix_sort_u32(ws.cls.as<uint32_t>(), ws.vert.as<int32_t>(), ws.cls_alt.as<uint32_t>(),
                           ws.vert_alt.as<int32_t>(), n, 8, ws.tmp.p, ws.tmp.cap, &in_alt, s));
    const uint32_t* cls_sorted = in_alt ? ws.cls_alt.as<uint32_t>() : ws.cls.as<uint32_t>();
    const int32_t* vert_sorted = in_alt ? ws.vert_alt.as<int32_t>() : ws.vert.as<int32_t>();
    int32_t* d_start = ws.small.as<int32_t>();
    HIP_TRY(launch_fill_i32(d_start, -1, NUM_CLS + 1, s));
    HIP_TRY(launch_class_starts(cls_sorted, n, d_start, s));
    int32_t start[NUM_CLS + 1];
    LV_TRY(read_back(g, {{start, d_start, sizeof start}}));
    start[NUM_CLS] = n;
    for (int c = NUM_CLS - 1; c >= 0; --c)
        if (start[c] < 0) start[c] = start[c + 1];
    const int32_t active = n - start[CLS_L4];  // vertices with at least one entry
    out.isolated = start[CLS_L4];
    HIP_TRY(ws.rows.ensure(sizeof(int4) * (size_t)std::max(active, 1)));
    HIP_TRY(launch_row_descriptors(vert_sorted + start[CLS_L4], active, G.off, G.k, ws.rows.as<int4>(), s));

    HubPlan hubs;
    LV_TRY(plan_hubs(g, G, vert_sorted + start[CLS_HUB], n - start[CLS_HUB], p.tune, hubs));
    const bool timing = (p.flags & LV_TIMING) != 0;
    const bool async = (p.flags & LV_ASYNC) != 0;
    // Entry cache: on the handle's input graph (its reverse-entry map
    // exists), for full synchronous sweeps.  The device decides per sweep
    // whether to read, fill or bypass it (k_sweep_end).
    const bool use_ec = G.rev && G.nnz > 0 && active > 0 && !(p.flags & (LV_NO_CACHE | LV_PRUNE | LV_ASYNC));
    if (use_ec) {
        HIP_TRY(ws.ce.ensure(sizeof(int2) * (size_t)G.nnz));
        HIP_TRY(ws.chg.ensure((size_t)std::max(active, 1)));
        const size_t tiles = ((size_t)active + 255) / 256;
        HIP_TRY(ws.rlist.ensure(sizeof(int4) * 256 * tiles));
        HIP_TRY(ws.rcnt.ensure(sizeof(int32_t) * tiles));
    }
    const int64_t ec_read_max = use_ec ? G.nnz * p.tune.cache_read_pct / 100 : -1;
    const int64_t ec_fill_max = use_ec ? G.nnz * p.tune.cache_fill_pct / 100 : -1;
    const int32_t nonhub = start[CLS_HUB] - start[CLS_L4];  // listed vertices below the hub class
    // the fused kernel's work items: blocks of rows, longest rows first
    FusedMap fmap{};
    const bool fused = p.tune.fused != 0 && !async;
    if (fused) {
        static const int32_t rows_per_item[NUM_CLS] = {0, 256, 128, 64, 32, 16, 8, 4, 2, 2, 1, 0};
        int32_t items = 0;
        for (int c = CLS_HUB - 1; c >= CLS_L4; --c) {
            const int32_t cnt = start[c + 1] - start[c];
            if (cnt <= 0) continue;
            const int q = fmap.nclass++;
            fmap.cls[q] = c;
            fmap.item_first[q] = items;
            fmap.row_first[q] = start[c] - start[CLS_L4];
            fmap.row_end[q] = start[c + 1] - start[CLS_L4];
            items += (cnt + rows_per_item[c] - 1) / rows_per_item[c];
        }
        fmap.item_first[fmap.nclass] = items;
    }
    int64_t cls_entries[NUM_CLS] = {};
    if (timing) {
        int64_t* d_ce = (int64_t*)(ws.small.as<char>() + 3328);
        HIP_TRY(hipMemsetAsync(d_ce, 0, sizeof cls_entries, s));
        HIP_TRY(launch_class_entries(vert_sorted, start, G.off, d_ce, s));
        HIP_TRY(hipMemcpyAsync(cls_entries, d_ce, sizeof cls_entries, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }

    SweepCtl* ctl = ws.ctl.as<SweepCtl>();
    // Singleton communities are named by vertex id; with degree-ordered
    // storage the id of position p is orig[p] and its volume sits at sigma[id].
    if (G.orig) {
        HIP_TRY(launch_copy_i32(ws.comm.as<int32_t>(), G.orig, n, s));
        HIP_TRY(launch_scatter_i32(G.k, G.orig, n, ws.sigma.as<int32_t>(), s));
    } else {
        HIP_TRY(launch_iota(ws.comm.as<int32_t>(), n, s));
        HIP_TRY(launch_copy_i32(ws.sigma.as<int32_t>(), G.k, n, s));
    }
    const int32_t* act_verts = vert_sorted + start[CLS_L4];  // vertices with entries (the only pairs ever gathered)
    HIP_TRY(launch_pairs(active, act_verts, ws.comm.as<int32_t>(), ws.sigma.as<int32_t>(), ws.cs.as<int2>(), nullptr, s));
    HIP_TRY(launch_ctl_init(ctl, G.G, gactive, ws.gdone.as<int32_t>(), ws.gsweeps.as<int32_t>(),
                            ws.gmoves.as<uint32_t>(), S, s));

    MoveArgs a{};
    a.off = G.off;
    a.idx = G.idx;
    a.w = G.w;
    a.k = G.k;
    a.comm = ws.comm.as<int32_t>();
    a.sigma = ws.sigma.as<int32_t>();
    a.cs = ws.cs.as<int2>();
    a.M = G.M;
    a.Mg = G.G > 1 ? G.Mg : nullptr;
    a.gid = G.G > 1 ? G.gid : nullptr;
    a.gdone = G.G > 1 ? ws.gdone.as<int32_t>() : nullptr;
    a.ctl = ctl;
    a.mode = mode;
    a.ce = use_ec ? ws.ce.as<int2>() : nullptr;
    a.table_pct = p.tune.table_pct;
    a.live_comm = async ? ws.comm.as<int32_t>() : nullptr;
    a.live_sigma = async ? ws.sigma.as<int32_t>() : nullptr;
    a.gmoves = ws.gmoves.as<uint32_t>();
    a.max_sweeps = S;
    a.prune_back = async ? 1 : 2;
    int32_t* mark = nullptr;
    if (p.flags & LV_PRUNE) {
        HIP_TRY(ws.mark.ensure(nb));
        mark = ws.mark.as<int32_t>();
        HIP_TRY(launch_fill_i32(mark, 0, n, s));
    }
    a.mark = mark;
    int32_t* dec_all = ws.dec.as<int32_t>();
    const int64_t theta = mode == MODE_LPA ? p.lpa_threshold : 0;

    Timer tm;
    tm.on = timing;
    tm.s = s;
    std::vector<std::vector<hipEvent_t>> ev;  // per sweep: [class begin/end..., sweep begin, moves end, sweep end]
    // One sweep: move kernels of every class, the partition path, commit,
    // pair refresh, per-graph stopping rule.
    auto launch_sweep = [&](bool singleton, std::vector<hipEvent_t>* e) -> lv_status {
        singleton = singleton && !async;  // an asynchronous sweep changes communities as it runs
        if (e) { e->assign(2 * NUM_CLS + 7, nullptr); HIP_TRY(tm.mark(&(*e)[2 * NUM_CLS])); }
        if (fused && !singleton) {
            a.verts = vert_sorted + start[CLS_L4];
            a.rows = ws.rows.as<int4>();
            a.dec = dec_all + start[CLS_L4];
            a.nverts = nonhub;
            if (e) HIP_TRY(tm.mark(&(*e)[2 * NUM_CLS + 5]));
            HIP_TRY(launch_move_fused(a, fmap, ctl, s));
            if (e) HIP_TRY(tm.mark(&(*e)[2 * NUM_CLS + 6]));
        } else {
            for (int c = CLS_L4; c < CLS_HUB; ++c) {
                a.verts = vert_sorted + start[c];
                a.rows = ws.rows.as<int4>() + (start[c] - start[CLS_L4]);
                a.dec = dec_all + start[c];
                a.nverts = start[c + 1] - start[c];
                if (a.nverts == 0) continue;
                if (e) HIP_TRY(tm.mark(&(*e)[2 * c]));
                HIP_TRY(launch_move_class(c, singleton, async, a, s));
                if (e) HIP_TRY(tm.mark(&(*e)[2 * c + 1]));
            }
        }
        if (hubs.nhubs > 0) {
            const hipStream_t hs = s;
            a.verts = vert_sorted + start[CLS_HUB];
            a.rows = nullptr;
            a.dec = dec_all + start[CLS_HUB];
            a.nverts = hubs.nhubs;
            if (e) HIP_TRY(tm.mark(&(*e)[2 * CLS_HUB]));
            if (!singleton && hubs.args.bucketed && hubs.args.nsc > 0) {
                HIP_TRY(launch_hub_scatter(a, hubs.args, hs));
                if (e) HIP_TRY(tm.mark(&(*e)[2 * NUM_CLS + 3]));
            }
            HIP_TRY(launch_hub_sweep(singleton, a, hubs.args, hs));
            if (e) HIP_TRY(tm.mark(&(*e)[2 * CLS_HUB + 1]));
        }
        if (e) HIP_TRY(tm.mark(&(*e)[2 * NUM_CLS + 1]));
        if (mark) {
            HIP_TRY(launch_mark_movers(ws.rows.as<int4>(), dec_all + start[CLS_L4], start[CLS_HUB] - start[CLS_L4], G.idx,
                                       mark, ctl, s));
            if (hubs.nhubs > 0) {
                a.dec = dec_all + start[CLS_HUB];
                HIP_TRY(launch_hub_mark(a, hubs.args, mark, s));
            }
        }
        if (!async) {  // asynchronous sweeps have moved already
            HIP_TRY(launch_apply(act_verts, dec_all + start[CLS_L4], active, G.k, a.gid, ws.comm.as<int32_t>(),
                                 mode == MODE_LPA ? nullptr : ws.sigma.as<int32_t>(), ctl, ws.gmoves.as<uint32_t>(),
                                 S, s));
            if (use_ec)
                HIP_TRY(launch_pairs_changed(active, nonhub, act_verts, G.off, ws.comm.as<int32_t>(),
                                             ws.sigma.as<int32_t>(), ws.cs.as<int2>(), ws.chg.as<uint8_t>(),
                                             ws.rlist.as<int4>(), ws.rcnt.as<int32_t>(), mode, ctl, s));
            else
                HIP_TRY(launch_pairs(active, act_verts, ws.comm.as<int32_t>(), ws.sigma.as<int32_t>(),
                                     ws.cs.as<int2>(), ctl, s));
        }
        // synchronous sweeps alternate direction, so a level ends after two
        // quiet sweeps; an asynchronous level ends after one (Alg. 2's test)
        HIP_TRY(launch_sweep_end(ctl, G.G, ws.gdone.as<int32_t>(), ws.gsweeps.as<int32_t>(),
                                 ws.gmoves.as<uint32_t>(), S, theta, async ? 1 : 2, ec_read_max, ec_fill_max, s));
        if (e) HIP_TRY(tm.mark(&(*e)[2 * NUM_CLS + 4]));
        if (use_ec) {  // rewrite the changed entries if the next sweep reads the cache
            HIP_TRY(launch_cache_refresh(active, ws.rlist.as<int4>(), ws.rcnt.as<int32_t>(), G.rev,
                                         ws.ce.as<int2>(), ctl, s));
            if (hubs.nhubs > 0) HIP_TRY(launch_hub_cache_refresh(a, hubs.args, ws.chg.as<uint8_t>() + nonhub, G.rev, s));
        }
        if (e) HIP_TRY(tm.mark(&(*e)[2 * NUM_CLS + 2]));
        return LV_OK;
    };
    const bool use_graph = !timing && !(p.flags & LV_NO_HIPGRAPH);
    // the sweeps' graph lives until the level's results are read back (one
    // stream synchronization per level); on an early return the stream is
    // drained before the graph is destroyed
    constexpr int POLL_LAG = 2;  // replays in flight while the host waits for the oldest
    struct GraphHolder {
        hipStream_t s;
        hipGraph_t gr = nullptr;
        hipGraphExec_t ex = nullptr;
        hipEvent_t ev[POLL_LAG] = {};
        ~GraphHolder()
        {
            if (ex || gr) (void)hipStreamSynchronize(s);
            if (ex) (void)hipGraphExecDestroy(ex);
            if (gr) (void)hipGraphDestroy(gr);
            for (hipEvent_t e : ev)
                if (e) (void)hipEventDestroy(e);
        }
    } held{s};
    const bool poll = use_graph && S > 2 && G.nnz >= ((int64_t)1 << 20);
    int32_t* h_flag = (int32_t*)((char*)g->pinned + poll_off);
    if (poll) {
        *h_flag = 0;
        for (hipEvent_t& e : held.ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    Timer ph;
    ph.s = s;
    hipEvent_t p0{}, p1{};
    if (use_graph) {
        // The first sweep (every community a single vertex) is launched
        // directly; while it runs, a later sweep is captured once and then
        // replayed up to max_sweeps - 1 times: the kernels read the sweep
        // counter and early-exit flag from the device.
        HIP_TRY(ph.mark(&p0));
        LV_TRY(launch_sweep(true, nullptr));
        if (S > 1) {
            hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) { set_error("hipStreamBeginCapture", e); return from_hip(e); }
            // On a large level each replay also copies the early-exit flag to
            // pinned memory, so that the host stops replaying once the level
            // has stopped (a stopped level's replays are launches that return
            // at once, about 0.2 ms each at R-MAT 24's size).
            lv_status st = launch_sweep(false, nullptr);
            if (st == LV_OK && poll) {
                const hipError_t ec = hipMemcpyAsync(h_flag, &ctl->all_done, sizeof(int32_t), hipMemcpyDeviceToHost, s);
                if (ec != hipSuccess) { set_error("hipMemcpyAsync", ec); st = from_hip(ec); }
            }
            e = hipStreamEndCapture(s, &held.gr);
            LV_TRY(st);
            if (e != hipSuccess) { set_error("hipStreamEndCapture", e); return from_hip(e); }
            e = hipGraphInstantiate(&held.ex, held.gr, nullptr, nullptr, 0);
            if (e != hipSuccess) { set_error("hipGraphInstantiate", e); return from_hip(e); }
            // with POLL_LAG replays queued, wait for the oldest and stop once it
            // found the level stopped: every later replay would return at once
            for (int32_t sw = 2, launched = 0; sw <= S; ++sw, ++launched) {
                if (poll && launched >= POLL_LAG) {
                    e = hipEventSynchronize(held.ev[launched % POLL_LAG]);
                    if (e != hipSuccess) { set_error("hipEventSynchronize", e); return from_hip(e); }
                    if (*(volatile int32_t*)h_flag) break;
                }
                e = hipGraphLaunch(held.ex, s);
                if (e != hipSuccess) { set_error("hipGraphLaunch", e); return from_hip(e); }
                if (poll) {
                    e = hipEventRecord(held.ev[launched % POLL_LAG], s);
                    if (e != hipSuccess) { set_error("hipEventRecord", e); return from_hip(e); }
                }
            }
        }
        HIP_TRY(ph.mark(&p1));
    } else {
        ev.resize(S);
        if (!timing) HIP_TRY(ph.mark(&p0));
        for (int32_t sw = 1; sw <= S; ++sw) LV_TRY(launch_sweep(sw == 1, timing ? &ev[sw - 1] : nullptr));
        if (!timing) HIP_TRY(ph.mark(&p1));
    }
    // LPA's commits leave the volumes alone (its scores never read them):
    // those of its final labels, for its modularity, are summed here
    if (mode == MODE_LPA && !async) {
        HIP_TRY(launch_fill_i32(ws.sigma.as<int32_t>(), 0, n, s));
        HIP_TRY(launch_volumes(act_verts, active, G.k, ws.comm.as<int32_t>(), ws.sigma.as<int32_t>(), s));
    }
    // per-graph sweep and move counts (one host round trip per level)
    uint32_t* h_moves = (uint32_t*)g->pinned;
    int32_t* h_sweeps = (int32_t*)(h_moves + (size_t)G.G * S);
    SweepCtl* h_ctl = (SweepCtl*)(((uintptr_t)(h_sweeps + G.G) + 15) & ~(uintptr_t)15);
    HIP_TRY(hipMemcpyAsync(h_moves, ws.gmoves.p, sizeof(uint32_t) * (size_t)G.G * S, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(h_sweeps, ws.gsweeps.p, sizeof(int32_t) * (size_t)G.G, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(h_ctl, ws.ctl.p, sizeof(SweepCtl), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    // every fallback scan of this level has run: a table its hubs used is
    // clean again (a level without hubs leaves the flag as it was)
    if (hubs.nhubs > 0) ws.hub_table_clean = true;
    if (!timing) out.sweep_ms = elapsed(p0, p1);
    out.cached_sweeps = use_ec ? h_ctl->ec_reads : 0;
    out.refreshed = use_ec ? (int64_t)h_ctl->refreshed : 0;
    out.ec_last = use_ec ? h_ctl->ec_last : EC_GATHER;
    out.moves.assign(h_moves, h_moves + (size_t)G.G * S);
    out.sweeps.assign(h_sweeps, h_sweeps + G.G);
    out.executed = 0;
    for (int32_t q = 0; q < G.G; ++q) out.executed = std::max(out.executed, out.sweeps[q]);
    // compulsory bytes of a sweep: 8 per CSR entry (index and weight) and 36
    // per vertex (offsets, label, degree and volume read; label and volume written)
    out.bytes = (8 * G.nnz + 36 * (int64_t)n) * out.executed;
    for (int32_t sw = 1; sw <= out.executed; ++sw) {
        const bool fused_sweep = fused && sw > 1 && fmap.nclass > 0;  // the classes below the hub class in one launch
        if (fused_sweep) {
            out.launches += 1;
            if (timing) {
                out.kern_ms[SLOT_FUSED] += elapsed(ev[sw - 1][2 * NUM_CLS + 5], ev[sw - 1][2 * NUM_CLS + 6]);
                out.kern_launches[SLOT_FUSED] += 1;
            }
        }
        for (int c = CLS_L4; c <= CLS_HUB; ++c) {
            const int32_t nv = start[c + 1] - start[c];
            if (nv == 0) continue;
            if (fused_sweep && c < CLS_HUB) {
                if (timing) out.kern_bytes[SLOT_FUSED] += 8 * cls_entries[c] + 36 * (int64_t)nv;
                continue;
            }
            out.launches += c == CLS_HUB ? (sw == 1 ? 2 : 2 + (hubs.args.bucketed && hubs.args.nsc > 0 ? 1 : 0) + (hubs.args.nins > 0 ? 3 : 0)) : 1;
            if (!timing) continue;
            const int slot = 2 * c + (sw == 1 ? 1 : 0) - 2;
            const std::vector<hipEvent_t>& E = ev[sw - 1];
            if (c == CLS_HUB && E[2 * NUM_CLS + 3]) {
                // the scatter pass reads the rows (the class's algorithmic bytes);
                // the partition workgroups read the buckets it wrote
                out.kern_ms[SLOT_HUB_SCATTER] += elapsed(E[2 * c], E[2 * NUM_CLS + 3]);
                out.kern_launches[SLOT_HUB_SCATTER] += 1;
                out.kern_bytes[SLOT_HUB_SCATTER] += 8 * cls_entries[c] + 36 * (int64_t)nv;
                out.kern_ms[slot] += elapsed(E[2 * NUM_CLS + 3], E[2 * c + 1]);
                out.kern_launches[slot] += 1;
                continue;
            }
            out.kern_ms[slot] += elapsed(E[2 * c], E[2 * c + 1]);
            out.kern_launches[slot] += 1;
            out.kern_bytes[slot] += 8 * cls_entries[c] + 36 * (int64_t)nv;
        }
        if (timing) {
            const std::vector<hipEvent_t>& E = ev[sw - 1];
            out.move_ms += elapsed(E[2 * NUM_CLS], E[2 * NUM_CLS + 1]);
            out.sweep_ms += elapsed(E[2 * NUM_CLS], E[2 * NUM_CLS + 2]);
            out.kern_ms[SLOT_COMMIT] += elapsed(E[2 * NUM_CLS + 1], E[2 * NUM_CLS + 4]);
            out.kern_launches[SLOT_COMMIT] += 1;
            if (use_ec) {
                out.kern_ms[SLOT_REFRESH] += elapsed(E[2 * NUM_CLS + 4], E[2 * NUM_CLS + 2]);
                out.kern_launches[SLOT_REFRESH] += 1;
            }
        }
    }
    return LV_OK;
}

// Renumber communities by smallest member (first occurrence) into ws.labels;
// n2 = communities; voff2[c] = first new label of graph c.
lv_status renumber(lv_graph* g, const LevelGraph& G, int32_t* n2, std::vector<int32_t>& voff2)
{
    Workspace& ws = g->ws;
    hipStream_t s = g->stream;
    const int32_t n = G.n;
    const size_t nb = sizeof(int32_t) * (size_t)(n + 1);
    HIP_TRY(ws.minv.ensure(nb));
    HIP_TRY(ws.flag.ensure(nb));
    HIP_TRY(ws.pos.ensure(nb));
    HIP_TRY(ws.labels.ensure(nb));
    HIP_TRY(ws.gmeta.ensure(sizeof(int32_t) * ((size_t)G.G + 1)));
    int32_t* pos = ws.pos.as<int32_t>();
    // pos[n] receives the total
    HIP_TRY(launch_renumber(n, ws.comm.as<int32_t>(), G.orig, ws.minv.as<int32_t>(), ws.flag.as<int32_t>(), pos,
                            ws.labels.as<int32_t>(), pos + n, ws.tmp.p, ws.tmp.cap, g->stream));
    // the new base of graph c is the number of communities before its first vertex
    std::vector<int32_t> at(G.voff.begin(), G.voff.end());
    HIP_TRY(hipMemcpyAsync(ws.gmeta.p, at.data(), sizeof(int32_t) * at.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(launch_gather_i32(pos, ws.gmeta.as<int32_t>(), G.G + 1, ws.gmeta.as<int32_t>(), s));
    voff2.resize(G.G + 1);
    LV_TRY(read_back(g, {{voff2.data(), ws.gmeta.p, sizeof(int32_t) * ((size_t)G.G + 1)}}));
    *n2 = voff2[G.G];
    return LV_OK;
}

struct Coarse {
    int32_t n2 = 0;
    int64_t nnz2 = 0;
    int32_t *off = nullptr, *idx = nullptr, *w = nullptr, *k = nullptr, *gid = nullptr;
    std::vector<int64_t> q_end;  // [G] Q_int of each graph's partition = M * Sigma_in - sum k'^2
    bool sorted = true;          // columns sorted within each row
};

// Aggregation (Algorithm 3): coarse CSR A' = S^T A S of the packed level into
// ping-pong slot `slot`, with each coarse vertex's graph and degree.
// Keys label(i) << colbits | label(j) of every CSR entry in ws.keys /
// ws.vals, *e1 = their number.  With `agg` equal keys are summed within tiles
// first and the tiles' distinct keys packed densely (the tiles' output goes
// to ws.keys_alt / ws.vals_alt first); else one key per entry.  ws.keys* must
// hold nnz items.
lv_status tile_keys(lv_graph* g, bool agg, int32_t n, const int32_t* off, const int32_t* idx, const int32_t* w,
                    int64_t nnz, const int32_t* labels, int colbits, const int32_t* gid, int64_t* sigma_in, int64_t* e1)
{
    Workspace& ws = g->ws;
    hipStream_t s = g->stream;
    const unsigned tiles = build_keys_tiles(n, nnz);
    if (!agg) {
        HIP_TRY(launch_build_keys(false, n, off, idx, w, nnz, labels, colbits, ws.keys.as<uint64_t>(),
                                  ws.vals.as<int32_t>(), nullptr, gid, sigma_in, s));
        *e1 = nnz;
        return LV_OK;
    }
    HIP_TRY(ws.tiles.ensure(sizeof(int32_t) * 5 * (size_t)tiles));
    HIP_TRY(ws.tmp.ensure(std::max(radix_tmp_bytes(nnz), scan_tmp_bytes(std::max<int64_t>(nnz, tiles), 8))));
    int32_t* meta = ws.tiles.as<int32_t>();
    int32_t* pos = meta + 4 * (size_t)tiles;
    int32_t* d_tot = (int32_t*)(ws.small.as<char>() + 2560);
    HIP_TRY(launch_build_keys(true, n, off, idx, w, nnz, labels, colbits, ws.keys_alt.as<uint64_t>(),
                              ws.vals_alt.as<int32_t>(), meta, gid, sigma_in, s));
    HIP_TRY(scan_exclusive_i32(meta, pos, tiles, d_tot, ws.tmp.p, ws.tmp.cap, s));
    int32_t tot = 0;
    SyncOnExit sync_tot{s};
    HIP_TRY(hipMemcpyAsync(&tot, d_tot, sizeof tot, hipMemcpyDeviceToHost, s));
    HIP_TRY(launch_compact_tiles(ws.keys_alt.as<uint64_t>(), ws.vals_alt.as<int32_t>(), meta, pos, tiles,
                                 ws.keys.as<uint64_t>(), ws.vals.as<int32_t>(), s));
    HIP_TRY(hipStreamSynchronize(s));
    *e1 = tot;
    return LV_OK;
}

// isolated: vertices without entries (each stays its own community), to
// judge how strongly the level merged.
// Aggregation by community: members' rows laid out by label, each coarse
// vertex's segment summed in LDS (segments of up to 8192 entries, by degree
// class) or sorted and reduced (longer ones), then packed into the coarse CSR
// of ping-pong slot `slot`.  d_sin[graph] += Sigma_in; *e2_out = coarse
// entries.  Uses ws.keys / ws.keys_alt (8 bytes per entry each) as staging.
lv_status aggregate_by_community(lv_graph* g, const LevelGraph& G, int32_t n2, int slot, int colbits, int32_t* gid2,
                                 int64_t* d_sin, int32_t* e2_out, const int32_t* bounds)
{
    Workspace& ws = g->ws;
    hipStream_t s = g->stream;
    const int32_t n = G.n;
    const int64_t E = G.nnz;
    const int32_t* labels = ws.labels.as<int32_t>();
    HIP_TRY(ws.tmp.ensure(std::max(radix_tmp_bytes(std::max<int64_t>(n, E)),
                                   scan_tmp_bytes(std::max<int64_t>(std::max<int64_t>(n, E), n2) + 1, 8))));
    // 1. positions grouped by label (stable: by position within a label)
    HIP_TRY(launch_copy_i32(ws.cls.as<int32_t>(), labels, n, s));
    HIP_TRY(launch_iota(ws.vert.as<int32_t>(), n, s));
    bool alt = false;
    HIP_TRY(radix_sort_u32(ws.cls.as<uint32_t>(), ws.vert.as<int32_t>(), ws.cls_alt.as<uint32_t>(),
                           ws.vert_alt.as<int32_t>(), n, colbits, ws.tmp.p, ws.tmp.cap, &alt, s));
    const uint32_t* lab_sorted = alt ? ws.cls_alt.as<uint32_t>() : ws.cls.as<uint32_t>();
    const int32_t* mem = alt ? ws.vert_alt.as<int32_t>() : ws.vert.as<int32_t>();
    // 2. entry offsets in member order, 3. each coarse vertex's segment
    HIP_TRY(ws.a_voff.ensure(sizeof(int32_t) * ((size_t)n + 1)));
    HIP_TRY(ws.a_seg.ensure(sizeof(int32_t) * ((size_t)n2 + 1)));
    int32_t* voff = ws.a_voff.as<int32_t>();
    int32_t* seg = ws.a_seg.as<int32_t>();
    HIP_TRY(launch_member_lengths(n, mem, G.off, voff, s));
    if (n > 0) HIP_TRY(scan_exclusive_i32(voff, voff, n, voff + n, ws.tmp.p, ws.tmp.cap, s));
    HIP_TRY(launch_segment_starts(n, lab_sorted, voff, n2, (int32_t)E, seg, s));
    // 4. staging: the members' rows, columns replaced by their labels
    int32_t* col = (int32_t*)ws.keys.p;
    int32_t* wt = G.w ? col + E : nullptr;
    int32_t* col2 = (int32_t*)ws.keys_alt.p;
    int32_t* wt2 = col2 + E;
    HIP_TRY(launch_perm_rows(n, voff, E, mem, G.off, G.idx, G.w, labels, col, wt, nullptr, nullptr, s));
    // 5. coarse vertices by segment length, with the local-moving classes'
    // bounds (the tuning's, never above a class's table)
    HIP_TRY(launch_classify(n2, seg, bounds, ws.cls.as<uint32_t>(), ws.vert.as<int32_t>(), s));
    HIP_TRY(radix_sort_u32(ws.cls.as<uint32_t>(), ws.vert.as<int32_t>(), ws.cls_alt.as<uint32_t>(),
                           ws.vert_alt.as<int32_t>(), n2, 8, ws.tmp.p, ws.tmp.cap, &alt, s));
    const uint32_t* cls_sorted = alt ? ws.cls_alt.as<uint32_t>() : ws.cls.as<uint32_t>();
    const int32_t* vsorted = alt ? ws.vert_alt.as<int32_t>() : ws.vert.as<int32_t>();
    int32_t* d_start = ws.small.as<int32_t>();
    HIP_TRY(launch_fill_i32(d_start, -1, NUM_CLS + 1, s));
    HIP_TRY(launch_class_starts(cls_sorted, n2, d_start, s));
    int32_t start[NUM_CLS + 1];
    LV_TRY(read_back(g, {{start, d_start, sizeof start}}));
    start[NUM_CLS] = n2;
    for (int c = NUM_CLS - 1; c >= 0; --c)
        if (start[c] < 0) start[c] = start[c + 1];
    // 6. segments of up to 8192 entries: summed in LDS
    HIP_TRY(ws.a_cnt.ensure(sizeof(int32_t) * ((size_t)n2 + 1)));
    int32_t* cnt = ws.a_cnt.as<int32_t>();
    HIP_TRY(launch_fill_i32(cnt, 0, (int64_t)n2 + 1, s));
    AggArgs aa{};
    aa.seg = seg;
    aa.col = col;
    aa.wt = wt;
    aa.col2 = col2;
    aa.wt2 = wt2;
    aa.cnt = cnt;
    aa.gid2 = gid2;
    aa.sigma_in = d_sin;
    for (int c = CLS_L4; c < CLS_HUB; ++c) {
        aa.verts = vsorted + start[c];
        aa.m = start[c + 1] - start[c];
        HIP_TRY(launch_agg_class(c, aa, s));
    }
    // 7. longer segments: keys sorted and reduced, placed at their segments
    const int32_t nh = n2 - start[CLS_HUB];
    if (nh > 0) {
        const int32_t* hv = vsorted + start[CLS_HUB];
        HIP_TRY(ws.a_hoff.ensure(sizeof(int32_t) * ((size_t)nh + 1)));
        int32_t* hoff = ws.a_hoff.as<int32_t>();
        HIP_TRY(launch_long_lengths(nh, hv, seg, hoff, s));
        HIP_TRY(scan_exclusive_i32(hoff, hoff, nh, hoff + nh, ws.tmp.p, ws.tmp.cap, s));
        int32_t eh = 0;
        LV_TRY(read_back(g, {{&eh, hoff + nh, sizeof eh}}));
        HIP_TRY(ws.h_keys.ensure(sizeof(uint64_t) * (size_t)std::max(eh, 1)));
        HIP_TRY(ws.h_keys_alt.ensure(sizeof(uint64_t) * (size_t)std::max(eh, 1)));
        HIP_TRY(ws.tmp.ensure(std::max(radix_tmp_bytes(eh), scan_tmp_bytes(eh, 8))));
        HIP_TRY(launch_long_keys(nh, hv, hoff, eh, seg, col, wt, colbits, ws.h_keys.as<uint64_t>(),
                                 ws.vals.as<int32_t>(), s));
        bool halt = false;
        HIP_TRY(radix_sort_u64(ws.h_keys.as<uint64_t>(), ws.vals.as<int32_t>(), ws.h_keys_alt.as<uint64_t>(),
                               ws.vals_alt.as<int32_t>(), eh, 2 * colbits, ws.tmp.p, ws.tmp.cap, &halt, s));
        const uint64_t* ks = halt ? ws.h_keys_alt.as<uint64_t>() : ws.h_keys.as<uint64_t>();
        const int32_t* vs = halt ? ws.vals_alt.as<int32_t>() : ws.vals.as<int32_t>();
        uint64_t* keys2 = halt ? ws.h_keys.as<uint64_t>() : ws.h_keys_alt.as<uint64_t>();
        int32_t* d_eu = (int32_t*)(ws.small.as<char>() + 2304);
        HIP_TRY(launch_segment_heads(ks, eh, ws.head.as<int32_t>(), s));
        HIP_TRY(scan_exclusive_i32(ws.head.as<int32_t>(), ws.head.as<int32_t>(), eh, d_eu, ws.tmp.p, ws.tmp.cap, s));
        int32_t eu = 0;
        LV_TRY(read_back(g, {{&eu, d_eu, sizeof eu}}));
        HIP_TRY(ws.h_col.ensure(sizeof(int32_t) * (size_t)std::max(eu, 1)));
        HIP_TRY(ws.h_wt.ensure(sizeof(int32_t) * (size_t)std::max(eu, 1)));
        HIP_TRY(ws.a_uoff.ensure(sizeof(int32_t) * ((size_t)n2 + 1)));
        HIP_TRY(hipMemsetAsync(ws.h_wt.p, 0, sizeof(int32_t) * (size_t)std::max(eu, 1), s));
        HIP_TRY(launch_segment_reduce(ks, vs, ws.head.as<int32_t>(), eh, colbits, ws.h_col.as<int32_t>(),
                                      ws.h_wt.as<int32_t>(), keys2, s));
        HIP_TRY(launch_row_offsets(keys2, eu, n2, colbits, ws.a_uoff.as<int32_t>(), s));
        HIP_TRY(launch_long_place(eu, keys2, ws.h_col.as<int32_t>(), ws.h_wt.as<int32_t>(), ws.a_uoff.as<int32_t>(),
                                  seg, colbits, col2, wt2, gid2, d_sin, s));
        HIP_TRY(launch_long_counts(nh, hv, ws.a_uoff.as<int32_t>(), cnt, s));
    }
    // 8. coarse row offsets and the packed rows
    int32_t* off2 = ws.g_off[slot].as<int32_t>();
    if (n2 > 0) HIP_TRY(scan_exclusive_i32(cnt, off2, n2, off2 + n2, ws.tmp.p, ws.tmp.cap, s));
    else HIP_TRY(launch_fill_i32(off2, 0, 1, s));
    int32_t e2 = 0;
    LV_TRY(read_back(g, {{&e2, off2 + n2, sizeof e2}}));
    HIP_TRY(ws.g_idx[slot].ensure(sizeof(int32_t) * (size_t)std::max(e2, 1)));
    HIP_TRY(ws.g_w[slot].ensure(sizeof(int32_t) * (size_t)std::max(e2, 1)));
    HIP_TRY(launch_pack_rows(n2, off2, e2, seg, col2, wt2, ws.g_idx[slot].as<int32_t>(), ws.g_w[slot].as<int32_t>(),
                             s));
    *e2_out = e2;
    return LV_OK;
}

// A level that merged weakly (at most 20 vertices with entries per
// community) is aggregated by community (lv_agg.hip), which leaves a coarse
// row's columns in table order; after a strong merge, or with by_sort, the
// entries' keys are sorted and reduced (summed within tiles first after a
// strong merge), which leaves them sorted.
lv_status aggregate(lv_graph* g, const LevelGraph& G, int32_t n2, int32_t isolated, int slot, Coarse& out,
                    bool by_sort = false, const int32_t* bounds = CLS_CAP)
{
    Workspace& ws = g->ws;
    hipStream_t s = g->stream;
    const int64_t E = G.nnz;
    const size_t E1 = (size_t)std::max<int64_t>(E, 1);
    const int colbits = bits_for(std::max<int64_t>(n2, 2));
    const int bits = 2 * colbits;
    HIP_TRY(ws.keys.ensure(sizeof(uint64_t) * E1));
    HIP_TRY(ws.keys_alt.ensure(sizeof(uint64_t) * E1));
    HIP_TRY(ws.vals.ensure(sizeof(int32_t) * E1));
    HIP_TRY(ws.vals_alt.ensure(sizeof(int32_t) * E1));
    HIP_TRY(ws.head.ensure(sizeof(int32_t) * E1));
    HIP_TRY(ws.tmp.ensure(std::max(radix_tmp_bytes(E), scan_tmp_bytes(std::max<int64_t>(E, n2 + 1), 8))));
    HIP_TRY(ws.g_off[slot].ensure(sizeof(int32_t) * ((size_t)n2 + 1)));
    HIP_TRY(ws.g_k[slot].ensure(sizeof(int32_t) * (size_t)std::max(n2, 1)));
    HIP_TRY(ws.g_gid[slot].ensure(sizeof(int32_t) * (size_t)std::max(n2, 1)));
    HIP_TRY(ws.gsum.ensure(sizeof(int64_t) * (size_t)G.G));
    HIP_TRY(ws.gsq.ensure(sizeof(int64_t) * (size_t)G.G));
    int64_t* d_sin = ws.gsum.as<int64_t>();
    int64_t* d_sq = ws.gsq.as<int64_t>();
    HIP_TRY(hipMemsetAsync(d_sin, 0, sizeof(int64_t) * (size_t)G.G, s));
    HIP_TRY(hipMemsetAsync(d_sq, 0, sizeof(int64_t) * (size_t)G.G, s));
    int32_t* gid2 = G.gid ? ws.g_gid[slot].as<int32_t>() : nullptr;
    HIP_TRY(launch_coarse_degree(G.n, ws.comm.as<int32_t>(), ws.labels.as<int32_t>(), ws.sigma.as<int32_t>(), G.gid,
                                 ws.g_k[slot].as<int32_t>(), gid2, s));
    HIP_TRY(launch_sum_sq(ws.g_k[slot].as<int32_t>(), n2, gid2, d_sq, s));
    // After a level that merged strongly (more than 20 vertices per community
    // with entries) most of a row's entries share a few keys: sum them within
    // tiles first, so that only the tiles' distinct keys are sorted.
    const bool agg = (int64_t)(n2 - isolated) * 20 < (int64_t)(G.n - isolated);
    if (!by_sort && !agg) {
        int32_t e2 = 0;
        LV_TRY(aggregate_by_community(g, G, n2, slot, colbits, gid2, d_sin, &e2, bounds));
        LV_TRY(ensure_pinned(g, std::max<size_t>(4096, 2 * sizeof(int64_t) * (size_t)G.G + 64)));
        int64_t* h_q = (int64_t*)g->pinned;
        HIP_TRY(hipMemcpyAsync(h_q, d_sin, sizeof(int64_t) * (size_t)G.G, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(h_q + G.G, d_sq, sizeof(int64_t) * (size_t)G.G, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        out.q_end.resize(G.G);
        for (int32_t c = 0; c < G.G; ++c) out.q_end[c] = G.Mh[c] * h_q[c] - h_q[G.G + c];
        out.n2 = n2;
        out.nnz2 = e2;
        out.off = ws.g_off[slot].as<int32_t>();
        out.idx = ws.g_idx[slot].as<int32_t>();
        out.w = ws.g_w[slot].as<int32_t>();
        out.k = ws.g_k[slot].as<int32_t>();
        out.gid = gid2;
        out.sorted = false;
        return LV_OK;
    }
    int64_t Ek = 0;
    LV_TRY(tile_keys(g, agg, G.n, G.off, G.idx, G.w, E, ws.labels.as<int32_t>(), colbits, G.gid, d_sin, &Ek));
    bool in_alt = false;
    HIP_TRY(radix_sort_u64(ws.keys.as<uint64_t>(), ws.vals.as<int32_t>(), ws.keys_alt.as<uint64_t>(),
                           ws.vals_alt.as<int32_t>(), Ek, bits, ws.tmp.p, ws.tmp.cap, &in_alt, s));
    const uint64_t* keys = in_alt ? ws.keys_alt.as<uint64_t>() : ws.keys.as<uint64_t>();
    const int32_t* vals = in_alt ? ws.vals_alt.as<int32_t>() : ws.vals.as<int32_t>();
    uint64_t* keys2 = in_alt ? ws.keys.as<uint64_t>() : ws.keys_alt.as<uint64_t>();  // the free sort buffer
    int32_t* d_e2 = (int32_t*)(ws.small.as<char>() + 2304);
    HIP_TRY(hipMemsetAsync(d_e2, 0, sizeof(int32_t), s));
    HIP_TRY(launch_segment_heads(keys, Ek, ws.head.as<int32_t>(), s));
    if (Ek > 0)
        HIP_TRY(scan_exclusive_i32(ws.head.as<int32_t>(), ws.head.as<int32_t>(), Ek, d_e2, ws.tmp.p, ws.tmp.cap, s));
    LV_TRY(ensure_pinned(g, std::max<size_t>(4096, 2 * sizeof(int64_t) * (size_t)G.G + 64)));
    int64_t* h_q = (int64_t*)g->pinned;
    HIP_TRY(hipMemcpyAsync(h_q, d_sin, sizeof(int64_t) * (size_t)G.G, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(h_q + G.G, d_sq, sizeof(int64_t) * (size_t)G.G, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(h_q + 2 * G.G, d_e2, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    int32_t e2 = 0;
    std::memcpy(&e2, h_q + 2 * G.G, sizeof e2);
    if (E == 0) e2 = 0;
    out.q_end.resize(G.G);
    for (int32_t c = 0; c < G.G; ++c) out.q_end[c] = G.Mh[c] * h_q[c] - h_q[G.G + c];
    HIP_TRY(ws.g_idx[slot].ensure(sizeof(int32_t) * (size_t)std::max(e2, 1)));
    HIP_TRY(ws.g_w[slot].ensure(sizeof(int32_t) * (size_t)std::max(e2, 1)));
    int32_t* off2 = ws.g_off[slot].as<int32_t>();
    HIP_TRY(hipMemsetAsync(ws.g_w[slot].p, 0, sizeof(int32_t) * (size_t)std::max(e2, 1), s));
    HIP_TRY(launch_segment_reduce(keys, vals, ws.head.as<int32_t>(), Ek, colbits, ws.g_idx[slot].as<int32_t>(),
                                  ws.g_w[slot].as<int32_t>(), keys2, s));
    HIP_TRY(launch_row_offsets(keys2, e2, n2, colbits, off2, s));
    out.n2 = n2;
    out.nnz2 = e2;
    out.off = off2;
    out.idx = ws.g_idx[slot].as<int32_t>();
    out.w = ws.g_w[slot].as<int32_t>();
    out.k = ws.g_k[slot].as<int32_t>();
    out.gid = gid2;
    out.sorted = true;
    return LV_OK;
}

// Entry offsets of the graphs of a packed CSR: eoff[c] = off[voff[c]].
lv_status graph_entry_offsets(lv_graph* g, const int32_t* off, const std::vector<int32_t>& voff,
                              std::vector<int64_t>& eoff)
{
    Workspace& ws = g->ws;
    hipStream_t s = g->stream;
    const int32_t m = (int32_t)voff.size();
    HIP_TRY(ws.gmeta.ensure(sizeof(int32_t) * (size_t)m));
    HIP_TRY(hipMemcpyAsync(ws.gmeta.p, voff.data(), sizeof(int32_t) * (size_t)m, hipMemcpyHostToDevice, s));
    HIP_TRY(launch_gather_i32(off, ws.gmeta.as<int32_t>(), m, ws.gmeta.as<int32_t>(), s));
    std::vector<int32_t> e(m);
    LV_TRY(read_back(g, {{e.data(), ws.gmeta.p, sizeof(int32_t) * (size_t)m}}));
    eoff.assign(e.begin(), e.end());
    return LV_OK;
}

// Next level's packed graph from the coarse one, keeping only the graphs in
// `keep` (coarse slots, increasing): their segments are copied, in order,
// into ping-pong slot `dst`.
lv_status repack(lv_graph* g, const Coarse& co, const std::vector<int32_t>& voff2, const std::vector<int64_t>& eoff2,
                 const std::vector<int32_t>& keep, int dst, LevelGraph& next)
{
    Workspace& ws = g->ws;
    hipStream_t s = g->stream;
    std::vector<RepackSeg> segs;
    int32_t nv = 0;
    int64_t ne = 0;
    next.voff.assign(1, 0);
    for (int32_t c : keep) {
        RepackSeg q{};
        q.src_off = co.off;
        q.src_idx = co.idx;
        q.src_w = co.w;
        q.src_k = co.k;
        q.src_vb = voff2[c];
        q.n = voff2[c + 1] - voff2[c];
        q.dst_vb = nv;
        q.dst_eb = ne;
        segs.push_back(q);
        nv += q.n;
        ne += eoff2[c + 1] - eoff2[c];
        next.voff.push_back(nv);
    }
    HIP_TRY(ws.segs.ensure(sizeof(RepackSeg) * segs.size()));
    SyncOnExit sync_segs{s};
    HIP_TRY(hipMemcpyAsync(ws.segs.p, segs.data(), sizeof(RepackSeg) * segs.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(ws.g_off[dst].ensure(sizeof(int32_t) * ((size_t)nv + 1)));
    HIP_TRY(ws.g_idx[dst].ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(ne, 1)));
    HIP_TRY(ws.g_w[dst].ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(ne, 1)));
    HIP_TRY(ws.g_k[dst].ensure(sizeof(int32_t) * (size_t)std::max(nv, 1)));
    HIP_TRY(ws.g_gid[dst].ensure(sizeof(int32_t) * (size_t)std::max(nv, 1)));
    HIP_TRY(launch_repack(ws.segs.as<RepackSeg>(), (int32_t)segs.size(), nv, ne, ws.g_off[dst].as<int32_t>(),
                          ws.g_idx[dst].as<int32_t>(), ws.g_w[dst].as<int32_t>(), ws.g_k[dst].as<int32_t>(),
                          ws.g_gid[dst].as<int32_t>(), nullptr, s));
    HIP_TRY(hipStreamSynchronize(s));  // the host segment list must outlive the copy
    next.n = nv;
    next.nnz = ne;
    next.off = ws.g_off[dst].as<int32_t>();
    next.idx = ws.g_idx[dst].as<int32_t>();
    next.w = ws.g_w[dst].as<int32_t>();
    next.k = ws.g_k[dst].as<int32_t>();
    next.G = (int32_t)keep.size();
    next.gid = next.G > 1 ? ws.g_gid[dst].as<int32_t>() : nullptr;
    return LV_OK;
}

// Upload per-graph M of a level (several graphs) to the device.
lv_status upload_M(lv_graph* g, DevBuf& buf, LevelGraph& G)
{
    G.M = G.Mh.empty() ? 0 : G.Mh[0];
    if (G.G <= 1) { G.Mg = nullptr; return LV_OK; }
    HIP_TRY(buf.ensure(sizeof(int64_t) * (size_t)G.G));
    HIP_TRY(hipMemcpyAsync(buf.p, G.Mh.data(), sizeof(int64_t) * (size_t)G.G, hipMemcpyHostToDevice, g->stream));
    HIP_TRY(hipStreamSynchronize(g->stream));
    G.Mg = buf.as<int64_t>();
    return LV_OK;
}

LevelGraph level0(lv_graph* g)
{
    LevelGraph G;
    G.n = g->n;
    G.nnz = g->nnz;
    G.off = g->off.as<int32_t>();
    G.idx = g->idx.as<int32_t>();
    G.w = g->weighted ? g->w.as<int32_t>() : nullptr;
    G.k = g->k.as<int32_t>();
    G.G = g->G;
    G.gid = g->G > 1 ? g->d_gid.as<int32_t>() : nullptr;
    G.Mg = g->G > 1 ? g->d_M.as<int64_t>() : nullptr;
    G.M = g->M[0];
    G.voff = g->voff;
    G.Mh = g->M;
    G.orig = g->reordered ? g->orig.as<int32_t>() : nullptr;
    G.rev = g->has_rev ? g->rev.as<int32_t>() : nullptr;
    return G;
}

// Autotuner: coordinate descent over the tuning knobs; each candidate is timed
// on the level-0 graph (a first sweep and two later sweeps, HIP events) and
// scored as the time of a whole level of max_sweeps sweeps.  Settings only
// choose which kernel handles which vertex, never the result.
lv_status autotune(lv_graph* g, const Params& base, lv_tuning* best, double* best_ms)
{
    *best = lv_tuning{};
    *best_ms = 0.0;
    if (g->n == 0 || g->nnz == 0) return LV_OK;
    auto cost = [&](const lv_tuning& t, double* ms) -> lv_status {
        Params p = base;
        p.max_sweeps = std::min(3, base.max_sweeps);
        p.flags = LV_TIMING | LV_NO_CACHE;  // the class kernels alone, each sweep gathering
        p.tune = make_tune(&t);
        SweepOut so;
        const LevelGraph G = level0(g);
        LV_TRY(run_sweeps(g, G, MODE_LOUVAIN, p, nullptr, so));
        double first = 0.0, later = 0.0;
        for (int q = 0; q < LV_KERNEL_SLOTS; ++q) {  // the move kernels (not the commit or the cache)
            if (q == SLOT_COMMIT || q == SLOT_REFRESH) continue;
            if (q < 2 * (NUM_CLS - 1) && (q & 1)) first += so.kern_ms[q];
            else later += so.kern_ms[q];
        }
        const int32_t nl = std::max(1, so.executed - 1);
        *ms = first + later / nl * std::max(0, base.max_sweeps - 1);
        return LV_OK;
    };
    double cur = 0.0;
    LV_TRY(cost(*best, &cur));
    struct Knob { int32_t lv_tuning::*field; std::vector<int32_t> values; };
    const std::vector<Knob> knobs = {
        {&lv_tuning::sub_max, {32, 8}},
        {&lv_tuning::wave_max, {128}},
        {&lv_tuning::block_max, {3072, 2048}},
        {&lv_tuning::hub_mode, {1}},
        {&lv_tuning::part_keys, {768, 1536}},
        {&lv_tuning::hub_chunk, {1024, 4096}},
        {&lv_tuning::part_slots, {1024}},
        {&lv_tuning::table_pct, {150, 200, 400}},
        {&lv_tuning::fused, {1}},
    };
    for (const Knob& kb : knobs) {
        lv_tuning keep = *best;
        for (int32_t v : kb.values) {
            lv_tuning t = *best;
            t.*(kb.field) = v;
            if (kb.field == &lv_tuning::part_keys && t.hub_mode == 1) t.part_keys = v * 8;  // compact tables are 8x larger
            double ms = 0.0;
            LV_TRY(cost(t, &ms));
            if (ms < cur * 0.98) { cur = ms; keep = t; }
        }
        *best = keep;
    }
    *best_ms = cur;
    return LV_OK;
}

// The tuning a call runs with: the caller's, else (LV_AUTOTUNE) the handle's
// autotuned setting, chosen on first use, else the defaults.
lv_status resolve_tuning(lv_graph* g, const lv_params* params, Params& p)
{
    if (!params || params->tuning || !(params->flags & LV_AUTOTUNE)) return LV_OK;
    if (!g->has_tuned) {
        double ms = 0.0;
        LV_TRY(autotune(g, p, &g->tuned, &ms));
        g->has_tuned = true;
    }
    p.tune = make_tune(&g->tuned);
    return LV_OK;
}

void fill_info(lv_level_info& li, const SweepOut& so, int32_t c, int32_t S)
{
    li.sweeps = so.sweeps[c];
    li.move_ms = so.move_ms;
    li.sweep_ms = so.sweep_ms;
    li.move_launches = so.launches;
    li.move_bytes = so.bytes;
    for (int t = 0; t < LV_KERNEL_SLOTS; ++t) {
        li.kern_ms[t] = so.kern_ms[t];
        li.kern_launches[t] = so.kern_launches[t];
        li.kern_bytes[t] = so.kern_bytes[t];
    }
    li.cached_sweeps = so.cached_sweeps;
    li.refreshed_entries = so.refreshed;
    (void)S;
}

// Multi-level Louvain (Algorithm 3) for every graph of the handle.
// Storage by descending number of entries within each packed graph (the
// graph id is the major key, so every graph keeps its vertex range): orig[p]
// = the vertex stored at position p, inv its inverse; the rows, weights (w
// may be null) and degrees permuted into off2 / idx2 / w2 / k2, column
// indices mapped to positions.  Sorts in ws.keys* / ws.vals*.
lv_status degree_order(lv_graph* g, int32_t n, int64_t nnz, const int32_t* off, const int32_t* idx, const int32_t* w,
                       const int32_t* k, const int32_t* gid, int32_t G, DevBuf& orig, DevBuf& inv, DevBuf& off2,
                       DevBuf& idx2, DevBuf& w2, DevBuf& k2, const int32_t* rank = nullptr, DevBuf* rev2 = nullptr)
{
    Workspace& ws = g->ws;
    hipStream_t s = g->stream;
    HIP_TRY(ws.small.ensure(4096));
    int32_t* d_max = (int32_t*)(ws.small.as<char>() + 3584);
    HIP_TRY(hipMemsetAsync(d_max, 0, sizeof(int32_t), s));
    HIP_TRY(launch_max_degree(n, off, d_max, s));
    int32_t maxdeg = 0;
    LV_TRY(read_back(g, {{&maxdeg, d_max, sizeof maxdeg}}));
    const int db = bits_for((int64_t)maxdeg + 1);
    const int bits = db + (G > 1 ? bits_for(G) : 0);
    const size_t nb = sizeof(int32_t) * (size_t)n;
    HIP_TRY(ws.keys.ensure(2 * nb));
    HIP_TRY(ws.keys_alt.ensure(2 * nb));
    HIP_TRY(ws.vals.ensure(nb));
    HIP_TRY(ws.vals_alt.ensure(nb));
    HIP_TRY(ws.tmp.ensure(std::max(radix_tmp_bytes(n), scan_tmp_bytes((int64_t)n + 1, 8))));
    HIP_TRY(launch_degree_keys(n, off, gid, maxdeg, db, ws.keys.as<uint64_t>(), ws.vals.as<int32_t>(), s));
    bool in_alt = false;
    HIP_TRY(radix_sort_u64(ws.keys.as<uint64_t>(), ws.vals.as<int32_t>(), ws.keys_alt.as<uint64_t>(),
                           ws.vals_alt.as<int32_t>(), n, bits, ws.tmp.p, ws.tmp.cap, &in_alt, s));
    HIP_TRY(orig.ensure(nb));
    HIP_TRY(inv.ensure(nb));
    HIP_TRY(launch_copy_i32(orig.as<int32_t>(), in_alt ? ws.vals_alt.as<int32_t>() : ws.vals.as<int32_t>(), n, s));
    HIP_TRY(launch_inverse(orig.as<int32_t>(), n, inv.as<int32_t>(), s));
    HIP_TRY(off2.ensure(sizeof(int32_t) * ((size_t)n + 1)));
    HIP_TRY(idx2.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(nnz, 1)));
    if (w) HIP_TRY(w2.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(nnz, 1)));
    HIP_TRY(k2.ensure(nb));
    HIP_TRY(launch_perm_lengths(orig.as<int32_t>(), n, off, off2.as<int32_t>(), s));
    HIP_TRY(scan_exclusive_i32(off2.as<int32_t>(), off2.as<int32_t>(), n, off2.as<int32_t>() + n, ws.tmp.p, ws.tmp.cap, s));
    if (rank) HIP_TRY(rev2->ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(nnz, 1)));
    HIP_TRY(launch_perm_rows(n, off2.as<int32_t>(), nnz, orig.as<int32_t>(), off, idx, w, inv.as<int32_t>(),
                             idx2.as<int32_t>(), w ? w2.as<int32_t>() : nullptr, rank,
                             rank ? rev2->as<int32_t>() : nullptr, s));
    HIP_TRY(launch_gather_i32(k, orig.as<int32_t>(), n, k2.as<int32_t>(), s));
    HIP_TRY(hipStreamSynchronize(s));
    return LV_OK;
}

// Sort the columns within every row of a device CSR in place (weights
// follow); uses ws.keys* / ws.vals* (at least nnz items each).
lv_status sort_rows(lv_graph* g, int32_t n, int64_t nnz, const int32_t* off, int32_t* idx, int32_t* w)
{
    if (n <= 0 || nnz <= 1) return LV_OK;
    Workspace& ws = g->ws;
    hipStream_t s = g->stream;
    const int cb = bits_for(std::max<int64_t>(n, 2));
    HIP_TRY(ws.keys.ensure(sizeof(uint64_t) * (size_t)nnz));
    HIP_TRY(ws.keys_alt.ensure(sizeof(uint64_t) * (size_t)nnz));
    HIP_TRY(ws.vals.ensure(sizeof(int32_t) * (size_t)nnz));
    HIP_TRY(ws.vals_alt.ensure(sizeof(int32_t) * (size_t)nnz));
    HIP_TRY(ws.tmp.ensure(radix_tmp_bytes(nnz)));
    HIP_TRY(launch_row_keys(n, off, nnz, idx, w, cb, ws.keys.as<uint64_t>(), ws.vals.as<int32_t>(), s));
    bool alt = false;
    HIP_TRY(radix_sort_u64(ws.keys.as<uint64_t>(), ws.vals.as<int32_t>(), ws.keys_alt.as<uint64_t>(),
                           ws.vals_alt.as<int32_t>(), nnz, 2 * cb, ws.tmp.p, ws.tmp.cap, &alt, s));
    HIP_TRY(launch_unpack_keys(nnz, alt ? ws.keys_alt.as<uint64_t>() : ws.keys.as<uint64_t>(),
                               alt ? ws.vals_alt.as<int32_t>() : ws.vals.as<int32_t>(), cb, idx, w, s));
    return LV_OK;
}

lv_status louvain_impl(lv_graph* g, const Params& p, bool keep_graphs, lv_result* r)
{
    hipStream_t s = g->stream;
    Workspace& ws = g->ws;
    const int32_t G0 = g->G, S = p.max_sweeps;
    r->G = G0;
    r->n0 = g->n;
    r->graphs.resize(G0);
    for (int32_t q = 0; q < G0; ++q) {
        GraphResult& gr = r->graphs[q];
        gr.n0 = g->voff[q + 1] - g->voff[q];
        gr.fin_base = g->voff[q];
        gr.M = g->M[q];
        gr.q_int = g->q0[q];
    }
    HIP_TRY(pool_take(g->pool, sizeof(int32_t) * (size_t)std::max(g->n, 1), r->final_labels));
    // final labels start as each vertex's index within its graph
    {
        HIP_TRY(ws.gmeta.ensure(sizeof(int32_t) * ((size_t)G0 + 1)));
        HIP_TRY(hipMemcpyAsync(ws.gmeta.p, g->voff.data(), sizeof(int32_t) * ((size_t)G0 + 1), hipMemcpyHostToDevice, s));
        // (a graph that accepts no level keeps the singleton partition in id order)
        HIP_TRY(launch_iota(r->final_labels.i32(), g->n, s));
        HIP_TRY(launch_local_labels(g->n, r->final_labels.i32(), G0 > 1 ? g->d_gid.as<int32_t>() : nullptr,
                                    ws.gmeta.as<int32_t>(), r->final_labels.i32(), s));
    }
    LevelGraph G = level0(g);
    std::vector<int64_t> eoff = g->eoff;
    std::vector<int32_t> orig(G0);
    for (int32_t q = 0; q < G0; ++q) orig[q] = q;
    std::vector<int64_t> qstart = g->q0;
    DevBuf Mbuf;
    int slot = 0;
    Timer tm;
    tm.on = true;  // phase times (renumber, aggregate) are always measured
    tm.s = s;
    for (;;) {
        SweepOut so;
        LV_TRY(run_sweeps(g, G, MODE_LOUVAIN, p, nullptr, so));
        hipEvent_t t0{}, t1{}, t2{};
        if (tm.on) HIP_TRY(tm.mark(&t0));
        int32_t n2 = 0;
        std::vector<int32_t> voff2;
        LV_TRY(renumber(g, G, &n2, voff2));
        if (tm.on) HIP_TRY(tm.mark(&t1));
        Coarse co;
        LV_TRY(aggregate(g, G, n2, so.isolated, slot, co, p.tune.agg_sort != 0, p.tune.bounds));
        std::vector<int64_t> eoff2;
        LV_TRY(graph_entry_offsets(g, co.off, voff2, eoff2));
        double ren_ms = 0, agg_ms = 0;
        if (tm.on) {
            HIP_TRY(tm.mark(&t2));
            HIP_TRY(hipStreamSynchronize(s));
            ren_ms = elapsed(t0, t1);
            agg_ms = elapsed(t1, t2);
            tm.used = 0;
        }
        // per-graph acceptance
        std::vector<int32_t> acc(G.G, 0), keep;
        bool any = false;
        for (int32_t c = 0; c < G.G; ++c) {
            acc[c] = co.q_end[c] > qstart[c] ? 1 : 0;
            any = any || acc[c];
        }
        std::shared_ptr<LabelStore> store;
        if (any) {
            store = std::make_shared<LabelStore>();
            store->n = G.n;
            HIP_TRY(pool_take(g->pool, sizeof(int32_t) * (size_t)std::max(G.n, 1), store->labels));
            if (G.orig)  // kept in vertex-id order
                HIP_TRY(launch_scatter_i32(ws.labels.as<int32_t>(), G.orig, G.n, store->labels.i32(), s));
            else
                HIP_TRY(launch_copy_i32(store->labels.i32(), ws.labels.as<int32_t>(), G.n, s));
        }
        for (int32_t c = 0; c < G.G; ++c) {
            GraphResult& gr = r->graphs[orig[c]];
            LevelRecord rec;
            lv_level_info& li = rec.info;
            li.n = G.voff[c + 1] - G.voff[c];
            li.n_next = voff2[c + 1] - voff2[c];
            li.nnz = eoff[c + 1] - eoff[c];
            li.q_start = qstart[c];
            li.q_end = co.q_end[c];
            li.accepted = acc[c];
            li.renumber_ms = ren_ms;
            li.aggregate_ms = agg_ms;
            fill_info(li, so, c, S);
            rec.moves.assign(so.moves.begin() + (size_t)c * S, so.moves.begin() + (size_t)c * S + so.sweeps[c]);
            if (acc[c]) {
                rec.store = store;
                rec.vbase = G.voff[c];
                rec.nbase = voff2[c];
                gr.q_int = co.q_end[c];
                ++gr.accepted;
                if (keep_graphs && G0 == 1) {
                    if (!co.sorted) LV_TRY(sort_rows(g, co.n2, co.nnz2, co.off, co.idx, co.w));
                    rec.g_off = std::make_shared<DevBuf>();
                    rec.g_idx = std::make_shared<DevBuf>();
                    rec.g_w = std::make_shared<DevBuf>();
                    HIP_TRY(rec.g_off->ensure(sizeof(int32_t) * ((size_t)co.n2 + 1)));
                    HIP_TRY(rec.g_idx->ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(co.nnz2, 1)));
                    HIP_TRY(rec.g_w->ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(co.nnz2, 1)));
                    HIP_TRY(launch_copy_i32(rec.g_off->as<int32_t>(), co.off, (int64_t)co.n2 + 1, s));
                    HIP_TRY(launch_copy_i32(rec.g_idx->as<int32_t>(), co.idx, co.nnz2, s));
                    HIP_TRY(launch_copy_i32(rec.g_w->as<int32_t>(), co.w, co.nnz2, s));
                    rec.g_nnz = co.nnz2;
                }
                if (gr.accepted < p.max_levels) keep.push_back(c);
            }
            gr.levels.push_back(std::move(rec));
        }
        // compose the final labels of the graphs that accepted this level, with
        // the level's labels in vertex-id order (the store's copy when the
        // level is stored by degree)
        if (any) {
            const int32_t* lab_id = G.orig ? store->labels.i32() : ws.labels.as<int32_t>();
            if (G0 == 1) {
                HIP_TRY(launch_compose(g->n, r->final_labels.i32(), lab_id, nullptr, nullptr, nullptr, nullptr, s));
            } else {
                std::vector<int32_t> meta((size_t)G0 + 2 * (size_t)G.G, -1);
                for (int32_t c = 0; c < G.G; ++c) {
                    if (acc[c]) meta[orig[c]] = c;
                    meta[G0 + c] = G.voff[c];
                    meta[G0 + G.G + c] = voff2[c];
                }
                HIP_TRY(ws.gmeta.ensure(sizeof(int32_t) * meta.size()));
                HIP_TRY(hipMemcpyAsync(ws.gmeta.p, meta.data(), sizeof(int32_t) * meta.size(), hipMemcpyHostToDevice, s));
                HIP_TRY(launch_compose(g->n, r->final_labels.i32(), lab_id,
                                       g->d_gid.as<int32_t>(), ws.gmeta.as<int32_t>(), ws.gmeta.as<int32_t>() + G0,
                                       ws.gmeta.as<int32_t>() + G0 + G.G, s));
                HIP_TRY(hipStreamSynchronize(s));
            }
        }
        if (keep.empty()) break;
        LevelGraph next;
        std::vector<int32_t> orig2;
        std::vector<int64_t> q2, eoff_next;
        for (int32_t c : keep) {
            orig2.push_back(orig[c]);
            q2.push_back(co.q_end[c]);
            next.Mh.push_back(G.Mh[c]);
        }
        if ((int32_t)keep.size() == G.G) {
            next.n = co.n2;
            next.nnz = co.nnz2;
            next.off = co.off;
            next.idx = co.idx;
            next.w = co.w;
            next.k = co.k;
            next.G = G.G;
            next.gid = G.G > 1 ? co.gid : nullptr;
            next.voff = voff2;
            eoff_next = eoff2;
            slot ^= 1;
        } else {
            LV_TRY(repack(g, co, voff2, eoff2, keep, slot ^ 1, next));
            eoff_next.assign(1, 0);
            for (int32_t c : keep) eoff_next.push_back(eoff_next.back() + (eoff2[c + 1] - eoff2[c]));
        }
        LV_TRY(upload_M(g, Mbuf, next));
        if (next.nnz >= p.tune.order_min && next.n >= 2) {
            // store a large coarse level by degree too (ids stay the coarse ids)
            LV_TRY(degree_order(g, next.n, next.nnz, next.off, next.idx, next.w, next.k, next.gid, next.G, ws.p_orig,
                                ws.p_inv, ws.p_off, ws.p_idx, ws.p_w, ws.p_k));
            next.off = ws.p_off.as<int32_t>();
            next.idx = ws.p_idx.as<int32_t>();
            next.w = next.w ? ws.p_w.as<int32_t>() : nullptr;
            next.k = ws.p_k.as<int32_t>();
            next.orig = ws.p_orig.as<int32_t>();
        }
        G = std::move(next);
        eoff = std::move(eoff_next);
        orig = std::move(orig2);
        qstart = std::move(q2);
    }
    HIP_TRY(hipStreamSynchronize(s));
    return LV_OK;
}

lv_status copy_out(int32_t* dst, const int32_t* src_dev, int64_t count, lv_memkind kind, hipStream_t s)
{
    if (count <= 0) return LV_OK;
    HIP_TRY(hipMemcpyAsync(dst, src_dev, sizeof(int32_t) * (size_t)count,
                           kind == LV_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    return LV_OK;
}

// LPA (Algorithm 1) as one level of synchronous sweeps for every graph of the
// handle; labels (numbered within each graph) into ws.labels' slot `out`.
lv_status lpa_impl(lv_graph* g, const Params& p, int32_t* out_dev, SweepOut& so, std::vector<int32_t>& voff2,
                   std::vector<int64_t>& q_int, double* ren_ms)
{
    Workspace& ws = g->ws;
    hipStream_t s = g->stream;
    LevelGraph G = level0(g);
    LV_TRY(run_sweeps(g, G, MODE_LPA, p, nullptr, so));
    Timer tm;
    tm.on = true;
    tm.s = s;
    hipEvent_t t0{}, t1{};
    if (tm.on) HIP_TRY(tm.mark(&t0));
    int32_t n2 = 0;
    LV_TRY(renumber(g, G, &n2, voff2));
    if (tm.on) HIP_TRY(tm.mark(&t1));
    // Q_int of each graph's partition: M * Sigma_in - sum of its community volumes squared
    HIP_TRY(ws.gsum.ensure(sizeof(int64_t) * (size_t)G.G));
    HIP_TRY(ws.gsq.ensure(sizeof(int64_t) * (size_t)G.G));
    HIP_TRY(hipMemsetAsync(ws.gsum.p, 0, sizeof(int64_t) * (size_t)G.G, s));
    HIP_TRY(hipMemsetAsync(ws.gsq.p, 0, sizeof(int64_t) * (size_t)G.G, s));
    // One graph whose last sweep read or filled the entry cache and moved no
    // vertex: the cache holds every entry's neighbour label of the final
    // labels, so Sigma_in streams it (plus the loops) instead of gathering.
    const bool cached = G.G == 1 && (int64_t)g->trace.size() == 1 && so.sweeps[0] >= 1 &&
                        (so.ec_last == EC_READ || so.ec_last == EC_FILL) && so.moves[(size_t)so.sweeps[0] - 1] == 0;
    if (cached)
        HIP_TRY(launch_sigma_in_cached(G.n, G.off, ws.ce.as<int2>(), G.w, G.nnz, ws.comm.as<int32_t>(),
                                       ws.gsum.as<int64_t>(), s));
    else
        HIP_TRY(launch_sigma_in(G.n, G.off, G.idx, G.w, G.nnz, ws.comm.as<int32_t>(), G.gid, ws.gsum.as<int64_t>(), s));
    HIP_TRY(launch_sum_sq(ws.sigma.as<int32_t>(), G.n, G.gid, ws.gsq.as<int64_t>(), s));
    std::vector<int64_t> sin(G.G), sq(G.G);
    SyncOnExit sync_sums{s};
    HIP_TRY(hipMemcpyAsync(sin.data(), ws.gsum.p, sizeof(int64_t) * (size_t)G.G, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(sq.data(), ws.gsq.p, sizeof(int64_t) * (size_t)G.G, hipMemcpyDeviceToHost, s));
    // labels numbered within each graph
    HIP_TRY(ws.gmeta.ensure(sizeof(int32_t) * ((size_t)G.G + 1)));
    HIP_TRY(hipMemcpyAsync(ws.gmeta.p, voff2.data(), sizeof(int32_t) * ((size_t)G.G + 1), hipMemcpyHostToDevice, s));
    if (G.orig) {  // vertex-id order
        HIP_TRY(launch_local_labels(G.n, ws.labels.as<int32_t>(), G.gid, ws.gmeta.as<int32_t>(), ws.pos.as<int32_t>(), s));
        HIP_TRY(launch_scatter_i32(ws.pos.as<int32_t>(), G.orig, G.n, out_dev, s));
    } else {
        HIP_TRY(launch_local_labels(G.n, ws.labels.as<int32_t>(), G.gid, ws.gmeta.as<int32_t>(), out_dev, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    if (cached) sin[0] += g->trace[0];
    q_int.resize(G.G);
    for (int32_t c = 0; c < G.G; ++c) q_int[c] = G.Mh[c] * sin[c] - sq[c];
    *ren_ms = tm.on ? elapsed(t0, t1) : 0.0;
    return LV_OK;
}

}  // namespace

// ============================================================================ ABI
extern "C" {

void lv_params_default(lv_params* p)
{
    if (!p) return;
    p->max_sweeps = 20;
    p->max_levels = 32;
    p->lpa_threshold = 0;
    p->flags = 0;
    p->tuning = nullptr;
}

const char* lv_status_str(lv_status s)
{
    switch (s) {
    case LV_OK: return "ok";
    case LV_E_ARG: return "invalid argument";
    case LV_E_CSR: return "malformed CSR";
    case LV_E_ASYMMETRIC: return "asymmetric graph";
    case LV_E_WEIGHT: return "weight < 1";
    case LV_E_OVERFLOW: return "total volume or size exceeds 2^31";
    case LV_E_NOMEM: return "out of device memory";
    case LV_E_HIP: return "HIP runtime error";
    case LV_E_BUSY: return "busy";
    case LV_E_TOO_LARGE: return "job exceeds the memory budget";
    case LV_E_CANCELLED: return "cancelled";
    case LV_E_STATE: return "invalid state";
    case LV_E_NOT_FOUND: return "not found";
    }
    return "unknown status";
}

const char* lv_last_error(void) { return g_last_error.c_str(); }

// Store the graph by descending degree within each packed graph: the
// gathered (community, volume) pairs of frequent neighbours then share cache
// lines.  Ids, and so every decision and label, stay those of the input.
static lv_status reorder_by_degree(lv_graph* g, const int32_t* rank)
{
    if (g->n < 2 || g->nnz == 0) return LV_OK;
    DevBuf off2, idx2, w2, k2;
    LV_TRY(degree_order(g, g->n, g->nnz, g->off.as<int32_t>(), g->idx.as<int32_t>(),
                        g->weighted ? g->w.as<int32_t>() : nullptr, g->k.as<int32_t>(),
                        g->G > 1 ? g->d_gid.as<int32_t>() : nullptr, g->G, g->orig, g->inv, off2, idx2, w2, k2, rank,
                        &g->rev));
    g->off.swap(off2);
    g->idx.swap(idx2);
    if (g->weighted) g->w.swap(w2);
    g->k.swap(k2);
    g->reordered = true;
    Workspace& ws = g->ws;
    for (DevBuf* b : {&off2, &idx2, &w2, &k2, &ws.keys, &ws.keys_alt, &ws.vals, &ws.vals_alt}) g->release_or_park(*b);
    return LV_OK;
}

// Device setup of a packed CSR (offsets/indices/weights in `kind` memory,
// graph g at vertices [voff[g], voff[g+1])): validation, loop doubling,
// degrees, per-graph M and singleton Q_int.
static lv_status graph_setup(lv_graph* g, int32_t n, const int32_t* offsets, const int32_t* indices,
                             const int32_t* weights, lv_memkind kind, uint32_t flags, const std::vector<int32_t>& voff)
{
    hipStream_t s = g->stream;
    LV_TRY(ensure_pinned(g, 4096));
    const hipMemcpyKind hk = kind == LV_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    HIP_TRY(g->off.ensure(sizeof(int32_t) * ((size_t)n + 1)));
    HIP_TRY(hipMemcpyAsync(g->off.p, offsets, sizeof(int32_t) * ((size_t)n + 1), hk, s));
    int32_t first_last[2];
    HIP_TRY(hipMemcpyAsync(&first_last[0], g->off.as<int32_t>(), sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&first_last[1], g->off.as<int32_t>() + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (first_last[0] != 0 || first_last[1] < 0) { set_error_msg("offsets[0] must be 0 and offsets[n] >= 0"); return LV_E_CSR; }
    if ((int64_t)first_last[1] > LV_MAX_NNZ) { set_error_msg("more than LV_MAX_NNZ entries"); return LV_E_OVERFLOW; }
    const int64_t nnz = first_last[1];
    const int32_t G = (int32_t)voff.size() - 1;
    g->n = n;
    g->nnz = nnz;
    g->G = G;
    g->voff = voff;
    HIP_TRY(g->idx.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(nnz, 1)));
    if (nnz > 0) HIP_TRY(hipMemcpyAsync(g->idx.p, indices, sizeof(int32_t) * (size_t)nnz, hk, s));
    Workspace& ws = g->ws;
    HIP_TRY(ws.small.ensure(4096));
    int32_t* d_err = ws.small.as<int32_t>();
    HIP_TRY(hipMemsetAsync(d_err, 0, 16, s));
    HIP_TRY(g->w.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(nnz, 1)));
    if (weights && nnz > 0) HIP_TRY(hipMemcpyAsync(g->w.p, weights, sizeof(int32_t) * (size_t)nnz, hk, s));
    HIP_TRY(launch_check_offsets(n, g->off.as<int32_t>(), nnz, d_err, s));
    int32_t err = 0;
    HIP_TRY(hipMemcpyAsync(&err, d_err, sizeof err, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (err & 1) { set_error_msg("offsets not non-decreasing or offsets[n] != nnz"); return LV_E_CSR; }
    const int32_t* w_in = weights ? g->w.as<int32_t>() : nullptr;
    HIP_TRY(launch_check_entries(n, g->off.as<int32_t>(), g->idx.as<int32_t>(), w_in, nnz, d_err, s));
    if (flags & LV_VALIDATE)
        HIP_TRY(launch_check_symmetric(n, g->off.as<int32_t>(), g->idx.as<int32_t>(), w_in, nnz, d_err, s));
    HIP_TRY(hipMemcpyAsync(&err, d_err, sizeof err, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (err & 2) { set_error_msg("column index out of range or row not strictly increasing"); return LV_E_CSR; }
    if (err & 4) { set_error_msg("weight < 1"); return LV_E_WEIGHT; }
    if (err & 8) { set_error_msg("entry without a symmetric partner of equal weight"); return LV_E_ASYMMETRIC; }
    // graph ids and entry offsets of the packed graphs
    HIP_TRY(ws.gmeta.ensure(sizeof(int32_t) * ((size_t)G + 1)));
    if (G > 1) {
        HIP_TRY(g->d_gid.ensure(sizeof(int32_t) * (size_t)std::max(n, 1)));
        HIP_TRY(hipMemcpyAsync(ws.gmeta.p, voff.data(), sizeof(int32_t) * ((size_t)G + 1), hipMemcpyHostToDevice, s));
        HIP_TRY(launch_fill_gid(ws.gmeta.as<int32_t>(), G, n, g->d_gid.as<int32_t>(), s));
    }
    const int32_t* gid = G > 1 ? g->d_gid.as<int32_t>() : nullptr;
    LV_TRY(graph_entry_offsets(g, g->off.as<int32_t>(), voff, g->eoff));
    // loops: A_vv = 2 w (weighted degree counts a loop twice)
    HIP_TRY(ws.minv.ensure(sizeof(int32_t) * (size_t)std::max(n, 1)));
    int32_t* diag = ws.minv.as<int32_t>();
    int32_t* d_any = d_err + 1;
    HIP_TRY(launch_diag_scan(n, g->off.as<int32_t>(), g->idx.as<int32_t>(), diag, d_any, s));
    int32_t any = 0;
    HIP_TRY(hipMemcpyAsync(&any, d_any, sizeof any, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    g->weighted = weights != nullptr || any != 0;
    HIP_TRY(g->k.ensure(sizeof(int32_t) * (size_t)std::max(n, 1)));
    if (g->weighted) {
        int64_t* d_tot = (int64_t*)(ws.small.as<char>() + 64);
        HIP_TRY(hipMemsetAsync(d_tot, 0, sizeof(int64_t), s));
        HIP_TRY(launch_adjacency_weights(n, w_in, diag, nnz, g->w.as<int32_t>(), d_err, s));
        HIP_TRY(ws.k64.ensure(sizeof(int64_t) * (size_t)std::max(n, 1)));
        HIP_TRY(launch_row_sums(n, g->off.as<int32_t>(), g->w.as<int32_t>(), nnz, g->k.as<int32_t>(),
                                ws.k64.as<int64_t>(), d_tot, s));
        HIP_TRY(hipStreamSynchronize(s));
        g->release_or_park(ws.k64);
    } else {
        g->release_or_park(g->w);
        HIP_TRY(launch_degree_unit(n, g->off.as<int32_t>(), g->k.as<int32_t>(), s));
    }
    // per-graph M, trace and sum of squared degrees
    HIP_TRY(ws.gsum.ensure(sizeof(int64_t) * (size_t)G));
    HIP_TRY(ws.gsq.ensure(sizeof(int64_t) * (size_t)G));
    HIP_TRY(ws.gdone.ensure(sizeof(int64_t) * (size_t)G));
    HIP_TRY(hipMemsetAsync(ws.gsum.p, 0, sizeof(int64_t) * (size_t)G, s));
    HIP_TRY(hipMemsetAsync(ws.gsq.p, 0, sizeof(int64_t) * (size_t)G, s));
    HIP_TRY(hipMemsetAsync(ws.gdone.p, 0, sizeof(int64_t) * (size_t)G, s));
    HIP_TRY(launch_seg_sum(g->k.as<int32_t>(), n, gid, ws.gsum.as<int64_t>(), s));
    HIP_TRY(launch_sum_sq(g->k.as<int32_t>(), n, gid, ws.gsq.as<int64_t>(), s));
    HIP_TRY(launch_trace(n, g->off.as<int32_t>(), g->idx.as<int32_t>(), g->weighted ? g->w.as<int32_t>() : nullptr, nnz,
                         gid, ws.gdone.as<int64_t>(), s));
    std::vector<int64_t> Ms(G), sq(G), tr(G);
    HIP_TRY(hipMemcpyAsync(&err, d_err, sizeof err, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(Ms.data(), ws.gsum.p, sizeof(int64_t) * (size_t)G, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(sq.data(), ws.gsq.p, sizeof(int64_t) * (size_t)G, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(tr.data(), ws.gdone.p, sizeof(int64_t) * (size_t)G, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (err & 16) { set_error_msg("a loop's doubled weight exceeds 2^31 - 1"); return LV_E_OVERFLOW; }
    g->M = Ms;
    g->trace = tr;
    g->q0.resize(G);
    for (int32_t q = 0; q < G; ++q) {
        if (Ms[q] > (int64_t)INT32_MAX) { set_error_msg("total volume M >= 2^31 (graph " + std::to_string(q) + ")"); return LV_E_OVERFLOW; }
        g->q0[q] = Ms[q] * tr[q] - sq[q];
    }
    if (G > 1) {
        HIP_TRY(g->d_M.ensure(sizeof(int64_t) * (size_t)G));
        HIP_TRY(hipMemcpyAsync(g->d_M.p, g->M.data(), sizeof(int64_t) * (size_t)G, hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    // reverse-entry ranks while the rows are still sorted by column
    DevBuf rank;
    bool rank_ok = false;
    if (!(flags & LV_NO_ENTRY_CACHE) && nnz > 0) {
        HIP_TRY(rank.ensure(sizeof(int32_t) * (size_t)nnz));
        HIP_TRY(hipMemsetAsync(d_err, 0, sizeof(int32_t), s));
        HIP_TRY(launch_reverse_rank(n, g->off.as<int32_t>(), g->idx.as<int32_t>(), nnz, rank.as<int32_t>(), d_err, s));
        HIP_TRY(hipMemcpyAsync(&err, d_err, sizeof err, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        rank_ok = (err & 32) == 0;  // an asymmetric graph (not validated) gets no cache
    }
    g->rev.release();
    if (!(flags & LV_KEEP_ORDER)) LV_TRY(reorder_by_degree(g, rank_ok ? rank.as<int32_t>() : nullptr));
    if (rank_ok && !g->reordered) {
        HIP_TRY(g->rev.ensure(sizeof(int32_t) * (size_t)nnz));
        HIP_TRY(launch_reverse_from_rank(n, g->off.as<int32_t>(), g->idx.as<int32_t>(), nnz, rank.as<int32_t>(),
                                         g->rev.as<int32_t>(), s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    g->has_rev = rank_ok;
    return LV_OK;
}

static lv_status new_graph(void* stream, lv_graph** out)
{
    lv_graph* g = new (std::nothrow) lv_graph();
    if (!g) return LV_E_NOMEM;
    hipError_t e = hipGetDevice(&g->device);
    if (e == hipSuccess) {
        if (stream) {
            g->stream = (hipStream_t)stream;
        } else {
            e = hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking);
            g->own_stream = e == hipSuccess;
        }
    }
    if (e != hipSuccess) {
        set_error("lv_graph_create", e);
        delete g;
        return from_hip(e);
    }
    *out = g;
    return LV_OK;
}

// Canonical CSR (n rows, sorted columns, equal keys merged with their values
// summed) from E (row << cb | col) keys in ws.keys / ws.vals, of which the
// `valid` smallest are entries (the rest carry the all-ones key).
static lv_status csr_from_keys(lv_graph* g, int64_t E, int64_t valid, int cb, int32_t n, DevBuf& off, DevBuf& idx,
                               DevBuf& w, int64_t& nnz, uint64_t** keys_out)
{
    Workspace& ws = g->ws;
    hipStream_t s = g->stream;
    bool in_alt = false;
    HIP_TRY(radix_sort_u64(ws.keys.as<uint64_t>(), ws.vals.as<int32_t>(), ws.keys_alt.as<uint64_t>(),
                           ws.vals_alt.as<int32_t>(), E, 2 * cb, ws.tmp.p, ws.tmp.cap, &in_alt, s));
    const uint64_t* keys = in_alt ? ws.keys_alt.as<uint64_t>() : ws.keys.as<uint64_t>();
    const int32_t* vals = in_alt ? ws.vals_alt.as<int32_t>() : ws.vals.as<int32_t>();
    uint64_t* keys2 = in_alt ? ws.keys.as<uint64_t>() : ws.keys_alt.as<uint64_t>();
    HIP_TRY(ws.head.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(valid, 1)));
    int32_t* d_e2 = (int32_t*)(ws.small.as<char>() + 2304);
    HIP_TRY(hipMemsetAsync(d_e2, 0, sizeof(int32_t), s));
    HIP_TRY(launch_segment_heads(keys, valid, ws.head.as<int32_t>(), s));
    if (valid > 0)
        HIP_TRY(scan_exclusive_i32(ws.head.as<int32_t>(), ws.head.as<int32_t>(), valid, d_e2, ws.tmp.p, ws.tmp.cap, s));
    int32_t e2 = 0;
    HIP_TRY(hipMemcpyAsync(&e2, d_e2, sizeof e2, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(off.ensure(sizeof(int32_t) * ((size_t)n + 1)));
    HIP_TRY(idx.ensure(sizeof(int32_t) * (size_t)std::max(e2, 1)));
    HIP_TRY(w.ensure(sizeof(int32_t) * (size_t)std::max(e2, 1)));
    HIP_TRY(hipMemsetAsync(w.p, 0, sizeof(int32_t) * (size_t)std::max(e2, 1), s));
    HIP_TRY(launch_segment_reduce(keys, vals, ws.head.as<int32_t>(), valid, cb, idx.as<int32_t>(), w.as<int32_t>(), keys2, s));
    HIP_TRY(launch_row_offsets(keys2, e2, n, cb, off.as<int32_t>(), s));
    nnz = e2;
    if (keys_out) *keys_out = keys2;
    return LV_OK;
}

static lv_status sort_workspace(lv_graph* g, int64_t E)
{
    Workspace& ws = g->ws;
    const size_t E1 = (size_t)std::max<int64_t>(E, 1);
    HIP_TRY(ws.small.ensure(4096));
    HIP_TRY(ws.keys.ensure(sizeof(uint64_t) * E1));
    HIP_TRY(ws.keys_alt.ensure(sizeof(uint64_t) * E1));
    HIP_TRY(ws.vals.ensure(sizeof(int32_t) * E1));
    HIP_TRY(ws.vals_alt.ensure(sizeof(int32_t) * E1));
    HIP_TRY(ws.tmp.ensure(std::max(radix_tmp_bytes(E), scan_tmp_bytes(E, 8))));
    return LV_OK;
}

static void release_sort_workspace(lv_graph* g)
{
    Workspace& ws = g->ws;
    ws.keys.release();
    ws.keys_alt.release();
    ws.vals.release();
    ws.vals_alt.release();
    ws.head.release();
}

static lv_status create_from_edges(lv_graph* g, int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                                   const int32_t* weights, lv_memkind kind, uint32_t flags)
{
    hipStream_t s = g->stream;
    Workspace& ws = g->ws;
    LV_TRY(ensure_pinned(g, 4096));
    // the edge list in device memory
    DevBuf d_src, d_dst, d_w;
    const int32_t* us = src;
    const int32_t* vs = dst;
    const int32_t* ws_in = weights;
    SyncOnExit sync_inputs{s};  // the caller's arrays need to live only for the call
    if (kind == LV_MEM_HOST && m > 0) {
        HIP_TRY(d_src.ensure(sizeof(int32_t) * (size_t)m));
        HIP_TRY(d_dst.ensure(sizeof(int32_t) * (size_t)m));
        HIP_TRY(hipMemcpyAsync(d_src.p, src, sizeof(int32_t) * (size_t)m, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(d_dst.p, dst, sizeof(int32_t) * (size_t)m, hipMemcpyHostToDevice, s));
        us = d_src.as<int32_t>();
        vs = d_dst.as<int32_t>();
        if (weights) {
            HIP_TRY(d_w.ensure(sizeof(int32_t) * (size_t)m));
            HIP_TRY(hipMemcpyAsync(d_w.p, weights, sizeof(int32_t) * (size_t)m, hipMemcpyHostToDevice, s));
            ws_in = d_w.as<int32_t>();
        }
    }
    const int cb = bits_for((int64_t)n + 1);
    const int64_t E = 2 * m;
    LV_TRY(sort_workspace(g, E));
    int64_t* d_stats = (int64_t*)(ws.small.as<char>() + 3840);
    int32_t* d_err = ws.small.as<int32_t>();
    HIP_TRY(hipMemsetAsync(d_stats, 0, 2 * sizeof(int64_t), s));
    HIP_TRY(hipMemsetAsync(d_err, 0, sizeof(int32_t), s));
    HIP_TRY(launch_edge_keys(m, us, vs, ws_in, n, cb, (flags & LV_EDGES_NO_LOOPS) != 0, ws.keys.as<uint64_t>(),
                             ws.vals.as<int32_t>(), d_stats, d_err, s));
    int64_t stats[2] = {0, 0};
    int32_t err = 0;
    HIP_TRY(hipMemcpyAsync(stats, d_stats, sizeof stats, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&err, d_err, sizeof err, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    d_src.release();
    d_dst.release();
    if (err & 2) { set_error_msg("edge endpoint outside [0, n)"); return LV_E_CSR; }
    if (err & 4) { set_error_msg("edge weight < 1"); return LV_E_WEIGHT; }
    // merged weights are sums of int32 weights: bounded by the volume, checked first
    if (!(flags & LV_EDGES_SIMPLE) && stats[1] > (int64_t)INT32_MAX) {
        set_error_msg("total volume M >= 2^31");
        return LV_E_OVERFLOW;
    }
    DevBuf off, idx, w;
    int64_t nnz = 0;
    LV_TRY(csr_from_keys(g, E, stats[0], cb, n, off, idx, w, nnz, nullptr));
    d_w.release();
    release_sort_workspace(g);
    const bool unit = (flags & LV_EDGES_SIMPLE) != 0;
    return graph_setup(g, n, off.as<int32_t>(), idx.as<int32_t>(), unit ? nullptr : w.as<int32_t>(), LV_MEM_DEVICE,
                       flags & (LV_KEEP_ORDER | LV_NO_ENTRY_CACHE), std::vector<int32_t>{0, n});
}

lv_status lv_graph_create_edges(int32_t n, int64_t m, const int32_t* src, const int32_t* dst, const int32_t* weights,
                                lv_memkind kind, uint32_t flags, void* stream, lv_graph** out)
{
    FaultScope fault_scope;
    if (!out || n < 0 || m < 0 || (m > 0 && (!src || !dst)) || (kind != LV_MEM_HOST && kind != LV_MEM_DEVICE)) {
        set_error_msg("lv_graph_create_edges: null out, n < 0, m < 0, null endpoints or bad memkind");
        return LV_E_ARG;
    }
    if ((flags & LV_EDGES_SIMPLE) && weights) {
        set_error_msg("lv_graph_create_edges: LV_EDGES_SIMPLE takes no weights");
        return LV_E_ARG;
    }
    if (n == INT32_MAX || m >= ((int64_t)1 << 30)) {
        set_error_msg("lv_graph_create_edges: n must be < 2^31 - 1 and 2m < 2^31");
        return LV_E_OVERFLOW;
    }
    lv_graph* g = nullptr;
    LV_TRY(new_graph(stream, &g));
    lv_status st = create_from_edges(g, n, m, src, dst, weights, kind, flags);
    if (st != LV_OK) {
        (void)hipStreamSynchronize(g->stream);
        delete g;
        return st;
    }
    *out = g;
    return LV_OK;
}

lv_status lv_graph_csr(lv_graph* g, int32_t* offsets, int32_t* indices, int32_t* weights, int64_t* nnz_out,
                       lv_memkind kind)
{
    if (!g || (kind != LV_MEM_HOST && kind != LV_MEM_DEVICE)) { set_error_msg("lv_graph_csr: null graph or bad memkind"); return LV_E_ARG; }
    if (nnz_out) *nnz_out = g->nnz;
    if (!offsets && !indices && !weights) return LV_OK;
    if (!offsets || (g->nnz > 0 && !indices)) { set_error_msg("lv_graph_csr: null offsets or indices"); return LV_E_ARG; }
    hipStream_t s = g->stream;
    Workspace& ws = g->ws;
    const int32_t n = g->n;
    const int cb = bits_for((int64_t)n + 1);
    LV_TRY(sort_workspace(g, g->nnz));
    // keys (id of the row, id of the column): the stored positions mapped back to ids
    DevBuf ids;
    const int32_t* labels = g->reordered ? g->orig.as<int32_t>() : nullptr;
    if (!labels) {
        HIP_TRY(ids.ensure(sizeof(int32_t) * (size_t)std::max(n, 1)));
        HIP_TRY(launch_iota(ids.as<int32_t>(), n, s));
        labels = ids.as<int32_t>();
    }
    int64_t* d_scratch = (int64_t*)(ws.small.as<char>() + 3840);
    HIP_TRY(hipMemsetAsync(d_scratch, 0, sizeof(int64_t), s));
    int64_t Ek = 0;
    LV_TRY(tile_keys(g, false, n, g->off.as<int32_t>(), g->idx.as<int32_t>(), g->weighted ? g->w.as<int32_t>() : nullptr,
                     g->nnz, labels, cb, nullptr, d_scratch, &Ek));
    DevBuf off, idx, w;
    int64_t nnz = 0;
    uint64_t* keys2 = nullptr;
    LV_TRY(csr_from_keys(g, Ek, Ek, cb, n, off, idx, w, nnz, &keys2));
    HIP_TRY(launch_halve_diagonal(keys2, nnz, cb, w.as<int32_t>(), s));
    const hipMemcpyKind hk = kind == LV_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    HIP_TRY(hipMemcpyAsync(offsets, off.p, sizeof(int32_t) * ((size_t)n + 1), hk, s));
    if (nnz > 0) HIP_TRY(hipMemcpyAsync(indices, idx.p, sizeof(int32_t) * (size_t)nnz, hk, s));
    if (weights && nnz > 0) HIP_TRY(hipMemcpyAsync(weights, w.p, sizeof(int32_t) * (size_t)nnz, hk, s));
    HIP_TRY(hipStreamSynchronize(s));
    release_sort_workspace(g);
    return LV_OK;
}

lv_status lv_graph_create_csr(int32_t n, const int32_t* offsets, const int32_t* indices, const int32_t* weights,
                              lv_memkind kind, uint32_t flags, void* stream, lv_graph** out)
{
    FaultScope fault_scope;
    if (!out || n < 0 || !offsets || (kind != LV_MEM_HOST && kind != LV_MEM_DEVICE)) {
        set_error_msg("lv_graph_create_csr: null out/offsets, n < 0 or bad memkind");
        return LV_E_ARG;
    }
    if (n == INT32_MAX) { set_error_msg("n must be < 2^31 - 1"); return LV_E_OVERFLOW; }
    if (kind == LV_MEM_HOST) {
        if ((int64_t)offsets[n] > LV_MAX_NNZ) { set_error_msg("more than LV_MAX_NNZ entries"); return LV_E_OVERFLOW; }
        if ((int64_t)offsets[n] > 0 && !indices) { set_error_msg("indices is null"); return LV_E_ARG; }
    } else if (!indices) {
        set_error_msg("indices is null");
        return LV_E_ARG;
    }
    lv_graph* g = nullptr;
    LV_TRY(new_graph(stream, &g));
    lv_status st = graph_setup(g, n, offsets, indices, weights, kind, flags, std::vector<int32_t>{0, n});
    if (st != LV_OK) {
        (void)hipStreamSynchronize(g->stream);
        delete g;
        return st;
    }
    *out = g;
    return LV_OK;
}

lv_status lv_graph_create_batch(int32_t count, const int32_t* n, const int32_t* const* offsets,
                                const int32_t* const* indices, const int32_t* const* weights, lv_memkind kind,
                                uint32_t flags, void* stream, lv_graph** out)
{
    FaultScope fault_scope;
    if (!out || count < 1 || !n || !offsets || !indices || (kind != LV_MEM_HOST && kind != LV_MEM_DEVICE)) {
        set_error_msg("lv_graph_create_batch: count >= 1 and non-null n/offsets/indices/out required");
        return LV_E_ARG;
    }
    // pack on the host: graph g's vertices and entries follow graph g-1's
    std::vector<int32_t> voff(1, 0);
    std::vector<std::vector<int32_t>> ho(count);
    int64_t nv = 0, ne = 0;
    bool any_w = false;
    for (int32_t q = 0; q < count; ++q) {
        if (n[q] < 0 || !offsets[q]) { set_error_msg("graph " + std::to_string(q) + ": n < 0 or null offsets"); return LV_E_ARG; }
        ho[q].resize((size_t)n[q] + 1);
        if (kind == LV_MEM_HOST) std::memcpy(ho[q].data(), offsets[q], sizeof(int32_t) * ho[q].size());
        else HIP_TRY(hipMemcpy(ho[q].data(), offsets[q], sizeof(int32_t) * ho[q].size(), hipMemcpyDeviceToHost));
        if (ho[q][0] != 0 || ho[q][n[q]] < 0) { set_error_msg("graph " + std::to_string(q) + ": bad offsets"); return LV_E_CSR; }
        if (ho[q][n[q]] > 0 && !indices[q]) { set_error_msg("graph " + std::to_string(q) + ": null indices"); return LV_E_ARG; }
        nv += n[q];
        ne += ho[q][n[q]];
        if (nv >= INT32_MAX || ne > LV_MAX_NNZ) { set_error_msg("packed graphs exceed 2^31 - 1 vertices or LV_MAX_NNZ entries"); return LV_E_OVERFLOW; }
        voff.push_back((int32_t)nv);
        any_w = any_w || (weights && weights[q]);
    }
    std::vector<int32_t> off((size_t)nv + 1), idx((size_t)std::max<int64_t>(ne, 1)), w;
    if (any_w) w.assign((size_t)std::max<int64_t>(ne, 1), 1);
    int64_t eb = 0;
    for (int32_t q = 0; q < count; ++q) {
        const int32_t vb = voff[q];
        const int64_t m = ho[q][n[q]];
        for (int32_t x = 0; x <= n[q]; ++x) off[(size_t)vb + x] = (int32_t)(ho[q][x] + eb);
        if (m > 0) {
            int32_t* dst = idx.data() + eb;
            if (kind == LV_MEM_HOST) std::memcpy(dst, indices[q], sizeof(int32_t) * (size_t)m);
            else HIP_TRY(hipMemcpy(dst, indices[q], sizeof(int32_t) * (size_t)m, hipMemcpyDeviceToHost));
            for (int64_t t = 0; t < m; ++t) {
                if (dst[t] < 0 || dst[t] >= n[q]) { set_error_msg("graph " + std::to_string(q) + ": index out of range"); return LV_E_CSR; }
                dst[t] += vb;
            }
            if (weights && weights[q]) {
                if (kind == LV_MEM_HOST) std::memcpy(w.data() + eb, weights[q], sizeof(int32_t) * (size_t)m);
                else HIP_TRY(hipMemcpy(w.data() + eb, weights[q], sizeof(int32_t) * (size_t)m, hipMemcpyDeviceToHost));
            }
        }
        eb += m;
    }
    lv_graph* g = nullptr;
    LV_TRY(new_graph(stream, &g));
    lv_status st = graph_setup(g, (int32_t)nv, off.data(), idx.data(), any_w ? w.data() : nullptr, LV_MEM_HOST, flags, voff);
    if (st != LV_OK) {
        (void)hipStreamSynchronize(g->stream);
        delete g;
        return st;
    }
    *out = g;
    return LV_OK;
}

lv_status lv_autotune(lv_graph* g, const lv_params* params, lv_tuning* out, double* est_ms)
{
    FaultScope fault_scope;
    if (!g || !out) { set_error_msg("lv_autotune: null graph or out"); return LV_E_ARG; }
    Params p;
    LV_TRY(read_params(params, p));
    lv_tuning t{};
    double ms = 0.0;
    LV_TRY(autotune(g, p, &t, &ms));
    g->tuned = t;
    g->has_tuned = true;
    *out = t;
    if (est_ms) *est_ms = ms;
    return LV_OK;
}

lv_status lv_graph_destroy(lv_graph* g)
{
    if (!g) return LV_E_ARG;
    (void)hipStreamSynchronize(g->stream);
    delete g;
    return LV_OK;
}

lv_status lv_graph_info(const lv_graph* g, int32_t* n, int64_t* nnz, int64_t* volume)
{
    if (!g) return LV_E_ARG;
    if (n) *n = g->n;
    if (nnz) *nnz = g->nnz;
    if (volume) *volume = g->M.empty() ? 0 : g->M[0];
    return LV_OK;
}

lv_status lv_graph_count(const lv_graph* g, int32_t* count)
{
    if (!g || !count) return LV_E_ARG;
    *count = g->G;
    return LV_OK;
}

lv_status lv_louvain(lv_graph* g, const lv_params* params, lv_result** out)
{
    FaultScope fault_scope;
    if (!g || !out) { set_error_msg("lv_louvain: null graph or out"); return LV_E_ARG; }
    Params p;
    LV_TRY(read_params(params, p));
    LV_TRY(resolve_tuning(g, params, p));
    lv_result* r = new (std::nothrow) lv_result();
    if (!r) return LV_E_NOMEM;
    const bool keep = params && (params->flags & LV_KEEP_GRAPHS);
    lv_status st = louvain_impl(g, p, keep, r);
    if (st != LV_OK) {
        (void)hipStreamSynchronize(g->stream);
        delete r;
        return st;
    }
    *out = r;
    return LV_OK;
}

static const GraphResult* graph_of(const lv_result* r, int32_t g)
{
    if (!r || g < 0 || g >= r->G) return nullptr;
    return &r->graphs[g];
}

lv_status lv_result_graph_num_levels(const lv_result* r, int32_t g, int32_t* accepted, int32_t* attempted)
{
    const GraphResult* gr = graph_of(r, g);
    if (!gr) return r ? LV_E_NOT_FOUND : LV_E_ARG;
    if (accepted) *accepted = gr->accepted;
    if (attempted) *attempted = (int32_t)gr->levels.size();
    return LV_OK;
}

lv_status lv_result_graph_level_info(const lv_result* r, int32_t g, int32_t level, lv_level_info* out)
{
    const GraphResult* gr = graph_of(r, g);
    if (!gr || !out) return (!r || !out) ? LV_E_ARG : LV_E_NOT_FOUND;
    if (level < 0 || level >= (int32_t)gr->levels.size()) return LV_E_NOT_FOUND;
    *out = gr->levels[level].info;
    return LV_OK;
}

lv_status lv_result_graph_level_moves(const lv_result* r, int32_t g, int32_t level, int64_t* moves, int32_t cap)
{
    const GraphResult* gr = graph_of(r, g);
    if (!r || (!moves && cap > 0) || cap < 0) return LV_E_ARG;
    if (!gr || level < 0 || level >= (int32_t)gr->levels.size()) return LV_E_NOT_FOUND;
    const auto& mv = gr->levels[level].moves;
    for (int32_t t = 0; t < cap && t < (int32_t)mv.size(); ++t) moves[t] = mv[t];
    return LV_OK;
}

lv_status lv_result_graph_level_labels(const lv_result* r, int32_t g, int32_t level, int32_t* labels, lv_memkind kind)
{
    const GraphResult* gr = graph_of(r, g);
    if (!r || !labels || (kind != LV_MEM_HOST && kind != LV_MEM_DEVICE)) return LV_E_ARG;
    if (!gr || level < 0 || level >= gr->accepted) return LV_E_NOT_FOUND;
    const LevelRecord& rec = gr->levels[level];
    const int32_t cnt = rec.info.n;
    if (cnt <= 0) return LV_OK;
    std::vector<int32_t> h((size_t)cnt);
    HIP_TRY(hipMemcpy(h.data(), rec.store->labels.i32() + rec.vbase, sizeof(int32_t) * (size_t)cnt,
                      hipMemcpyDeviceToHost));
    for (auto& x : h) x -= rec.nbase;
    HIP_TRY(hipMemcpy(labels, h.data(), sizeof(int32_t) * (size_t)cnt,
                      kind == LV_MEM_HOST ? hipMemcpyHostToHost : hipMemcpyHostToDevice));
    return LV_OK;
}

lv_status lv_result_graph_final_labels(const lv_result* r, int32_t g, int32_t* labels, lv_memkind kind)
{
    const GraphResult* gr = graph_of(r, g);
    if (!r || !labels || (kind != LV_MEM_HOST && kind != LV_MEM_DEVICE)) return LV_E_ARG;
    if (!gr) return LV_E_NOT_FOUND;
    return copy_out(labels, r->final_labels.i32() + gr->fin_base, gr->n0, kind, nullptr);
}

lv_status lv_result_graph_modularity(const lv_result* r, int32_t g, int64_t* q_int, int64_t* m, double* q)
{
    const GraphResult* gr = graph_of(r, g);
    if (!r) return LV_E_ARG;
    if (!gr) return LV_E_NOT_FOUND;
    if (q_int) *q_int = gr->q_int;
    if (m) *m = gr->M;
    if (q) *q = gr->M > 0 ? (double)gr->q_int / ((double)gr->M * (double)gr->M) : 0.0;
    return LV_OK;
}

lv_status lv_result_final_labels_all(const lv_result* r, int32_t* labels, lv_memkind kind)
{
    if (!r || !labels || (kind != LV_MEM_HOST && kind != LV_MEM_DEVICE)) return LV_E_ARG;
    return copy_out(labels, r->final_labels.i32(), r->n0, kind, nullptr);
}

lv_status lv_result_modularity_all(const lv_result* r, int64_t* q_int, int64_t* m, double* q)
{
    if (!r) return LV_E_ARG;
    for (int32_t c = 0; c < r->G; ++c) {
        const GraphResult& gr = r->graphs[c];
        if (q_int) q_int[c] = gr.q_int;
        if (m) m[c] = gr.M;
        if (q) q[c] = gr.M > 0 ? (double)gr.q_int / ((double)gr.M * (double)gr.M) : 0.0;
    }
    return LV_OK;
}

lv_status lv_result_num_levels(const lv_result* r, int32_t* accepted, int32_t* attempted)
{
    return lv_result_graph_num_levels(r, 0, accepted, attempted);
}
lv_status lv_result_level_info(const lv_result* r, int32_t level, lv_level_info* out)
{
    return lv_result_graph_level_info(r, 0, level, out);
}
lv_status lv_result_level_moves(const lv_result* r, int32_t level, int64_t* moves, int32_t cap)
{
    return lv_result_graph_level_moves(r, 0, level, moves, cap);
}
lv_status lv_result_level_labels(const lv_result* r, int32_t level, int32_t* labels, lv_memkind kind)
{
    return lv_result_graph_level_labels(r, 0, level, labels, kind);
}
lv_status lv_result_final_labels(const lv_result* r, int32_t* labels, lv_memkind kind)
{
    return lv_result_graph_final_labels(r, 0, labels, kind);
}
lv_status lv_result_modularity(const lv_result* r, int64_t* q_int, int64_t* m, double* q)
{
    return lv_result_graph_modularity(r, 0, q_int, m, q);
}

lv_status lv_result_level_graph(const lv_result* r, int32_t level, int32_t* offsets, int32_t* indices,
                                int32_t* weights, int64_t* nnz, lv_memkind kind)
{
    const GraphResult* gr = graph_of(r, 0);
    if (!r || !nnz) return LV_E_ARG;
    if (!gr || level < 0 || level >= gr->accepted) return LV_E_NOT_FOUND;
    const LevelRecord& rec = gr->levels[level];
    if (!rec.g_off) return LV_E_STATE;
    *nnz = rec.g_nnz;
    if (offsets) LV_TRY(copy_out(offsets, rec.g_off->as<int32_t>(), (int64_t)rec.info.n_next + 1, kind, nullptr));
    if (indices) LV_TRY(copy_out(indices, rec.g_idx->as<int32_t>(), rec.g_nnz, kind, nullptr));
    if (weights) LV_TRY(copy_out(weights, rec.g_w->as<int32_t>(), rec.g_nnz, kind, nullptr));
    return LV_OK;
}

lv_status lv_result_destroy(lv_result* r)
{
    if (!r) return LV_E_ARG;
    (void)hipDeviceSynchronize();
    delete r;
    return LV_OK;
}

static lv_status modularity_impl(lv_graph* g, const int32_t* labels_dev, int64_t* q_int)
{
    Workspace& ws = g->ws;
    hipStream_t s = g->stream;
    const int32_t n = g->n;
    HIP_TRY(ws.k64.ensure(sizeof(int64_t) * (size_t)std::max(n, 1)));
    int64_t* d_q = (int64_t*)(ws.small.as<char>() + 2816);
    int32_t* d_err = (int32_t*)(ws.small.as<char>() + 3072);
    HIP_TRY(hipMemsetAsync(ws.k64.p, 0, sizeof(int64_t) * (size_t)std::max(n, 1), s));
    HIP_TRY(hipMemsetAsync(d_q, 0, 2 * sizeof(int64_t), s));
    HIP_TRY(hipMemsetAsync(d_err, 0, sizeof(int32_t), s));
    HIP_TRY(launch_check_labels(labels_dev, n, d_err, s));
    int32_t err = 0;
    HIP_TRY(hipMemcpyAsync(&err, d_err, sizeof err, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (err) { set_error_msg("labels must lie in [0, n)"); return LV_E_ARG; }
    HIP_TRY(launch_modularity_parts(n, g->off.as<int32_t>(), g->idx.as<int32_t>(), g->weighted ? g->w.as<int32_t>() : nullptr,
                                    g->nnz, g->k.as<int32_t>(), labels_dev, ws.k64.as<int64_t>(), d_q, s));
    int64_t q2[2];
    HIP_TRY(hipMemcpyAsync(q2, d_q, sizeof q2, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    ws.k64.release();
    *q_int = g->M[0] * q2[0] - q2[1];
    return LV_OK;
}

lv_status lv_probe_gather(lv_graph* g, int32_t reps, double* entries_per_s)
{
    if (!g || reps < 1 || !entries_per_s) { set_error_msg("lv_probe_gather: null graph/out or reps < 1"); return LV_E_ARG; }
    hipStream_t s = g->stream;
    DevBuf tab, sink;
    HIP_TRY(tab.ensure(sizeof(int2) * (size_t)std::max(g->n, 1)));
    HIP_TRY(sink.ensure(sizeof(unsigned long long)));
    HIP_TRY(hipMemsetAsync(tab.p, 0x5a, sizeof(int2) * (size_t)std::max(g->n, 1), s));
    const int32_t* idx = g->idx.as<int32_t>();
    HIP_TRY(launch_probe_gather(idx, tab.as<int2>(), g->nnz, sink.as<unsigned long long>(), s));  // warm-up
    Timer t;
    t.s = s;
    hipEvent_t e0{}, e1{};
    HIP_TRY(t.mark(&e0));
    for (int32_t r = 0; r < reps; ++r) HIP_TRY(launch_probe_gather(idx, tab.as<int2>(), g->nnz, sink.as<unsigned long long>(), s));
    HIP_TRY(t.mark(&e1));
    HIP_TRY(hipStreamSynchronize(s));
    const double ms = elapsed(e0, e1) / reps;
    *entries_per_s = ms > 0 ? (double)g->nnz / (ms * 1e-3) : 0.0;
    return LV_OK;
}

lv_status lv_probe_copy(lv_graph* g, int32_t reps, double* bytes_per_s)
{
    if (!g || reps < 1 || !bytes_per_s) { set_error_msg("lv_probe_copy: null graph/out or reps < 1"); return LV_E_ARG; }
    hipStream_t s = g->stream;
    const int64_t n = g->nnz;
    if (n <= 0) { *bytes_per_s = 0.0; return LV_OK; }
    DevBuf dst;
    HIP_TRY(dst.ensure(sizeof(int32_t) * (size_t)n));
    const int32_t* src = g->idx.as<int32_t>();
    HIP_TRY(launch_probe_copy(src, dst.as<int32_t>(), n, s));  // warm-up
    Timer t;
    t.s = s;
    hipEvent_t e0{}, e1{};
    HIP_TRY(t.mark(&e0));
    for (int32_t r = 0; r < reps; ++r) HIP_TRY(launch_probe_copy(src, dst.as<int32_t>(), n, s));
    HIP_TRY(t.mark(&e1));
    HIP_TRY(hipStreamSynchronize(s));
    const double ms = elapsed(e0, e1) / reps;
    *bytes_per_s = ms > 0 ? 2.0 * sizeof(int32_t) * (double)n / (ms * 1e-3) : 0.0;
    return LV_OK;
}

lv_status lv_modularity(lv_graph* g, const int32_t* labels, lv_memkind kind, int64_t* q_int, int64_t* m, double* q)
{
    FaultScope fault_scope;
    if (!g || !labels || (kind != LV_MEM_HOST && kind != LV_MEM_DEVICE)) return LV_E_ARG;
    if (g->G != 1) { set_error_msg("lv_modularity takes a single-graph handle"); return LV_E_STATE; }
    Workspace& ws = g->ws;
    HIP_TRY(ws.small.ensure(4096));
    const int32_t* dl = labels;
    SyncOnExit sync_labels{g->stream};  // the caller's labels need to live only for the call
    if (kind == LV_MEM_HOST) {
        HIP_TRY(ws.labels.ensure(sizeof(int32_t) * (size_t)std::max(g->n, 1)));
        if (g->n > 0)
            HIP_TRY(hipMemcpyAsync(ws.labels.p, labels, sizeof(int32_t) * (size_t)g->n, hipMemcpyHostToDevice, g->stream));
        dl = ws.labels.as<int32_t>();
    }
    if (g->reordered && g->n > 0) {  // to storage positions
        HIP_TRY(ws.pos.ensure(sizeof(int32_t) * ((size_t)g->n + 1)));
        HIP_TRY(launch_gather_i32(dl, g->orig.as<int32_t>(), g->n, ws.pos.as<int32_t>(), g->stream));
        dl = ws.pos.as<int32_t>();
    }
    int64_t qi = 0;
    LV_TRY(modularity_impl(g, dl, &qi));
    const int64_t M = g->M[0];
    if (q_int) *q_int = qi;
    if (m) *m = M;
    if (q) *q = M > 0 ? (double)qi / ((double)M * (double)M) : 0.0;
    return LV_OK;
}

lv_status lv_lpa_batch(lv_graph* g, const lv_params* params, int32_t* labels, lv_memkind kind, int32_t* sweeps,
                       int64_t* q_int, int64_t* m, int64_t* moves, int32_t moves_stride)
{
    FaultScope fault_scope;
    if (!g || !labels || (kind != LV_MEM_HOST && kind != LV_MEM_DEVICE) || moves_stride < 0 ||
        (moves && moves_stride == 0))
        return LV_E_ARG;
    Params p;
    LV_TRY(read_params(params, p));
    LV_TRY(resolve_tuning(g, params, p));
    Workspace& ws = g->ws;
    HIP_TRY(ws.pos.ensure(sizeof(int32_t) * ((size_t)g->n + 1)));
    // device-resident output: the labels are written in place; host output
    // goes through a pooled buffer
    const bool direct = kind == LV_MEM_DEVICE && g->n > 0;
    PooledBuf out;
    if (!direct) HIP_TRY(pool_take(g->pool, sizeof(int32_t) * (size_t)std::max(g->n, 1), out));
    int32_t* dst = direct ? labels : out.i32();
    SweepOut so;
    std::vector<int32_t> voff2;
    std::vector<int64_t> qi;
    double ren = 0;
    LV_TRY(lpa_impl(g, p, dst, so, voff2, qi, &ren));
    if (!direct) LV_TRY(copy_out(labels, dst, g->n, kind, g->stream));
    for (int32_t c = 0; c < g->G; ++c) {
        if (sweeps) sweeps[c] = so.sweeps[c];
        if (q_int) q_int[c] = qi[c];
        if (m) m[c] = g->M[c];
        if (moves)
            for (int32_t t = 0; t < moves_stride; ++t)
                moves[(size_t)c * moves_stride + t] = t < so.sweeps[c] ? (int64_t)so.moves[(size_t)c * p.max_sweeps + t] : 0;
    }
    return LV_OK;
}

lv_status lv_lpa(lv_graph* g, const lv_params* params, int32_t* labels, lv_memkind kind, lv_level_info* info,
                 int64_t* moves_out, int32_t moves_cap)
{
    FaultScope fault_scope;
    if (!g || !labels || (kind != LV_MEM_HOST && kind != LV_MEM_DEVICE) || moves_cap < 0 || (moves_cap > 0 && !moves_out))
        return LV_E_ARG;
    if (g->G != 1) { set_error_msg("lv_lpa takes a single-graph handle (see lv_lpa_batch)"); return LV_E_STATE; }
    Params p;
    LV_TRY(read_params(params, p));
    LV_TRY(resolve_tuning(g, params, p));
    DevBuf out;
    HIP_TRY(out.ensure(sizeof(int32_t) * (size_t)std::max(g->n, 1)));
    SweepOut so;
    std::vector<int32_t> voff2;
    std::vector<int64_t> qi;
    double ren = 0;
    LV_TRY(lpa_impl(g, p, out.as<int32_t>(), so, voff2, qi, &ren));
    LV_TRY(copy_out(labels, out.as<int32_t>(), g->n, kind, g->stream));
    for (int32_t t = 0; t < moves_cap && t < so.sweeps[0]; ++t) moves_out[t] = so.moves[t];
    if (info) {
        lv_level_info li{};
        li.n = g->n;
        li.n_next = voff2[1];
        li.nnz = g->nnz;
        li.q_start = g->q0[0];
        li.q_end = qi[0];
        li.accepted = 1;
        li.renumber_ms = ren;
        fill_info(li, so, 0, p.max_sweeps);
        *info = li;
    }
    return LV_OK;
}

}  // extern "C"

#include "lv_server.inc"
#include "lv_noalloc.inc"
