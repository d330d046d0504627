// C ABI of the Louvain library (declared in include/lv.h): argument checks,
// device workspace, and the host-side level driver of Algorithm 3 around the
// HIP kernels of lv_kernels.hip.
#include "lv.h"
#include "lv_internal.h"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <string>
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

// Allocation with optional fault injection: LV_FAULT_ALLOC_AT=k makes the
// k-th device allocation of the process fail with out-of-memory.
long g_alloc_count = 0;
hipError_t dev_alloc(void** p, size_t bytes)
{
    ++g_alloc_count;
    static long fail_at = [] {
        const char* v = std::getenv("LV_FAULT_ALLOC_AT");
        return v ? std::atol(v) : 0L;
    }();
    if (fail_at > 0 && g_alloc_count == fail_at) { *p = nullptr; return hipErrorOutOfMemory; }
    return hipMalloc(p, bytes ? bytes : 1);
}

// Grow-only device buffer.
struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
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
};

struct Workspace {
    DevBuf comm, sigma, dec, cls, vert, cls_alt, vert_alt, minv, flag, pos, labels, tmp, small;
    DevBuf keys, keys_alt, vals, vals_alt, head;
    DevBuf g_off[2], g_idx[2], g_w[2], g_k[2];
    DevBuf hub_table, hub_meta, hub_part, hub_rows, hub_pairs;
    DevBuf k64, cs;
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
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.f;
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

}  // namespace

struct lv_graph {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int32_t n = 0;
    int64_t nnz = 0;
    DevBuf off, idx, w, k;
    bool weighted = false;  // false: every A entry is 1 (no weights, no loops)
    int64_t M = 0, trace = 0, sumk2 = 0;
    Workspace ws;
    int32_t* pinned = nullptr;  // small host staging area
    ~lv_graph()
    {
        if (pinned) (void)hipHostFree(pinned);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
};

namespace {

struct LevelRecord {
    lv_level_info info{};
    std::vector<int64_t> moves;
    DevBuf labels;                  // accepted levels only
    DevBuf g_off, g_idx, g_w;       // coarse graph (LV_KEEP_GRAPHS)
    int64_t g_nnz = 0;
};

}  // namespace

struct lv_result {
    int32_t n0 = 0;
    int64_t M = 0;
    int64_t q_int = 0;
    int32_t accepted = 0;
    std::vector<std::unique_ptr<LevelRecord>> levels;
    DevBuf final_labels;
};

namespace {

struct Tune {
    int32_t bounds[NUM_CLS];
    int32_t part_keys;  // expected distinct communities per partition workgroup
    int32_t part_slots; // LDS slots of a partition workgroup (power of two)
    int32_t pregather;  // partition mode (see lv_tuning.hub_mode)
    int32_t fb_chunk;   // entries / slots per workgroup on the global-table fallback
};

Tune make_tune(const lv_tuning* t)
{
    Tune u;
    for (int c = 0; c < NUM_CLS; ++c) u.bounds[c] = CLS_CAP[c];
    u.part_keys = 8192;
    u.part_slots = 16384;
    u.pregather = 0;
    u.fb_chunk = 4096;
    if (t) {
        // sub_max bounds the 8- and 32-lane classes, wave_max the wavefront
        // class, block_max the workgroup classes; each is clamped to what the
        // class's table holds, so no setting can overflow a table.
        if (t->sub_max > 0) {
            u.bounds[CLS_G8] = std::min(CLS_CAP[CLS_G8], t->sub_max);
            u.bounds[CLS_G32] = std::min(CLS_CAP[CLS_G32], std::max(u.bounds[CLS_G8], t->sub_max));
        }
        if (t->wave_max > 0) u.bounds[CLS_G64] = std::min(CLS_CAP[CLS_G64], std::max(u.bounds[CLS_G32], t->wave_max));
        if (t->block_max > 0) {
            u.bounds[CLS_B256] = std::min(CLS_CAP[CLS_B256], std::max(u.bounds[CLS_G64], t->block_max));
            u.bounds[CLS_B512] = std::min(CLS_CAP[CLS_B512], std::max(u.bounds[CLS_B256], t->block_max));
            u.bounds[CLS_B4K] = std::min(CLS_CAP[CLS_B4K], std::max(u.bounds[CLS_B512], t->block_max));
        }
        if (t->hub_mode == 2) {
            u.pregather = 1;
            u.part_slots = 8192;
            u.part_keys = 6144;
        }
        const uint64_t max_slots = u.pregather ? 8192 : 16384;
        if (t->part_slots > 0)
            u.part_slots = (int32_t)std::min<uint64_t>(max_slots, std::max<uint64_t>(64, next_pow2((uint64_t)t->part_slots)));
        if (t->part_keys > 0) u.part_keys = std::max(32, t->part_keys);
    }
    // a single partition must always fit: part_keys <= 3/4 of the slots
    u.part_keys = std::min(u.part_keys, u.part_slots / 4 * 3);
    // keep bounds non-decreasing
    for (int c = CLS_G32; c < CLS_HUB; ++c) u.bounds[c] = std::max(u.bounds[c], u.bounds[c - 1]);
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

// One level's graph (device pointers).
struct LevelGraph {
    int32_t n;
    int64_t nnz;
    const int32_t* off;
    const int32_t* idx;
    const int32_t* w;  // null = unit
    const int32_t* k;
};

struct SweepOut {
    std::vector<int64_t> moves;
    double move_ms = 0, sweep_ms = 0;
    int64_t launches = 0;
    int64_t bytes = 0;
    double kern_ms[LV_KERNEL_SLOTS] = {};
    int64_t kern_launches[LV_KERNEL_SLOTS] = {};
    int64_t kern_bytes[LV_KERNEL_SLOTS] = {};
};

// Hub (global table) layout for one level.
struct HubPlan {
    int32_t nhubs = 0;
    HubArgs args{};
};

lv_status plan_hubs(lv_graph* g, const LevelGraph& G, const int32_t* hub_verts, int32_t nhubs, const Tune& tu,
                    HubPlan& plan)
{
    Workspace& ws = g->ws;
    hipStream_t s = g->stream;
    plan.nhubs = nhubs;
    if (nhubs == 0) return LV_OK;
    // row starts and lengths of the hubs, read back to size the layout
    HIP_TRY(ws.hub_rows.ensure(sizeof(int32_t) * 2 * (size_t)nhubs));
    int32_t* d_beg = ws.hub_rows.as<int32_t>();
    int32_t* d_len = d_beg + nhubs;
    HIP_TRY(launch_gather_rows(hub_verts, nhubs, G.off, d_beg, d_len, s));
    std::vector<int32_t> beg(nhubs), len(nhubs), hv(nhubs);
    HIP_TRY(hipMemcpyAsync(beg.data(), d_beg, sizeof(int32_t) * nhubs, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(len.data(), d_len, sizeof(int32_t) * nhubs, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(hv.data(), hub_verts, sizeof(int32_t) * nhubs, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    std::vector<int32_t> parts(nhubs), first_blk(nhubs + 1), blk_hub, blk_part;
    std::vector<int64_t> tab_off(nhubs), pair_off(nhubs);
    int64_t npairs = 0;
    std::vector<int32_t> tab_cap(nhubs), ins_hub, ins_beg, ins_end, scan_hub, scan_beg, scan_end, fpart_first(nhubs + 1);
    int64_t slots = 0;
    for (int32_t h = 0; h < nhubs; ++h) {
        const int32_t P = (int32_t)std::max<int64_t>(1, ((int64_t)len[h] + tu.part_keys - 1) / tu.part_keys);
        parts[h] = P;
        first_blk[h] = (int32_t)blk_hub.size();
        for (int32_t q = 0; q < P; ++q) { blk_hub.push_back(h); blk_part.push_back(q); }
        fpart_first[h] = (int32_t)scan_hub.size();
        tab_off[h] = slots;
        tab_cap[h] = 0;
        pair_off[h] = npairs;
        if (P == 1) continue;  // one partition of <= part_keys keys always fits its LDS table
        if (tu.pregather) npairs += len[h];
        const uint64_t cap = std::max<uint64_t>(64, next_pow2(2ull * (uint64_t)len[h]));
        if (cap > (uint64_t)INT32_MAX) { set_error_msg("hub table too large"); return LV_E_OVERFLOW; }
        tab_cap[h] = (int32_t)cap;
        slots += (int64_t)cap;
        for (int64_t e = beg[h]; e < (int64_t)beg[h] + len[h]; e += tu.fb_chunk) {
            ins_hub.push_back(h);
            ins_beg.push_back((int32_t)e);
            ins_end.push_back((int32_t)std::min<int64_t>(e + tu.fb_chunk, (int64_t)beg[h] + len[h]));
        }
        for (int64_t t = 0; t < (int64_t)cap; t += tu.fb_chunk) {
            scan_hub.push_back(h);
            scan_beg.push_back((int32_t)t);
            scan_end.push_back((int32_t)std::min<int64_t>(t + tu.fb_chunk, (int64_t)cap));
        }
    }
    first_blk[nhubs] = (int32_t)blk_hub.size();
    fpart_first[nhubs] = (int32_t)scan_hub.size();
    const int32_t nblk = (int32_t)blk_hub.size(), nins = (int32_t)ins_hub.size(), nscan = (int32_t)scan_hub.size();
    // metadata: int64 tab_off first, then the int32 arrays
    std::vector<int32_t> pack;
    auto put = [&](const std::vector<int32_t>& v) {
        const size_t at = pack.size();
        pack.insert(pack.end(), v.begin(), v.end());
        return at;
    };
    const size_t o_hv = put(hv), o_parts = put(parts), o_fb = put(first_blk), o_bh = put(blk_hub), o_bp = put(blk_part);
    const size_t o_cap = put(tab_cap), o_ih = put(ins_hub), o_ib = put(ins_beg), o_ie = put(ins_end);
    const size_t o_sh = put(scan_hub), o_sb = put(scan_beg), o_se = put(scan_end), o_ff = put(fpart_first);
    const size_t b64 = sizeof(int64_t) * (size_t)nhubs;
    HIP_TRY(ws.hub_meta.ensure(2 * b64 + sizeof(int32_t) * pack.size() + 64));
    char* base = ws.hub_meta.as<char>();
    int32_t* p32 = (int32_t*)(base + 2 * b64);
    HIP_TRY(hipMemcpyAsync(base, tab_off.data(), b64, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(base + b64, pair_off.data(), b64, hipMemcpyHostToDevice, s));
    HIP_TRY(ws.hub_pairs.ensure(sizeof(int2) * (size_t)std::max<int64_t>(npairs, 1)));
    HIP_TRY(hipMemcpyAsync(p32, pack.data(), sizeof(int32_t) * pack.size(), hipMemcpyHostToDevice, s));
    // partial results + flags: [nblk] x (int64 score, int32 comm, wown, flag), [nhubs] fb_flag, [nscan] fallback partials
    const size_t part_bytes = (size_t)nblk * (8 + 4 * 3) + (size_t)nhubs * 4 + (size_t)std::max(nscan, 1) * (8 + 4 * 2);
    HIP_TRY(ws.hub_part.ensure(part_bytes + 64));
    char* pb = ws.hub_part.as<char>();
    HubArgs& a = plan.args;
    a = HubArgs{};
    a.nhubs = nhubs;
    a.part_mask = (uint32_t)tu.part_slots - 1u;
    a.pregather = tu.pregather;
    a.hub_vert = p32 + o_hv;
    a.hub_parts = p32 + o_parts;
    a.hub_first_blk = p32 + o_fb;
    a.blk_hub = p32 + o_bh;
    a.blk_part = p32 + o_bp;
    a.nblk = nblk;
    a.part_score = (int64_t*)pb;
    a.part_comm = (int32_t*)(a.part_score + nblk);
    a.part_wown = a.part_comm + nblk;
    a.part_flag = a.part_wown + nblk;
    a.fb_flag = a.part_flag + nblk;
    int64_t* fps = (int64_t*)(((uintptr_t)(a.fb_flag + nhubs) + 7) & ~(uintptr_t)7);
    a.fpart_score = fps;
    a.fpart_comm = (int32_t*)(fps + std::max(nscan, 1));
    a.fpart_wown = a.fpart_comm + std::max(nscan, 1);
    a.fpart_first = p32 + o_ff;
    a.tab_off = (const int64_t*)base;
    a.pair_off = (const int64_t*)(base + b64);
    a.pairs = ws.hub_pairs.as<int2>();
    a.tab_cap = p32 + o_cap;
    a.ins_hub = p32 + o_ih;
    a.ins_beg = p32 + o_ib;
    a.ins_end = p32 + o_ie;
    a.nins = nins;
    a.scan_hub = p32 + o_sh;
    a.scan_beg = p32 + o_sb;
    a.scan_end = p32 + o_se;
    a.nscan = nscan;
    HIP_TRY(hipMemsetAsync(a.fb_flag, 0, sizeof(int32_t) * (size_t)nhubs, s));
    HIP_TRY(ws.hub_table.ensure(sizeof(int32_t) * 2 * (size_t)std::max<int64_t>(slots, 1)));
    a.table = ws.hub_table.as<int32_t>();
    HIP_TRY(launch_hub_clear(a.table, slots, s));
    // the host vectors must outlive the asynchronous copies
    HIP_TRY(hipStreamSynchronize(s));
    return LV_OK;
}

// Synchronous local-moving sweeps of one level (Algorithm 2; Algorithm 1 in
// LPA mode).  On return ws.comm holds the level's labels and ws.sigma the
// community volumes.
lv_status run_sweeps(lv_graph* g, const LevelGraph& G, int mode, const Params& p, SweepOut& out)
{
    Workspace& ws = g->ws;
    hipStream_t s = g->stream;
    const int32_t n = G.n;
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
    HIP_TRY(hipMemcpyAsync(start, d_start, sizeof start, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    start[NUM_CLS] = n;
    for (int c = NUM_CLS - 1; c >= 0; --c)
        if (start[c] < 0) start[c] = start[c + 1];
    const int32_t active = n - start[CLS_G8];  // vertices with at least one entry

    HubPlan hubs;
    LV_TRY(plan_hubs(g, G, vert_sorted + start[CLS_HUB], n - start[CLS_HUB], p.tune, hubs));
    // CSR entries per class, for the per-kernel algorithmic byte counts
    int64_t cls_entries[NUM_CLS] = {};
    if (p.flags & LV_TIMING) {
        int64_t* d_ce = (int64_t*)(ws.small.as<char>() + 3328);
        HIP_TRY(hipMemsetAsync(d_ce, 0, sizeof cls_entries, s));
        HIP_TRY(launch_class_entries(vert_sorted, start, G.off, d_ce, s));
        HIP_TRY(hipMemcpyAsync(cls_entries, d_ce, sizeof cls_entries, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    const int64_t wbytes = G.w ? 8 : 4;

    HIP_TRY(launch_iota(ws.comm.as<int32_t>(), n, s));
    HIP_TRY(launch_copy_i32(ws.sigma.as<int32_t>(), G.k, n, s));
    HIP_TRY(launch_pairs(n, ws.comm.as<int32_t>(), ws.sigma.as<int32_t>(), ws.cs.as<int2>(), s));
    uint32_t* d_count = (uint32_t*)(ws.small.as<char>() + 1024);

    MoveArgs a{};
    a.off = G.off;
    a.idx = G.idx;
    a.w = G.w;
    a.k = G.k;
    a.comm = ws.comm.as<int32_t>();
    a.sigma = ws.sigma.as<int32_t>();
    a.cs = ws.cs.as<int2>();
    a.M = g->M;
    a.mode = mode;
    int32_t* dec_all = ws.dec.as<int32_t>();

    Timer tm;
    tm.on = (p.flags & LV_TIMING) != 0;
    tm.s = s;
    const int64_t sweep_bytes = 4 * ((int64_t)n + 1) + (G.w ? 8 : 4) * G.nnz + 12 * (int64_t)n;
    const int64_t theta = mode == MODE_LPA ? p.lpa_threshold : 0;
    out.moves.clear();
    for (int32_t sw = 1; sw <= p.max_sweeps; ++sw) {
        a.dir = (sw % 2 == 1) ? DIR_DOWN : DIR_UP;
        const bool singleton = sw == 1;
        HIP_TRY(hipMemsetAsync(d_count, 0, sizeof(uint32_t), s));
        hipEvent_t e0{}, e1{}, e2{};
        hipEvent_t kb[NUM_CLS] = {}, kend[NUM_CLS] = {};
        if (tm.on) HIP_TRY(tm.mark(&e0));
        for (int c = CLS_G8; c < CLS_HUB; ++c) {
            a.verts = vert_sorted + start[c];
            a.dec = dec_all + start[c];
            a.nverts = start[c + 1] - start[c];
            if (a.nverts == 0) continue;
            if (tm.on) HIP_TRY(tm.mark(&kb[c]));
            HIP_TRY(launch_move_class(c, singleton, a, s));
            if (tm.on) HIP_TRY(tm.mark(&kend[c]));
            ++out.launches;
        }
        if (hubs.nhubs > 0) {
            a.dec = dec_all + start[CLS_HUB];
            if (tm.on) HIP_TRY(tm.mark(&kb[CLS_HUB]));
            HIP_TRY(launch_hub_sweep(singleton, a, hubs.args, s));
            if (tm.on) HIP_TRY(tm.mark(&kend[CLS_HUB]));
            out.launches += singleton ? 2 : 3;
        }
        if (tm.on) HIP_TRY(tm.mark(&e1));
        HIP_TRY(launch_apply(vert_sorted + start[CLS_G8], dec_all + start[CLS_G8], active, G.k,
                             ws.comm.as<int32_t>(), ws.sigma.as<int32_t>(), d_count, s));
        HIP_TRY(launch_pairs(n, ws.comm.as<int32_t>(), ws.sigma.as<int32_t>(), ws.cs.as<int2>(), s));
        if (tm.on) HIP_TRY(tm.mark(&e2));
        uint32_t cnt = 0;
        HIP_TRY(hipMemcpyAsync(g->pinned, d_count, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        std::memcpy(&cnt, g->pinned, sizeof cnt);
        out.moves.push_back((int64_t)cnt);
        out.bytes += sweep_bytes;
        if (tm.on) {
            out.move_ms += elapsed(e0, e1);
            out.sweep_ms += elapsed(e0, e2);
            for (int c = CLS_G8; c <= CLS_HUB; ++c) {
                const int32_t nv = start[c + 1] - start[c];
                if (nv == 0) continue;
                const int slot = 2 * c + (singleton ? 1 : 0) - 2;
                out.kern_ms[slot] += elapsed(kb[c], kend[c]);
                out.kern_launches[slot] += 1;
                out.kern_bytes[slot] += wbytes * cls_entries[c] + 20 * (int64_t)nv;
            }
            tm.used = 0;
        }
        const size_t m = out.moves.size();
        if (m >= 2 && out.moves[m - 1] <= theta && out.moves[m - 2] <= theta) break;
    }
    return LV_OK;
}

struct Coarse {
    int32_t n2 = 0;
    int64_t nnz2 = 0;
    int32_t *off = nullptr, *idx = nullptr, *w = nullptr, *k = nullptr;
    int64_t q_end = 0;
};

// Renumber communities by smallest member (first occurrence); labels -> ws.labels.
lv_status renumber(lv_graph* g, int32_t n, int32_t* n2)
{
    Workspace& ws = g->ws;
    hipStream_t s = g->stream;
    const size_t nb = sizeof(int32_t) * (size_t)std::max(n, 1);
    HIP_TRY(ws.minv.ensure(nb));
    HIP_TRY(ws.flag.ensure(nb));
    HIP_TRY(ws.pos.ensure(nb));
    HIP_TRY(ws.labels.ensure(nb));
    int32_t* d_n2 = (int32_t*)(ws.small.as<char>() + 2048);
    HIP_TRY(launch_renumber(n, ws.comm.as<int32_t>(), ws.minv.as<int32_t>(), ws.flag.as<int32_t>(),
                            ws.pos.as<int32_t>(), ws.labels.as<int32_t>(), d_n2, ws.tmp.p, ws.tmp.cap, g->stream));
    HIP_TRY(hipMemcpyAsync(g->pinned, d_n2, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    std::memcpy(n2, g->pinned, sizeof(int32_t));
    return LV_OK;
}

// Aggregation (Algorithm 3): coarse CSR A' = S^T A S into ping-pong slot `slot`;
// also Q_end = M * Sigma_in - sum_P k'_P^2, the modularity of the level's partition.
lv_status aggregate(lv_graph* g, const LevelGraph& G, int32_t n2, int slot, Coarse& out)
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
    int64_t* d_q = (int64_t*)(ws.small.as<char>() + 2560);  // [0] Sigma_in, [1] sum k'^2
    HIP_TRY(hipMemsetAsync(d_q, 0, 2 * sizeof(int64_t), s));
    HIP_TRY(launch_coarse_degree(G.n, ws.comm.as<int32_t>(), ws.flag.as<int32_t>(), ws.labels.as<int32_t>(),
                                 ws.sigma.as<int32_t>(), ws.g_k[slot].as<int32_t>(), s));
    HIP_TRY(launch_sum_sq(ws.g_k[slot].as<int32_t>(), n2, d_q + 1, s));
    HIP_TRY(launch_build_keys(G.n, G.off, G.idx, G.w, E, ws.labels.as<int32_t>(), colbits, ws.keys.as<uint64_t>(),
                              ws.vals.as<int32_t>(), d_q, s));
    bool in_alt = false;
    HIP_TRY(radix_sort_u64(ws.keys.as<uint64_t>(), ws.vals.as<int32_t>(), ws.keys_alt.as<uint64_t>(),
                           ws.vals_alt.as<int32_t>(), E, bits, ws.tmp.p, ws.tmp.cap, &in_alt, s));
    const uint64_t* keys = in_alt ? ws.keys_alt.as<uint64_t>() : ws.keys.as<uint64_t>();
    const int32_t* vals = in_alt ? ws.vals_alt.as<int32_t>() : ws.vals.as<int32_t>();
    uint64_t* keys2 = in_alt ? ws.keys.as<uint64_t>() : ws.keys_alt.as<uint64_t>();  // the free sort buffer
    int32_t* d_e2 = (int32_t*)(ws.small.as<char>() + 2304);
    HIP_TRY(launch_segment_heads(keys, E, ws.head.as<int32_t>(), s));
    HIP_TRY(scan_exclusive_i32(ws.head.as<int32_t>(), ws.head.as<int32_t>(), E, d_e2, ws.tmp.p, ws.tmp.cap, s));
    int64_t q2[2];
    HIP_TRY(hipMemcpyAsync(g->pinned, d_e2, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(g->pinned + 2, d_q, sizeof q2, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    int32_t e2 = 0;
    std::memcpy(&e2, g->pinned, sizeof e2);
    std::memcpy(q2, g->pinned + 2, sizeof q2);
    if (E == 0) e2 = 0;
    HIP_TRY(ws.g_idx[slot].ensure(sizeof(int32_t) * (size_t)std::max(e2, 1)));
    HIP_TRY(ws.g_w[slot].ensure(sizeof(int32_t) * (size_t)std::max(e2, 1)));
    int32_t* off2 = ws.g_off[slot].as<int32_t>();
    HIP_TRY(hipMemsetAsync(ws.g_w[slot].p, 0, sizeof(int32_t) * (size_t)std::max(e2, 1), s));
    HIP_TRY(launch_segment_reduce(keys, vals, ws.head.as<int32_t>(), E, colbits, ws.g_idx[slot].as<int32_t>(),
                                  ws.g_w[slot].as<int32_t>(), keys2, s));
    HIP_TRY(launch_row_offsets(keys2, e2, n2, colbits, off2, s));
    out.n2 = n2;
    out.nnz2 = e2;
    out.off = off2;
    out.idx = ws.g_idx[slot].as<int32_t>();
    out.w = ws.g_w[slot].as<int32_t>();
    out.k = ws.g_k[slot].as<int32_t>();
    out.q_end = g->M * q2[0] - q2[1];
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

static lv_status graph_setup(lv_graph* g, int32_t n, const int32_t* offsets, const int32_t* indices,
                             const int32_t* weights, lv_memkind kind, uint32_t flags)
{
    hipStream_t s = g->stream;
    HIP_TRY(hipHostMalloc((void**)&g->pinned, 4096, hipHostMallocDefault));
    // offsets first: nnz is needed to size the rest
    HIP_TRY(g->off.ensure(sizeof(int32_t) * ((size_t)n + 1)));
    HIP_TRY(hipMemcpyAsync(g->off.p, offsets, sizeof(int32_t) * ((size_t)n + 1),
                           kind == LV_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, s));
    int32_t first_last[2];
    HIP_TRY(hipMemcpyAsync(&first_last[0], g->off.as<int32_t>(), sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&first_last[1], g->off.as<int32_t>() + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (first_last[0] != 0 || first_last[1] < 0) { set_error_msg("offsets[0] must be 0 and offsets[n] >= 0"); return LV_E_CSR; }
    const int64_t nnz = first_last[1];
    g->n = n;
    g->nnz = nnz;
    HIP_TRY(g->idx.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(nnz, 1)));
    if (nnz > 0)
        HIP_TRY(hipMemcpyAsync(g->idx.p, indices, sizeof(int32_t) * (size_t)nnz,
                               kind == LV_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, s));
    Workspace& ws = g->ws;
    HIP_TRY(ws.small.ensure(4096));
    int32_t* d_err = ws.small.as<int32_t>();
    HIP_TRY(hipMemsetAsync(d_err, 0, 16, s));
    // caller weights staged in the w buffer (converted in place below)
    HIP_TRY(g->w.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(nnz, 1)));
    if (weights && nnz > 0)
        HIP_TRY(hipMemcpyAsync(g->w.p, weights, sizeof(int32_t) * (size_t)nnz,
                               kind == LV_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, s));
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
    int64_t* d_tot = (int64_t*)(ws.small.as<char>() + 64);
    HIP_TRY(hipMemsetAsync(d_tot, 0, 3 * sizeof(int64_t), s));
    if (g->weighted) {
        HIP_TRY(launch_adjacency_weights(n, w_in, diag, nnz, g->w.as<int32_t>(), d_err, s));
        HIP_TRY(ws.k64.ensure(sizeof(int64_t) * (size_t)std::max(n, 1)));
        HIP_TRY(launch_row_sums(n, g->off.as<int32_t>(), g->w.as<int32_t>(), nnz, g->k.as<int32_t>(),
                                ws.k64.as<int64_t>(), d_tot, s));
        ws.k64.release();
    } else {
        g->w.release();
        HIP_TRY(launch_degree_unit(n, g->off.as<int32_t>(), g->k.as<int32_t>(), s));
        if (nnz > 0) {
            int64_t t = nnz;
            HIP_TRY(hipMemcpyAsync(d_tot, &t, sizeof t, hipMemcpyHostToDevice, s));
        }
    }
    int64_t tot = 0;
    HIP_TRY(hipMemcpyAsync(&err, d_err, sizeof err, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&tot, d_tot, sizeof tot, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if ((err & 16) || tot > (int64_t)INT32_MAX) { set_error_msg("total volume M >= 2^31"); return LV_E_OVERFLOW; }
    g->M = tot;
    int64_t* d_q = d_tot + 1;
    HIP_TRY(launch_sum_sq_trace(n, g->off.as<int32_t>(), g->idx.as<int32_t>(), g->weighted ? g->w.as<int32_t>() : nullptr,
                                nnz, g->k.as<int32_t>(), d_q, s));
    int64_t q2[2];
    HIP_TRY(hipMemcpyAsync(q2, d_q, sizeof q2, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    g->sumk2 = q2[0];
    g->trace = q2[1];
    return LV_OK;
}

lv_status lv_graph_create_csr(int32_t n, const int32_t* offsets, const int32_t* indices, const int32_t* weights,
                              lv_memkind kind, uint32_t flags, void* stream, lv_graph** out)
{
    if (!out || n < 0 || !offsets || (kind != LV_MEM_HOST && kind != LV_MEM_DEVICE)) {
        set_error_msg("lv_graph_create_csr: null out/offsets, n < 0 or bad memkind");
        return LV_E_ARG;
    }
    if (n == INT32_MAX) { set_error_msg("n must be < 2^31 - 1"); return LV_E_OVERFLOW; }
    if (kind == LV_MEM_HOST) {
        if ((int64_t)offsets[n] > 0 && !indices) { set_error_msg("indices is null"); return LV_E_ARG; }
    } else if (!indices) {
        set_error_msg("indices is null");
        return LV_E_ARG;
    }
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
        set_error("lv_graph_create_csr", e);
        delete g;
        return from_hip(e);
    }
    lv_status st = graph_setup(g, n, offsets, indices, weights, kind, flags);
    if (st != LV_OK) {
        (void)hipStreamSynchronize(g->stream);
        delete g;
        return st;
    }
    *out = g;
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
    if (volume) *volume = g->M;
    return LV_OK;
}

static lv_status louvain_impl(lv_graph* g, const Params& p, bool keep_graphs, lv_result* r)
{
    hipStream_t s = g->stream;
    Workspace& ws = g->ws;
    r->n0 = g->n;
    r->M = g->M;
    HIP_TRY(r->final_labels.ensure(sizeof(int32_t) * (size_t)std::max(g->n, 1)));
    HIP_TRY(launch_iota(r->final_labels.as<int32_t>(), g->n, s));
    LevelGraph G{g->n, g->nnz, g->off.as<int32_t>(), g->idx.as<int32_t>(), g->weighted ? g->w.as<int32_t>() : nullptr,
                 g->k.as<int32_t>()};
    int64_t q_start = g->M * g->trace - g->sumk2;
    r->q_int = q_start;
    int slot = 0;
    Timer tm;
    tm.on = (p.flags & LV_TIMING) != 0;
    tm.s = s;
    for (;;) {
        auto rec = std::make_unique<LevelRecord>();
        SweepOut so;
        LV_TRY(run_sweeps(g, G, MODE_LOUVAIN, p, so));
        hipEvent_t t0{}, t1{}, t2{};
        if (tm.on) HIP_TRY(tm.mark(&t0));
        int32_t n2 = 0;
        LV_TRY(renumber(g, G.n, &n2));
        if (tm.on) HIP_TRY(tm.mark(&t1));
        Coarse co;
        LV_TRY(aggregate(g, G, n2, slot, co));
        if (tm.on) {
            HIP_TRY(tm.mark(&t2));
            HIP_TRY(hipStreamSynchronize(s));
            rec->info.renumber_ms = elapsed(t0, t1);
            rec->info.aggregate_ms = elapsed(t1, t2);
            tm.used = 0;
        }
        lv_level_info& li = rec->info;
        li.n = G.n;
        li.n_next = n2;
        li.nnz = G.nnz;
        li.sweeps = (int32_t)so.moves.size();
        li.q_start = q_start;
        li.q_end = co.q_end;
        li.accepted = co.q_end > q_start ? 1 : 0;
        li.move_ms = so.move_ms;
        li.sweep_ms = so.sweep_ms;
        li.move_launches = so.launches;
        li.move_bytes = so.bytes;
        for (int t = 0; t < LV_KERNEL_SLOTS; ++t) {
            li.kern_ms[t] = so.kern_ms[t];
            li.kern_launches[t] = so.kern_launches[t];
            li.kern_bytes[t] = so.kern_bytes[t];
        }
        rec->moves = so.moves;
        const bool accepted = li.accepted != 0;
        if (accepted) {
            HIP_TRY(rec->labels.ensure(sizeof(int32_t) * (size_t)std::max(G.n, 1)));
            HIP_TRY(launch_copy_i32(rec->labels.as<int32_t>(), ws.labels.as<int32_t>(), G.n, s));
            HIP_TRY(launch_compose(g->n, r->final_labels.as<int32_t>(), ws.labels.as<int32_t>(), s));
            if (keep_graphs) {
                HIP_TRY(rec->g_off.ensure(sizeof(int32_t) * ((size_t)co.n2 + 1)));
                HIP_TRY(rec->g_idx.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(co.nnz2, 1)));
                HIP_TRY(rec->g_w.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(co.nnz2, 1)));
                HIP_TRY(launch_copy_i32(rec->g_off.as<int32_t>(), co.off, (int64_t)co.n2 + 1, s));
                HIP_TRY(launch_copy_i32(rec->g_idx.as<int32_t>(), co.idx, co.nnz2, s));
                HIP_TRY(launch_copy_i32(rec->g_w.as<int32_t>(), co.w, co.nnz2, s));
                rec->g_nnz = co.nnz2;
            }
            r->q_int = co.q_end;
            ++r->accepted;
        }
        r->levels.push_back(std::move(rec));
        if (!accepted || r->accepted >= p.max_levels) break;
        G = LevelGraph{co.n2, co.nnz2, co.off, co.idx, co.w, co.k};
        q_start = co.q_end;
        slot ^= 1;
    }
    HIP_TRY(hipStreamSynchronize(s));
    return LV_OK;
}

lv_status lv_louvain(lv_graph* g, const lv_params* params, lv_result** out)
{
    if (!g || !out) { set_error_msg("lv_louvain: null graph or out"); return LV_E_ARG; }
    Params p;
    LV_TRY(read_params(params, p));
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

lv_status lv_result_num_levels(const lv_result* r, int32_t* accepted, int32_t* attempted)
{
    if (!r) return LV_E_ARG;
    if (accepted) *accepted = r->accepted;
    if (attempted) *attempted = (int32_t)r->levels.size();
    return LV_OK;
}

lv_status lv_result_level_info(const lv_result* r, int32_t level, lv_level_info* out)
{
    if (!r || !out) return LV_E_ARG;
    if (level < 0 || level >= (int32_t)r->levels.size()) return LV_E_NOT_FOUND;
    *out = r->levels[level]->info;
    return LV_OK;
}

lv_status lv_result_level_moves(const lv_result* r, int32_t level, int64_t* moves, int32_t cap)
{
    if (!r || (!moves && cap > 0) || cap < 0) return LV_E_ARG;
    if (level < 0 || level >= (int32_t)r->levels.size()) return LV_E_NOT_FOUND;
    const auto& mv = r->levels[level]->moves;
    for (int32_t t = 0; t < cap && t < (int32_t)mv.size(); ++t) moves[t] = mv[t];
    return LV_OK;
}

lv_status lv_result_level_labels(const lv_result* r, int32_t level, int32_t* labels, lv_memkind kind)
{
    if (!r || !labels) return LV_E_ARG;
    if (level < 0 || level >= r->accepted) return LV_E_NOT_FOUND;
    const LevelRecord& rec = *r->levels[level];
    return copy_out(labels, rec.labels.as<int32_t>(), rec.info.n, kind, nullptr);
}

lv_status lv_result_level_graph(const lv_result* r, int32_t level, int32_t* offsets, int32_t* indices,
                                int32_t* weights, int64_t* nnz, lv_memkind kind)
{
    if (!r || !nnz) return LV_E_ARG;
    if (level < 0 || level >= r->accepted) return LV_E_NOT_FOUND;
    const LevelRecord& rec = *r->levels[level];
    if (!rec.g_off.p) return LV_E_STATE;
    *nnz = rec.g_nnz;
    if (offsets) LV_TRY(copy_out(offsets, rec.g_off.as<int32_t>(), (int64_t)rec.info.n_next + 1, kind, nullptr));
    if (indices) LV_TRY(copy_out(indices, rec.g_idx.as<int32_t>(), rec.g_nnz, kind, nullptr));
    if (weights) LV_TRY(copy_out(weights, rec.g_w.as<int32_t>(), rec.g_nnz, kind, nullptr));
    return LV_OK;
}

lv_status lv_result_final_labels(const lv_result* r, int32_t* labels, lv_memkind kind)
{
    if (!r || !labels) return LV_E_ARG;
    return copy_out(labels, r->final_labels.as<int32_t>(), r->n0, kind, nullptr);
}

lv_status lv_result_modularity(const lv_result* r, int64_t* q_int, int64_t* m, double* q)
{
    if (!r) return LV_E_ARG;
    if (q_int) *q_int = r->q_int;
    if (m) *m = r->M;
    if (q) *q = r->M > 0 ? (double)r->q_int / ((double)r->M * (double)r->M) : 0.0;
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
    *q_int = g->M * q2[0] - q2[1];
    return LV_OK;
}

lv_status lv_modularity(lv_graph* g, const int32_t* labels, lv_memkind kind, int64_t* q_int, int64_t* m, double* q)
{
    if (!g || !labels || (kind != LV_MEM_HOST && kind != LV_MEM_DEVICE)) return LV_E_ARG;
    Workspace& ws = g->ws;
    const int32_t* dl = labels;
    if (kind == LV_MEM_HOST) {
        HIP_TRY(ws.labels.ensure(sizeof(int32_t) * (size_t)std::max(g->n, 1)));
        if (g->n > 0)
            HIP_TRY(hipMemcpyAsync(ws.labels.p, labels, sizeof(int32_t) * (size_t)g->n, hipMemcpyHostToDevice, g->stream));
        dl = ws.labels.as<int32_t>();
    }
    int64_t qi = 0;
    LV_TRY(modularity_impl(g, dl, &qi));
    if (q_int) *q_int = qi;
    if (m) *m = g->M;
    if (q) *q = g->M > 0 ? (double)qi / ((double)g->M * (double)g->M) : 0.0;
    return LV_OK;
}

lv_status lv_lpa(lv_graph* g, const lv_params* params, int32_t* labels, lv_memkind kind, lv_level_info* info,
                 int64_t* moves_out, int32_t moves_cap)
{
    if (!g || !labels || (kind != LV_MEM_HOST && kind != LV_MEM_DEVICE) || moves_cap < 0 || (moves_cap > 0 && !moves_out))
        return LV_E_ARG;
    Params p;
    LV_TRY(read_params(params, p));
    LevelGraph G{g->n, g->nnz, g->off.as<int32_t>(), g->idx.as<int32_t>(), g->weighted ? g->w.as<int32_t>() : nullptr,
                 g->k.as<int32_t>()};
    SweepOut so;
    LV_TRY(run_sweeps(g, G, MODE_LPA, p, so));
    int32_t n2 = 0;
    hipEvent_t t0{}, t1{};
    Timer tm;
    tm.on = (p.flags & LV_TIMING) != 0;
    tm.s = g->stream;
    if (tm.on) HIP_TRY(tm.mark(&t0));
    LV_TRY(renumber(g, g->n, &n2));
    if (tm.on) HIP_TRY(tm.mark(&t1));
    // Q_int of the final partition: M * Sigma_in - sum of the community volumes squared
    int64_t* d_q = (int64_t*)(g->ws.small.as<char>() + 2816);
    HIP_TRY(hipMemsetAsync(d_q, 0, 2 * sizeof(int64_t), g->stream));
    HIP_TRY(launch_sigma_in(G.n, G.off, G.idx, G.w, G.nnz, g->ws.comm.as<int32_t>(), d_q, g->stream));
    HIP_TRY(launch_sum_sq(g->ws.sigma.as<int32_t>(), G.n, d_q + 1, g->stream));
    int64_t q2[2];
    HIP_TRY(hipMemcpyAsync(g->pinned, d_q, sizeof q2, hipMemcpyDeviceToHost, g->stream));
    HIP_TRY(hipStreamSynchronize(g->stream));
    std::memcpy(q2, g->pinned, sizeof q2);
    const int64_t qi = g->M * q2[0] - q2[1];
    LV_TRY(copy_out(labels, g->ws.labels.as<int32_t>(), g->n, kind, g->stream));
    for (int32_t t = 0; t < moves_cap && t < (int32_t)so.moves.size(); ++t) moves_out[t] = so.moves[t];
    if (info) {
        lv_level_info li{};
        li.n = g->n;
        li.n_next = n2;
        li.nnz = g->nnz;
        li.sweeps = (int32_t)so.moves.size();
        li.q_start = g->M * g->trace - g->sumk2;
        li.q_end = qi;
        li.accepted = 1;
        li.move_ms = so.move_ms;
        li.sweep_ms = so.sweep_ms;
        li.renumber_ms = tm.on ? elapsed(t0, t1) : 0.0;
        li.move_launches = so.launches;
        li.move_bytes = so.bytes;
        for (int t = 0; t < LV_KERNEL_SLOTS; ++t) {
            li.kern_ms[t] = so.kern_ms[t];
            li.kern_launches[t] = so.kern_launches[t];
            li.kern_bytes[t] = so.kern_bytes[t];
        }
        *info = li;
    }
    return LV_OK;
}

}  // extern "C"
