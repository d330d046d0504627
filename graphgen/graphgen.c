/*
 * Seeded synthetic graph generators.
 *
 * Shared input source for the CPU oracle and the GPU library: it contains no
 * community-detection arithmetic, only sampling and CSR canonicalisation.
 *
 * Every generator is deterministic for a given seed and independent of the
 * OpenMP thread count: random numbers come from a counter-based generator
 * (SplitMix64's output function, Steele, Lea and Flood, OOPSLA 2014, applied
 * to key + (counter+1) * golden-ratio increment), and the CSR builder sorts
 * every row, so scheduling never shows in the output.
 *
 * Output CSR contract (the graph model of the paper's Section II-A: undirected,
 * unit weight when unweighted): symmetric, int32 row offsets, column indices
 * strictly increasing within each row, no self-loops, no duplicate entries.
 * Buffers are malloc'd here and released with gg_free().
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define GG_OK 0
#define GG_E_ARG 1
#define GG_E_NOMEM 2
#define GG_E_TOO_BIG 3

static const uint64_t GOLDEN = 0x9E3779B97F4A7C15ULL;

static inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* The counter-th output of a SplitMix64 stream whose state starts at key. */
static inline uint64_t rnd(uint64_t key, uint64_t counter)
{
    return mix64(key + (counter + 1) * GOLDEN);
}

static inline uint64_t stream_key(uint64_t seed, uint64_t tag)
{
    return mix64(seed * GOLDEN ^ mix64(tag + 0x632BE59BD9B4E019ULL));
}

/* Uniform double in [0,1) from the top 53 bits. */
static inline double u01(uint64_t h) { return (double)(h >> 11) * (1.0 / 9007199254740992.0); }

void gg_free(void* p) { free(p); }

/* OpenMP team size for the calling thread's later generator calls */
void gg_set_threads(int t) { if (t > 0) omp_set_num_threads(t); }

uint64_t gg_rand(uint64_t key, uint64_t counter) { return rnd(key, counter); }
uint64_t gg_stream_key(uint64_t seed, uint64_t tag) { return stream_key(seed, tag); }

static int cmp_i32(const void* a, const void* b)
{
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

/*
 * Undirected edge list -> canonical symmetric CSR.  Pairs with u == v are
 * dropped, both directions of every other pair are stored, duplicates are
 * merged (kept once).  Endpoints must lie in [0, n).
 */
static int build_csr(int32_t n, int64_t m, const int32_t* eu, const int32_t* ev,
                     int32_t** off_out, int32_t** idx_out, int64_t* nnz_out)
{
    int64_t* pos = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    if (!pos) return GG_E_NOMEM;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; ++e) {
        int32_t u = eu[e], v = ev[e];
        if (u == v) continue;
#pragma omp atomic
        pos[u + 1]++;
#pragma omp atomic
        pos[v + 1]++;
    }
    for (int32_t i = 0; i < n; ++i) pos[i + 1] += pos[i];
    int64_t total = pos[n];
    int32_t* tmp = (int32_t*)malloc((size_t)(total > 0 ? total : 1) * sizeof(int32_t));
    int64_t* cur = (int64_t*)malloc((size_t)(n + 1) * sizeof(int64_t));
    if (!tmp || !cur) { free(pos); free(tmp); free(cur); return GG_E_NOMEM; }
    memcpy(cur, pos, (size_t)(n + 1) * sizeof(int64_t));
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; ++e) {
        int32_t u = eu[e], v = ev[e];
        if (u == v) continue;
        int64_t p, q;
#pragma omp atomic capture
        p = cur[u]++;
#pragma omp atomic capture
        q = cur[v]++;
        tmp[p] = v;
        tmp[q] = u;
    }
    free(cur);
    int64_t* uniq = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    if (!uniq) { free(pos); free(tmp); return GG_E_NOMEM; }
#pragma omp parallel for schedule(dynamic, 256)
    for (int32_t r = 0; r < n; ++r) {
        int64_t b = pos[r], e = pos[r + 1];
        if (e - b > 1) qsort(tmp + b, (size_t)(e - b), sizeof(int32_t), cmp_i32);
        int64_t u = 0;
        for (int64_t t = b; t < e; ++t)
            if (t == b || tmp[t] != tmp[t - 1]) ++u;
        uniq[r + 1] = u;
    }
    for (int32_t i = 0; i < n; ++i) uniq[i + 1] += uniq[i];
    int64_t nnz = uniq[n];
    if (nnz > INT32_MAX) { free(pos); free(tmp); free(uniq); return GG_E_TOO_BIG; }
    int32_t* off = (int32_t*)malloc((size_t)(n + 1) * sizeof(int32_t));
    int32_t* idx = (int32_t*)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
    if (!off || !idx) { free(pos); free(tmp); free(uniq); free(off); free(idx); return GG_E_NOMEM; }
#pragma omp parallel for schedule(dynamic, 256)
    for (int32_t r = 0; r < n; ++r) {
        int64_t b = pos[r], e = pos[r + 1], o = uniq[r];
        off[r] = (int32_t)o;
        for (int64_t t = b; t < e; ++t)
            if (t == b || tmp[t] != tmp[t - 1]) idx[o++] = tmp[t];
    }
    off[n] = (int32_t)nnz;
    free(pos); free(tmp); free(uniq);
    *off_out = off; *idx_out = idx; *nnz_out = nnz;
    return GG_OK;
}

int gg_csr_from_edges(int32_t n, int64_t m, const int32_t* eu, const int32_t* ev,
                      int32_t** off, int32_t** idx, int64_t* nnz)
{
    if (n < 0 || m < 0) return GG_E_ARG;
    for (int64_t e = 0; e < m; ++e)
        if (eu[e] < 0 || eu[e] >= n || ev[e] < 0 || ev[e] >= n) return GG_E_ARG;
    return build_csr(n, m, eu, ev, off, idx, nnz);
}

/*
 * R-MAT (Chakrabarti, Zhan, Faloutsos, SDM 2004): each of `samples` edges
 * descends `scale` levels, choosing quadrant (row bit, col bit) = (0,0), (0,1),
 * (1,0), (1,1) with probabilities a, b, c, 1-a-b-c.  No noise, no id
 * permutation.  Endpoints >= n are dropped (n <= 2^scale).  Each level draws a
 * 32-bit uniform; two levels share one 64-bit counter output.
 */
int gg_rmat_edges(int32_t scale, int32_t n, int64_t samples, double a, double b, double c, uint64_t seed,
                  int32_t* eu, int32_t* ev)
{
    if (scale < 1 || scale > 30 || n < 1 || n > (1LL << scale) || samples < 0) return GG_E_ARG;
    if (a < 0 || b < 0 || c < 0 || a + b + c > 1.0) return GG_E_ARG;
    const uint64_t ta = (uint64_t)(a * 4294967296.0);
    const uint64_t tb = (uint64_t)((a + b) * 4294967296.0);
    const uint64_t tc = (uint64_t)((a + b + c) * 4294967296.0);
    const uint64_t key = stream_key(seed, 0x524D4154ULL);
    const int draws = (scale + 1) / 2;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < samples; ++e) {
        uint32_t r = 0, col = 0;
        uint64_t h = 0;
        for (int l = 0; l < scale; ++l) {
            if ((l & 1) == 0) h = rnd(key, (uint64_t)e * (uint64_t)draws + (uint64_t)(l >> 1));
            uint64_t u = (l & 1) ? (h >> 32) : (h & 0xFFFFFFFFULL);
            uint32_t rb, cb;
            if (u < ta) { rb = 0; cb = 0; }
            else if (u < tb) { rb = 0; cb = 1; }
            else if (u < tc) { rb = 1; cb = 0; }
            else { rb = 1; cb = 1; }
            r = (r << 1) | rb;
            col = (col << 1) | cb;
        }
        if ((int64_t)r >= n || (int64_t)col >= n) { eu[e] = 0; ev[e] = 0; }  /* dropped as a loop */
        else { eu[e] = (int32_t)r; ev[e] = (int32_t)col; }
    }
    return GG_OK;
}

int gg_rmat(int32_t scale, int32_t n, int64_t samples, double a, double b, double c,
            uint64_t seed, int32_t** off, int32_t** idx, int64_t* nnz)
{
    if (samples < 0) return GG_E_ARG;
    int32_t* eu = (int32_t*)malloc((size_t)(samples > 0 ? samples : 1) * sizeof(int32_t));
    int32_t* ev = (int32_t*)malloc((size_t)(samples > 0 ? samples : 1) * sizeof(int32_t));
    if (!eu || !ev) { free(eu); free(ev); return GG_E_NOMEM; }
    int rc = gg_rmat_edges(scale, n, samples, a, b, c, seed, eu, ev);
    if (rc == GG_OK) rc = build_csr(n, samples, eu, ev, off, idx, nnz);
    free(eu); free(ev);
    return rc;
}

/*
 * Planted-partition stochastic block model.  Vertices are cut into blocks of
 * `block_size` (the last block takes the remainder).  Each unordered pair
 * {i, j}, i != j, is an edge independently with probability p_in (same block)
 * or p_out.  Pairs of one block pair are enumerated in a fixed linear order
 * and sampled by geometric skips (Batagelj and Brandes, Phys. Rev. E 71,
 * 2005), which draws exactly the per-pair Bernoulli distribution.
 */
static int64_t sbm_pair_stream(int32_t n, int32_t bs, int32_t nb, int64_t pq, double p_in,
                               double p_out, uint64_t key, int32_t* eu, int32_t* ev)
{
    int32_t P = 0;
    int64_t rem = pq;
    while (rem >= nb - P) { rem -= nb - P; ++P; }
    int32_t Q = P + (int32_t)rem;
    int32_t p0 = P * bs, q0 = Q * bs;
    int32_t sp = (P == nb - 1) ? n - p0 : bs;
    int32_t sq = (Q == nb - 1) ? n - q0 : bs;
    double p = (P == Q) ? p_in : p_out;
    int64_t count = (P == Q) ? (int64_t)sp * (sp - 1) / 2 : (int64_t)sp * sq;
    if (p <= 0.0 || count == 0) return 0;
    uint64_t skey = mix64(key ^ ((uint64_t)pq * 0xD1B54A32D192ED03ULL));
    double lq = (p >= 1.0) ? 0.0 : log1p(-p);
    int64_t t = -1, emitted = 0;
    uint64_t draw = 0;
    for (;;) {
        int64_t skip = 0;
        if (p < 1.0) {
            double u = u01(rnd(skey, draw++));
            double s = floor(log1p(-u) / lq);
            if (s > (double)count) break;
            skip = (int64_t)s;
        }
        t += 1 + skip;
        if (t >= count) break;
        int32_t i, j;
        if (P == Q) {
            /* t enumerates pairs (i < j) row by row: row i holds sp-1-i pairs */
            int64_t rr = t;
            int32_t r = 0;
            /* closed-form start, then fix up */
            double dn = (double)sp;
            double est = floor(dn - 0.5 - sqrt((dn - 0.5) * (dn - 0.5) - 2.0 * (double)rr));
            if (est < 0) est = 0;
            r = (int32_t)est;
            int64_t start = (int64_t)r * (2LL * sp - r - 1) / 2;
            while (r > 0 && start > rr) { --r; start = (int64_t)r * (2LL * sp - r - 1) / 2; }
            while (start + (sp - 1 - r) <= rr) { start += sp - 1 - r; ++r; }
            i = p0 + r;
            j = p0 + r + 1 + (int32_t)(rr - start);
        } else {
            i = p0 + (int32_t)(t / sq);
            j = q0 + (int32_t)(t % sq);
        }
        if (eu) { eu[emitted] = i; ev[emitted] = j; }
        ++emitted;
    }
    return emitted;
}

int gg_sbm(int32_t n, int32_t block_size, double p_in, double p_out, uint64_t seed,
           int32_t** off, int32_t** idx, int64_t* nnz)
{
    if (n < 1 || block_size < 1 || p_in < 0 || p_in > 1 || p_out < 0 || p_out > 1) return GG_E_ARG;
    int32_t nb = (n + block_size - 1) / block_size;
    int64_t npairs = (int64_t)nb * (nb + 1) / 2;
    uint64_t key = stream_key(seed, 0x53424DULL);
    int64_t* cnt = (int64_t*)calloc((size_t)npairs + 1, sizeof(int64_t));
    if (!cnt) return GG_E_NOMEM;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t pq = 0; pq < npairs; ++pq)
        cnt[pq + 1] = sbm_pair_stream(n, block_size, nb, pq, p_in, p_out, key, NULL, NULL);
    for (int64_t t = 0; t < npairs; ++t) cnt[t + 1] += cnt[t];
    int64_t m = cnt[npairs];
    int32_t* eu = (int32_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    int32_t* ev = (int32_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    if (!eu || !ev) { free(cnt); free(eu); free(ev); return GG_E_NOMEM; }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t pq = 0; pq < npairs; ++pq)
        sbm_pair_stream(n, block_size, nb, pq, p_in, p_out, key, eu + cnt[pq], ev + cnt[pq]);
    free(cnt);
    int rc = build_csr(n, m, eu, ev, off, idx, nnz);
    free(eu); free(ev);
    return rc;
}

/*
 * Per-entry weights for a canonical CSR: w(u,v) = lo + (hash(seed, min, max)
 * mod (hi-lo+1)), identical for both directions of a pair.
 */
int gg_pair_weights(int32_t n, const int32_t* off, const int32_t* idx, int32_t lo, int32_t hi,
                    uint64_t seed, int32_t* w)
{
    if (lo < 1 || hi < lo) return GG_E_ARG;
    uint64_t key = stream_key(seed, 0x574754ULL);
    uint64_t span = (uint64_t)(hi - lo) + 1;
#pragma omp parallel for schedule(dynamic, 1024)
    for (int32_t r = 0; r < n; ++r)
        for (int32_t e = off[r]; e < off[r + 1]; ++e) {
            int32_t c = idx[e];
            uint64_t a = (uint64_t)(r < c ? r : c), b = (uint64_t)(r < c ? c : r);
            w[e] = lo + (int32_t)(rnd(key, (a << 32) | b) % span);
        }
    return GG_OK;
}

/*
 * LFR-style benchmark graph, after the method description of Lancichinetti,
 * Fortunato and Radicchi (Phys. Rev. E 78, 046110, 2008):
 *   1. degrees k_v from a power law with exponent tau1 on [kmin, kmax], where
 *      kmin is solved so that the (continuous) mean equals mean_deg;
 *   2. community sizes from a power law with exponent tau2 on [smin, smax],
 *      drawn until they cover n (the last size is trimmed; a remainder below
 *      smin is spread over the earlier communities);
 *   3. each vertex splits its degree into round((1-mu) k) internal and the rest
 *      external stubs, and joins a community larger than its internal degree,
 *      chosen with probability proportional to remaining capacity (largest
 *      internal degrees placed first);
 *   4. internal stubs are paired by a configuration model inside each
 *      community, external stubs by one configuration model over all vertices.
 * Simplifications (documented): self-loops and multi-edges produced by the
 * pairing are dropped instead of rewired, and external pairs that land inside
 * one community are kept.  Weights are attached separately (gg_pair_weights).
 * Output membership[v] is the planted community of v.
 */
static double pl_sample(double u, double lo, double hi, double tau)
{
    double e = 1.0 - tau;
    double a = pow(lo, e), b = pow(hi, e);
    return pow(a + u * (b - a), 1.0 / e);
}

static double pl_mean(double lo, double hi, double tau)
{
    double num = (pow(hi, 2.0 - tau) - pow(lo, 2.0 - tau)) / (2.0 - tau);
    double den = (pow(hi, 1.0 - tau) - pow(lo, 1.0 - tau)) / (1.0 - tau);
    return num / den;
}

/* Fenwick tree over remaining community capacities. */
static void fw_add(int64_t* t, int32_t n, int32_t i, int64_t d)
{
    for (++i; i <= n; i += i & -i) t[i] += d;
}
static int64_t fw_prefix(const int64_t* t, int32_t i)
{
    int64_t s = 0;
    for (; i > 0; i -= i & -i) s += t[i];
    return s;
}
/* smallest index i with prefix(i+1) > target */
static int32_t fw_find(const int64_t* t, int32_t n, int64_t target)
{
    int32_t pos = 0, step = 1;
    while (step * 2 <= n) step *= 2;
    for (; step > 0; step >>= 1)
        if (pos + step <= n && t[pos + step] <= target) { pos += step; target -= t[pos]; }
    return pos;
}

typedef struct { int32_t kint; uint32_t tie; int32_t v; } lfr_vrec;
static int cmp_vrec(const void* a, const void* b)
{
    const lfr_vrec* x = (const lfr_vrec*)a;
    const lfr_vrec* y = (const lfr_vrec*)b;
    if (x->kint != y->kint) return (x->kint < y->kint) - (x->kint > y->kint);  /* descending */
    if (x->tie != y->tie) return (x->tie > y->tie) - (x->tie < y->tie);
    return (x->v > y->v) - (x->v < y->v);
}

static void shuffle_i32(int32_t* a, int64_t len, uint64_t key)
{
    for (int64_t i = len - 1; i > 0; --i) {
        int64_t j = (int64_t)(rnd(key, (uint64_t)i) % (uint64_t)(i + 1));
        int32_t t = a[i]; a[i] = a[j]; a[j] = t;
    }
}

int gg_lfr(int32_t n, double tau1, double mean_deg, int32_t kmax, double tau2, int32_t smin,
           int32_t smax, double mu, uint64_t seed, int32_t** off, int32_t** idx, int64_t* nnz,
           int32_t** membership_out, int32_t* ncomm_out)
{
    if (n < 2 || tau1 <= 2.0 || tau2 <= 1.0 || kmax < 2 || smin < 2 || smax < smin || mu < 0 || mu > 1 ||
        mean_deg < 1.0 || mean_deg >= kmax || (int64_t)smax > n)
        return GG_E_ARG;
    /* 1. kmin by bisection on the continuous mean */
    double lo = 1.0, hi = (double)kmax;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (pl_mean(mid, kmax, tau1) < mean_deg) lo = mid; else hi = mid;
    }
    double kmin = 0.5 * (lo + hi);
    int32_t* deg = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    int32_t* kint = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    int32_t* memb = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    if (!deg || !kint || !memb) { free(deg); free(kint); free(memb); return GG_E_NOMEM; }
    uint64_t kd = stream_key(seed, 0x4C46524BULL);
#pragma omp parallel for schedule(static)
    for (int32_t v = 0; v < n; ++v) {
        double x = pl_sample(u01(rnd(kd, (uint64_t)v)), kmin, (double)kmax, tau1);
        int32_t k = (int32_t)floor(x + 0.5);
        if (k < 1) k = 1;
        if (k > kmax) k = kmax;
        deg[v] = k;
        kint[v] = (int32_t)floor((1.0 - mu) * k + 0.5);
    }
    /* 2. community sizes */
    int32_t cap_c = n / smin + 2, nc = 0;
    int32_t* size = (int32_t*)malloc((size_t)cap_c * sizeof(int32_t));
    if (!size) { free(deg); free(kint); free(memb); return GG_E_NOMEM; }
    uint64_t ks = stream_key(seed, 0x4C465253ULL);
    int64_t covered = 0;
    while (covered < n) {
        double x = pl_sample(u01(rnd(ks, (uint64_t)nc)), (double)smin, (double)smax, tau2);
        int32_t s = (int32_t)floor(x + 0.5);
        if (s < smin) s = smin;
        if (s > smax) s = smax;
        if (covered + s > n) s = (int32_t)(n - covered);
        size[nc++] = s;
        covered += s;
    }
    if (nc > 1 && size[nc - 1] < smin) {  /* spread a short remainder */
        int32_t r = size[--nc];
        for (int32_t t = 0; r > 0; t = (t + 1) % nc, --r) size[t]++;
    }
    /* communities by size, descending (stable by index) */
    int32_t* corder = (int32_t*)malloc((size_t)nc * sizeof(int32_t));
    int64_t* fw = (int64_t*)calloc((size_t)nc + 1, sizeof(int64_t));
    lfr_vrec* vr = (lfr_vrec*)malloc((size_t)n * sizeof(lfr_vrec));
    if (!corder || !fw || !vr) {
        free(deg); free(kint); free(memb); free(size); free(corder); free(fw); free(vr);
        return GG_E_NOMEM;
    }
    for (int32_t t = 0; t < nc; ++t) corder[t] = t;
    for (int32_t t = 1; t < nc; ++t) {  /* insertion sort keeps it simple; nc ~ n / 1000 */
        int32_t x = corder[t], j = t - 1;
        while (j >= 0 && (size[corder[j]] < size[x])) { corder[j + 1] = corder[j]; --j; }
        corder[j + 1] = x;
    }
    int64_t* remaining = (int64_t*)malloc((size_t)nc * sizeof(int64_t));
    if (!remaining) {
        free(deg); free(kint); free(memb); free(size); free(corder); free(fw); free(vr);
        return GG_E_NOMEM;
    }
    for (int32_t t = 0; t < nc; ++t) { remaining[t] = size[corder[t]]; fw_add(fw, nc, t, remaining[t]); }
    /* 3. place vertices, largest internal degree first */
    uint64_t kt = stream_key(seed, 0x4C465254ULL);
    for (int32_t v = 0; v < n; ++v) { vr[v].kint = kint[v]; vr[v].tie = (uint32_t)rnd(kt, (uint64_t)v); vr[v].v = v; }
    qsort(vr, (size_t)n, sizeof(lfr_vrec), cmp_vrec);
    uint64_t kp = stream_key(seed, 0x4C465250ULL);
    for (int32_t t = 0; t < n; ++t) {
        int32_t v = vr[t].v;
        /* eligible: communities (in size order) with size > kint: a prefix */
        int32_t lo_i = 0, hi_i = nc;
        while (lo_i < hi_i) {
            int32_t mid = (lo_i + hi_i) / 2;
            if (size[corder[mid]] > kint[v]) lo_i = mid + 1; else hi_i = mid;
        }
        int32_t elig = lo_i;
        int64_t cap = fw_prefix(fw, elig);
        int32_t slot;
        if (cap > 0) {
            int64_t target = (int64_t)(rnd(kp, (uint64_t)v) % (uint64_t)cap);
            slot = fw_find(fw, nc, target);
        } else {
            /* no eligible capacity: take the community with the most room and cap kint */
            int64_t best = -1; slot = 0;
            for (int32_t s = 0; s < nc; ++s) if (remaining[s] > best) { best = remaining[s]; slot = s; }
            if (kint[v] > size[corder[slot]] - 1) kint[v] = size[corder[slot]] - 1;
        }
        remaining[slot]--;
        fw_add(fw, nc, slot, -1);
        memb[v] = corder[slot];
    }
    free(vr); free(fw); free(remaining); free(corder);
    /* 4a. internal stubs per community */
    int64_t* cstart = (int64_t*)calloc((size_t)nc + 1, sizeof(int64_t));
    int64_t next_total = 0;
    if (!cstart) { free(deg); free(kint); free(memb); free(size); return GG_E_NOMEM; }
    for (int32_t v = 0; v < n; ++v) cstart[memb[v] + 1] += kint[v];
    for (int32_t t = 0; t < nc; ++t) cstart[t + 1] += cstart[t];
    int64_t nint = cstart[nc];
    int64_t next = 0;
    for (int32_t v = 0; v < n; ++v) next += deg[v] - kint[v];
    next_total = next;
    int32_t* istub = (int32_t*)malloc((size_t)(nint > 0 ? nint : 1) * sizeof(int32_t));
    int32_t* estub = (int32_t*)malloc((size_t)(next_total > 0 ? next_total : 1) * sizeof(int32_t));
    int64_t* cur = (int64_t*)malloc((size_t)(nc + 1) * sizeof(int64_t));
    if (!istub || !estub || !cur) {
        free(deg); free(kint); free(memb); free(size); free(cstart); free(istub); free(estub); free(cur);
        return GG_E_NOMEM;
    }
    memcpy(cur, cstart, (size_t)(nc + 1) * sizeof(int64_t));
    int64_t ep = 0;
    for (int32_t v = 0; v < n; ++v) {
        for (int32_t s = 0; s < kint[v]; ++s) istub[cur[memb[v]]++] = v;
        for (int32_t s = 0; s < deg[v] - kint[v]; ++s) estub[ep++] = v;
    }
    free(cur);
    uint64_t kw = stream_key(seed, 0x4C464957ULL);
#pragma omp parallel for schedule(dynamic, 4)
    for (int32_t cc = 0; cc < nc; ++cc)
        shuffle_i32(istub + cstart[cc], cstart[cc + 1] - cstart[cc], mix64(kw ^ (uint64_t)cc));
    shuffle_i32(estub, next_total, stream_key(seed, 0x4C464557ULL));
    /* 4b. pair consecutive stubs */
    int64_t m = 0;
    int64_t* pstart = (int64_t*)calloc((size_t)nc + 1, sizeof(int64_t));
    if (!pstart) {
        free(deg); free(kint); free(memb); free(size); free(cstart); free(istub); free(estub);
        return GG_E_NOMEM;
    }
    for (int32_t cc = 0; cc < nc; ++cc) pstart[cc + 1] = pstart[cc] + (cstart[cc + 1] - cstart[cc]) / 2;
    m = pstart[nc] + next_total / 2;
    int32_t* eu = (int32_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    int32_t* ev = (int32_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    if (!eu || !ev) {
        free(deg); free(kint); free(memb); free(size); free(cstart); free(istub); free(estub);
        free(pstart); free(eu); free(ev);
        return GG_E_NOMEM;
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (int32_t cc = 0; cc < nc; ++cc) {
        int64_t b = cstart[cc], pairs = (cstart[cc + 1] - cstart[cc]) / 2;
        for (int64_t t = 0; t < pairs; ++t) {
            eu[pstart[cc] + t] = istub[b + 2 * t];
            ev[pstart[cc] + t] = istub[b + 2 * t + 1];
        }
    }
    int64_t base = pstart[nc];
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < next_total / 2; ++t) {
        eu[base + t] = estub[2 * t];
        ev[base + t] = estub[2 * t + 1];
    }
    free(istub); free(estub); free(cstart); free(pstart); free(deg); free(kint); free(size);
    int rc = build_csr(n, m, eu, ev, off, idx, nnz);
    free(eu); free(ev);
    if (rc != GG_OK) { free(memb); return rc; }
    *membership_out = memb;
    *ncomm_out = nc;
    return GG_OK;
}
