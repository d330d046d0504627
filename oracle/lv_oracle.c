/*
 * CPU oracle for the Louvain local-moving method and its label-propagation
 * mode.  TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
 * CPU-baseline leg are its only users.  It shares no code with the GPU library
 * and is written for clarity, not speed: int64 arithmetic throughout, a dense
 * per-thread accumulator per vertex, qsort for coarsening.  OpenMP only splits
 * the vertex loop of a sweep; every vertex's decision reads the previous
 * sweep's state alone, so results do not depend on the thread count.
 *
 * Notation (paper, Section II): A is the symmetric weight matrix, with a loop
 * of weight w stored as A_vv = 2w because the weighted degree counts loops
 * twice; k_i = deg_w(i) = sum_j A_ij; M = vol_w(V) = sum_i k_i;
 * Sigma_tot(C) = vol_w(C); W_i(C) = cut_w(i, C \ {i}).
 *
 * Deterministic semantics (readings of the paper, fixed here):
 *   - sweeps are synchronous: every vertex decides against the previous
 *     sweep's labels and community volumes;
 *   - each vertex takes the argmax over all neighbouring communities (Alg. 2
 *     takes it over every neighbour), ties to the smallest id;
 *   - it moves only if that best score is strictly above staying (Alg. 2's
 *     Delta Q > 0 test) and the target lies in the sweep's allowed direction:
 *     odd sweeps allow only moves to a smaller community id, even sweeps only
 *     to a larger one;
 *   - communities are renumbered by their smallest member vertex id.
 */
#include <limits.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_OK 0
#define ORC_E_ARG 1
#define ORC_E_NOMEM 2
#define ORC_E_OVERFLOW 3

#define ORC_LOUVAIN 0
#define ORC_LPA 1
#define ORC_DOWN 0
#define ORC_UP 1

int orc_num_threads(void) { return omp_get_max_threads(); }
void orc_set_threads(int t) { if (t > 0) omp_set_num_threads(t); }

/*
 * Weighted adjacency from a caller CSR (Section II-A, weighted degree): the
 * diagonal entry of a loop is doubled.  Rejects weights < 1 and any total
 * volume M >= 2^31 (the integer score is exact in int64 below that bound).
 */
int orc_adjacency(int32_t n, const int32_t* off, const int32_t* idx, const int32_t* w, int32_t* a)
{
    int64_t total = 0;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t e = off[i]; e < off[i + 1]; ++e) {
            int64_t x = w ? (int64_t)w[e] : 1;
            if (x < 1) return ORC_E_ARG;
            if (idx[e] == i) x *= 2;
            if (x > INT32_MAX) return ORC_E_OVERFLOW;
            a[e] = (int32_t)x;
            total += x;
            if (total > INT32_MAX) return ORC_E_OVERFLOW;
        }
    return ORC_OK;
}

/* k_i = sum_j A_ij (deg_w, Section II-A); returns M = vol_w(V). */
int64_t orc_degrees(int32_t n, const int32_t* off, const int32_t* a, int64_t* k)
{
    int64_t M = 0;
    for (int32_t i = 0; i < n; ++i) {
        int64_t s = 0;
        for (int32_t e = off[i]; e < off[i + 1]; ++e) s += a[e];
        k[i] = s;
        M += s;
    }
    return M;
}

/*
 * Modularity (Section II-C) in integer form:
 *   Q = sum_C [ Sigma_in(C)/M - (Sigma_tot(C)/M)^2 ] = Q_int / M^2,
 *   Q_int = M * sum_C Sigma_in(C) - sum_C Sigma_tot(C)^2,
 * where Sigma_in(C) = sum_{i,j in C} A_ij.  Labels must lie in [0, n).
 */
int orc_modularity(int32_t n, const int32_t* off, const int32_t* idx, const int32_t* a,
                   const int32_t* labels, int64_t* q_int, int64_t* m_out)
{
    int64_t* tot = (int64_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    if (!tot) return ORC_E_NOMEM;
    int64_t in = 0, M = 0;
    for (int32_t i = 0; i < n; ++i) {
        if (labels[i] < 0 || labels[i] >= n) { free(tot); return ORC_E_ARG; }
        for (int32_t e = off[i]; e < off[i + 1]; ++e) {
            M += a[e];
            tot[labels[i]] += a[e];
            if (labels[idx[e]] == labels[i]) in += a[e];
        }
    }
    int64_t sq = 0;
    for (int32_t c = 0; c < n; ++c) sq += tot[c] * tot[c];
    free(tot);
    *q_int = M * in - sq;
    *m_out = M;
    return ORC_OK;
}

/*
 * Decision of one vertex in one synchronous sweep.
 *
 * Louvain (Alg. 2, gain of Eq. 1): for a neighbouring community C != A = c(i),
 *   score(C) = M * W_i(C) - k_i * Sigma_tot(C),
 *   stay     = M * W_i(A) - k_i * (Sigma_tot(A) - k_i),
 * and Delta Q_{i->C} = 2 (score(C) - stay) / M^2 (Eq. 1 with its vol_w(A^-),
 * vol_w(B^-) and cut_w terms written out).  LPA (Alg. 1, PLPMove): score(C) =
 * W_i(C), stay = W_i(A).  Only communities of neighbours j != i are candidates;
 * the best one (ties to the smallest id) is taken over all of them, and the
 * vertex moves there only when its score is strictly above stay and the
 * target id is below A in a DOWN sweep or above A in an UP sweep.
 *
 * acc/mark/list are caller scratch of length n (mark values are unique per
 * call through `stamp`).
 */
static int32_t decide(int32_t i, const int32_t* off, const int32_t* idx, const int32_t* a,
                      const int64_t* k, int64_t M, const int32_t* c, const int64_t* sigma, int dir,
                      int mode, int64_t* acc, int64_t* mark, int32_t* list, int64_t stamp)
{
    const int32_t A = c[i];
    int32_t nl = 0;
    for (int32_t e = off[i]; e < off[i + 1]; ++e) {
        int32_t j = idx[e];
        if (j == i) continue;
        int32_t C = c[j];
        if (mark[C] != stamp) { mark[C] = stamp; acc[C] = 0; list[nl++] = C; }
        acc[C] += a[e];
    }
    int64_t wA = (mark[A] == stamp) ? acc[A] : 0;
    int have = 0;
    int32_t best = A;
    int64_t best_score = 0;
    for (int32_t t = 0; t < nl; ++t) {
        int32_t C = list[t];
        if (C == A) continue;
        int64_t s = (mode == ORC_LOUVAIN) ? M * acc[C] - k[i] * sigma[C] : acc[C];
        if (!have || s > best_score || (s == best_score && C < best)) {
            have = 1; best = C; best_score = s;
        }
    }
    int64_t stay = (mode == ORC_LOUVAIN) ? M * wA - k[i] * (sigma[A] - k[i]) : wA;
    if (!have || best_score <= stay) return A;
    if (dir == ORC_DOWN && best > A) return A;
    if (dir == ORC_UP && best < A) return A;
    return best;
}

/* Decisions of the listed vertices against state (c, sigma); used for sampled checks. */
int orc_decide_vertices(int32_t n, const int32_t* off, const int32_t* idx, const int32_t* a,
                        const int64_t* k, int64_t M, const int32_t* c, const int64_t* sigma, int dir,
                        int mode, const int32_t* verts, int32_t nv, int32_t* out)
{
    int rc = ORC_OK;
#pragma omp parallel
    {
        int64_t* acc = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
        int64_t* mark = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
        int32_t* list = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
        if (!acc || !mark || !list) {
#pragma omp atomic write
            rc = ORC_E_NOMEM;
        } else {
            for (int32_t t = 0; t < n; ++t) mark[t] = -1;
#pragma omp for schedule(dynamic, 64)
            for (int32_t t = 0; t < nv; ++t)
                out[t] = decide(verts[t], off, idx, a, k, M, c, sigma, dir, mode, acc, mark, list, t);
        }
        free(acc); free(mark); free(list);
    }
    return rc;
}

/*
 * One synchronous sweep; returns the number of movers (or -1).  With an
 * `active` mask (NULL = every vertex) a vertex whose mask byte is 0 is not
 * evaluated and keeps its community.
 */
int64_t orc_sweep(int32_t n, const int32_t* off, const int32_t* idx, const int32_t* a,
                  const int64_t* k, int64_t M, const int32_t* c, const int64_t* sigma, int dir, int mode,
                  const uint8_t* active, int32_t* c_next)
{
    int64_t moves = 0;
    int failed = 0;
#pragma omp parallel reduction(+ : moves)
    {
        int64_t* acc = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
        int64_t* mark = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
        int32_t* list = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
        if (!acc || !mark || !list) {
#pragma omp atomic write
            failed = 1;
        } else {
            for (int32_t t = 0; t < n; ++t) mark[t] = -1;
#pragma omp for schedule(dynamic, 1024)
            for (int32_t i = 0; i < n; ++i) {
                c_next[i] = (active && !active[i]) ? c[i]
                                                   : decide(i, off, idx, a, k, M, c, sigma, dir, mode, acc, mark, list, i);
                if (c_next[i] != c[i]) ++moves;
            }
        }
        free(acc); free(mark); free(list);
    }
    return failed ? -1 : moves;
}

/*
 * One level of local moving (Alg. 2; Alg. 1 in LPA mode) from singletons:
 * c = identity, Sigma_tot = k.  Sweep s (1-based) moves DOWN when s is odd and
 * UP when s is even.  After sweep s, Sigma_tot is recomputed from the new labels.
 * The level stops after sweep s when s >= 2 and the last two sweeps each
 * moved at most `theta` vertices (theta = 0 for Louvain), or when s reaches
 * max_sweeps.  Writes the final labels to c and the per-sweep mover counts
 * to moves[0..sweeps-1]; returns the sweep count (or a negative error).
 *
 * prune != 0 restricts evaluation to active vertices (Alg. 1's V_active and
 * Alg. 2's needCheck: a vertex is reconsidered only after its own community
 * or a neighbour's changed).  Under synchronous sweeps whose direction
 * alternates, a vertex is evaluated in sweep s when s <= 2, or when it or one
 * of its neighbours changed community in sweep s-1 or in sweep s-2; the second
 * sweep back covers a move the previous sweep's direction did not allow.
 * Vertices that are not evaluated keep their community.
 */
int32_t orc_local_move(int32_t n, const int32_t* off, const int32_t* idx, const int32_t* a, int mode,
                       int32_t max_sweeps, int64_t theta, int prune, int32_t* c, int64_t* moves)
{
    if (max_sweeps < 1) return -ORC_E_ARG;
    const size_t nn = (size_t)(n > 0 ? n : 1);
    int64_t* k = (int64_t*)malloc(nn * sizeof(int64_t));
    int64_t* sigma = (int64_t*)malloc(nn * sizeof(int64_t));
    int32_t* nxt = (int32_t*)malloc(nn * sizeof(int32_t));
    uint8_t* chg1 = (uint8_t*)calloc(nn, 1);  /* changed in the previous sweep */
    uint8_t* chg2 = (uint8_t*)calloc(nn, 1);  /* changed in the sweep before it */
    uint8_t* act = (uint8_t*)malloc(nn);
    if (!k || !sigma || !nxt || !chg1 || !chg2 || !act) {
        free(k); free(sigma); free(nxt); free(chg1); free(chg2); free(act);
        return -ORC_E_NOMEM;
    }
    int64_t M = orc_degrees(n, off, a, k);
    for (int32_t i = 0; i < n; ++i) { c[i] = i; sigma[i] = k[i]; }
    int32_t s;
    int rc = 0;
    for (s = 1; s <= max_sweeps; ++s) {
        int dir = (s % 2 == 1) ? ORC_DOWN : ORC_UP;
        const uint8_t* mask = NULL;
        if (prune && s > 2) {
            for (int32_t i = 0; i < n; ++i) act[i] = chg1[i] | chg2[i];
            mask = act;
        }
        int64_t mv = orc_sweep(n, off, idx, a, k, M, c, sigma, dir, mode, mask, nxt);
        if (mv < 0) { rc = -ORC_E_NOMEM; break; }
        moves[s - 1] = mv;
        if (prune) {
            /* chg2 <- chg1, then chg1 <- {movers and every neighbour of a mover} */
            uint8_t* t = chg2; chg2 = chg1; chg1 = t;
            memset(chg1, 0, nn);
            for (int32_t i = 0; i < n; ++i)
                if (nxt[i] != c[i]) {
                    chg1[i] = 1;
                    for (int32_t e = off[i]; e < off[i + 1]; ++e) chg1[idx[e]] = 1;
                }
        }
        memcpy(c, nxt, (size_t)n * sizeof(int32_t));
        for (int32_t i = 0; i < n; ++i) sigma[i] = 0;
        for (int32_t i = 0; i < n; ++i) sigma[c[i]] += k[i];
        if (s >= 2 && moves[s - 1] <= theta && moves[s - 2] <= theta) break;
    }
    free(k); free(sigma); free(nxt); free(chg1); free(chg2); free(act);
    if (rc) return rc;
    return s > max_sweeps ? max_sweeps : s;
}

/*
 * Contiguous renumbering (aggregation phase, Section III-B: community ids are
 * remapped to 0..k-1), ordered by each community's smallest member vertex:
 * scanning vertices in increasing id, a community gets the next new id when
 * first seen.  Returns the number of communities.
 */
int32_t orc_renumber(int32_t n, const int32_t* c, int32_t* labels)
{
    int32_t* map = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!map) return -ORC_E_NOMEM;
    for (int32_t t = 0; t < n; ++t) map[t] = -1;
    int32_t next = 0;
    for (int32_t i = 0; i < n; ++i) {
        if (c[i] < 0 || c[i] >= n) { free(map); return -ORC_E_ARG; }
        if (map[c[i]] < 0) map[c[i]] = next++;
        labels[i] = map[c[i]];
    }
    free(map);
    return next;
}

typedef struct { int32_t r, c, w; } orc_trip;
static int cmp_trip(const void* x, const void* y)
{
    const orc_trip* p = (const orc_trip*)x;
    const orc_trip* q = (const orc_trip*)y;
    if (p->r != q->r) return (p->r > q->r) - (p->r < q->r);
    return (p->c > q->c) - (p->c < q->c);
}

/*
 * Aggregation (Alg. 3, Aggregation; Section III-B): every entry (i, j, A_ij)
 * becomes (labels[i], labels[j], A_ij); equal endpoint pairs are merged with
 * their weights summed, giving A' = S^T A S as a CSR with sorted columns.
 * Diagonal entries of A' collect the community's internal weight, already in
 * the doubled-loop convention.  Output buffers must hold n2+1 offsets and up
 * to nnz entries; returns the number of coarse entries.
 */
int64_t orc_aggregate(int32_t n, const int32_t* off, const int32_t* idx, const int32_t* a,
                      const int32_t* labels, int32_t n2, int32_t* off2, int32_t* idx2, int32_t* a2)
{
    int64_t nnz = off[n];
    orc_trip* t = (orc_trip*)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(orc_trip));
    if (!t) return -ORC_E_NOMEM;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t e = off[i]; e < off[i + 1]; ++e) {
            t[e].r = labels[i];
            t[e].c = labels[idx[e]];
            t[e].w = a[e];
        }
    qsort(t, (size_t)nnz, sizeof(orc_trip), cmp_trip);
    int64_t out = 0;
    for (int32_t r = 0; r <= n2; ++r) off2[r] = 0;
    for (int64_t e = 0; e < nnz; ++e) {
        if (e > 0 && t[e].r == t[e - 1].r && t[e].c == t[e - 1].c) {
            int64_t s = (int64_t)a2[out - 1] + t[e].w;
            if (s > INT32_MAX) { free(t); return -ORC_E_OVERFLOW; }
            a2[out - 1] = (int32_t)s;
        } else {
            idx2[out] = t[e].c;
            a2[out] = t[e].w;
            off2[t[e].r + 1]++;
            ++out;
        }
    }
    for (int32_t r = 0; r < n2; ++r) off2[r + 1] += off2[r];
    free(t);
    return out;
}

/* Q_int of the singleton partition: M * trace(A) - sum_i k_i^2 (Section II-C). */
int64_t orc_singleton_qint(int32_t n, const int32_t* off, const int32_t* idx, const int32_t* a)
{
    int64_t M = 0, tr = 0, sq = 0;
    for (int32_t i = 0; i < n; ++i) {
        int64_t k = 0;
        for (int32_t e = off[i]; e < off[i + 1]; ++e) {
            k += a[e];
            if (idx[e] == i) tr += a[e];
        }
        M += k;
        sq += k * k;
    }
    return M * tr - sq;
}
