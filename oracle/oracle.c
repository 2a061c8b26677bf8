/*
 * ORACLE: plain, slow, sequential CPU implementation of the Voronoi-cell
 * 2-approximation Steiner tree (Mehlhorn's construction as parallelised in
 * Alg. 2 of Reza, Sanders, Pearce, "Towards Distributed 2-Approximation
 * Steiner Minimal Trees in Billion-edge Graphs", arXiv:2205.14503).
 *
 * THIS IS TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may call it.  It shares no code, header, table
 * or helper with the GPU library and must never be used as a fallback for it.
 *
 * All arithmetic is integer.  Distances are computed in uint64 without
 * saturation; the overflow rules below decide when the 32-bit result would not
 * be representable.
 *
 * Readings of the paper fixed here (the paper leaves ties open):
 *  - seeds are deduplicated and sorted; seed index i = rank of the seed;
 *  - a vertex belongs to the cell of the seed minimising (distance, index)
 *    lexicographically (Section II defines cells by strict distance and is
 *    silent on equidistant vertices);
 *  - pred(v) is the smallest neighbour u, then smallest CSR offset e in row v,
 *    with src(u) == src(v) and dist(u) + w(e) == dist(v) (Alg. 4 sets pred
 *    in arrival order, which is not deterministic);
 *  - among cross-cell edges of one cell pair with equal
 *    d1(s,u)+d(u,v)+d1(v,t), the one with the smallest edge id wins, where the
 *    edge id is the CSR offset of the half-edge leaving the smaller endpoint
 *    (Alg. 2 Step 2 and Alg. 5 say only that a tie-break is used);
 *  - the MST of G'1 is the unique MST under the strict order (d'1, i, j);
 *  - unreachable distances, overflow: EOVERFLOW if some finite distance is
 *    >= 2^32-1 or some cross-cell sum d1+d+d1 is >= 2^32;
 *    EDISCONNECTED if the seeds do not all lie in one component.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum {
    ORACLE_OK = 0,
    ORACLE_EINVAL = -1,
    ORACLE_ENOMEM = -2,
    ORACLE_EDISCONNECTED = -3,
    ORACLE_EOVERFLOW = -4
};

#define DIST_INF UINT64_MAX
#define IDX_NONE UINT32_MAX
#define DIST32_LIMIT 0xFFFFFFFFULL /* largest distance the 32-bit form cannot hold */

/* ---------------------------------------------------------------- input -- */

/* Graph accepted by the method: n >= 1, monotone row offsets ending at nnz,
 * nnz < 2^32 (edge ids are 32-bit), columns < n, weights >= 1 (Table II: the
 * distance function maps to positive integers), rows sorted by column. */
int oracle_check_graph(uint32_t n, uint64_t nnz, const uint64_t *row_ptr, const uint32_t *col,
                       const uint32_t *w) {
    if (n == 0 || nnz >= (1ULL << 32)) return ORACLE_EINVAL;
    if (row_ptr[0] != 0 || row_ptr[n] != nnz) return ORACLE_EINVAL;
    for (uint32_t v = 0; v < n; v++) {
        if (row_ptr[v + 1] < row_ptr[v]) return ORACLE_EINVAL;
        for (uint64_t e = row_ptr[v]; e < row_ptr[v + 1]; e++) {
            if (col[e] >= n || w[e] == 0) return ORACLE_EINVAL;
            if (e > row_ptr[v] && col[e] < col[e - 1]) return ORACLE_EINVAL;
        }
    }
    return ORACLE_OK;
}

static int cmp_u32(const void *a, const void *b) {
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return (x > y) - (x < y);
}

/* S = sorted set of the given seeds.  k == 0 or a seed >= n is EINVAL. */
int oracle_canon_seeds(uint32_t n, const uint32_t *seeds, uint32_t k, uint32_t *S, uint32_t *k_out) {
    if (k == 0) return ORACLE_EINVAL;
    for (uint32_t i = 0; i < k; i++)
        if (seeds[i] >= n) return ORACLE_EINVAL;
    memcpy(S, seeds, (size_t)k * sizeof(uint32_t));
    qsort(S, k, sizeof(uint32_t), cmp_u32);
    uint32_t m = 0;
    for (uint32_t i = 0; i < k; i++)
        if (m == 0 || S[m - 1] != S[i]) S[m++] = S[i];
    *k_out = m;
    return ORACLE_OK;
}

/* ------------------------------------------------- Step 1: Voronoi cells -- */

/* Binary min-heap of (dist, seed index, vertex), ordered lexicographically. */
typedef struct {
    uint64_t d;
    uint32_t i, v;
} hitem;

static int hless(hitem a, hitem b) { return a.d < b.d || (a.d == b.d && a.i < b.i); }

typedef struct {
    hitem *a;
    uint64_t len, cap;
} heap;

static int hpush(heap *h, hitem x) {
    if (h->len == h->cap) {
        uint64_t nc = h->cap ? 2 * h->cap : 1024;
        hitem *na = (hitem *)realloc(h->a, nc * sizeof(hitem));
        if (!na) return -1;
        h->a = na;
        h->cap = nc;
    }
    uint64_t c = h->len++;
    h->a[c] = x;
    while (c > 0) {
        uint64_t p = (c - 1) / 2;
        if (!hless(h->a[c], h->a[p])) break;
        hitem t = h->a[c]; h->a[c] = h->a[p]; h->a[p] = t;
        c = p;
    }
    return 0;
}

static hitem hpop(heap *h) {
    hitem top = h->a[0];
    h->a[0] = h->a[--h->len];
    uint64_t c = 0;
    for (;;) {
        uint64_t l = 2 * c + 1, r = l + 1, m = c;
        if (l < h->len && hless(h->a[l], h->a[m])) m = l;
        if (r < h->len && hless(h->a[r], h->a[m])) m = r;
        if (m == c) break;
        hitem t = h->a[c]; h->a[c] = h->a[m]; h->a[m] = t;
        c = m;
    }
    return top;
}

/* Alg. 2 Step 1 / Alg. 4: every vertex gets src (seed index) and the distance
 * d1(src, v).  Computed as multi-source Dijkstra over the (dist, index) order,
 * so (dist[v], src[v]) = min over seeds i of (d(s_i, v), i).  Vertices no seed
 * reaches keep DIST_INF / IDX_NONE (Alg. 3 initialisation). */
int oracle_voronoi(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, const uint32_t *w,
                   uint32_t k, const uint32_t *S, uint64_t *dist, uint32_t *src) {
    heap h = {0, 0, 0};
    for (uint32_t v = 0; v < n; v++) {
        dist[v] = DIST_INF;
        src[v] = IDX_NONE;
    }
    for (uint32_t i = 0; i < k; i++) {
        dist[S[i]] = 0;
        src[S[i]] = i;
        if (hpush(&h, (hitem){0, i, S[i]})) { free(h.a); return ORACLE_ENOMEM; }
    }
    while (h.len) {
        hitem x = hpop(&h);
        if (x.d != dist[x.v] || x.i != src[x.v]) continue; /* stale entry */
        for (uint64_t e = row_ptr[x.v]; e < row_ptr[x.v + 1]; e++) {
            uint32_t u = col[e];
            hitem cand = {x.d + w[e], x.i, u};
            hitem cur = {dist[u], src[u], u};
            if (hless(cand, cur)) {
                dist[u] = cand.d;
                src[u] = cand.i;
                if (hpush(&h, cand)) { free(h.a); return ORACLE_ENOMEM; }
            }
        }
    }
    free(h.a);
    return ORACLE_OK;
}

/* pred(v) for every vertex (the predecessor Alg. 4 records while relaxing, made canonical):
 * seeds point to themselves, unreached vertices to IDX_NONE, any other v to
 * the first entry of row v (smallest neighbour, then smallest offset) that is
 * in the same cell and lies on a shortest path: dist[u] + w == dist[v]. */
void oracle_pred(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, const uint32_t *w,
                 uint32_t k, const uint32_t *S, const uint64_t *dist, const uint32_t *src,
                 uint32_t *pred) {
    for (uint32_t v = 0; v < n; v++) pred[v] = IDX_NONE;
    for (uint32_t v = 0; v < n; v++) {
        if (dist[v] == DIST_INF || dist[v] == 0) continue;
        for (uint64_t e = row_ptr[v]; e < row_ptr[v + 1]; e++) {
            uint32_t u = col[e];
            if (dist[u] != DIST_INF && src[u] == src[v] && dist[u] + w[e] == dist[v]) {
                pred[v] = u;
                break;
            }
        }
    }
    for (uint32_t i = 0; i < k; i++) pred[S[i]] = S[i];
}

/* EOVERFLOW if some reached vertex is at distance >= 2^32-1 (the 32-bit form
 * reserves 2^32-1 for "unreached"). */
int oracle_check_dist(uint32_t n, const uint64_t *dist) {
    for (uint32_t v = 0; v < n; v++)
        if (dist[v] != DIST_INF && dist[v] >= DIST32_LIMIT) return ORACLE_EOVERFLOW;
    return ORACLE_OK;
}

/* --------------------------------------------- Step 2: distance graph G'1 -- */

typedef struct {
    uint32_t i, j; /* seed indices, i < j */
    uint64_t bsum; /* d1(s_i,a) + d(a,b) + d1(b,s_j) */
    uint32_t e;    /* CSR offset of the half-edge a -> b, a < b */
} cross;

static int cmp_cross_pair(const void *x, const void *y) {
    const cross *a = (const cross *)x, *b = (const cross *)y;
    if (a->i != b->i) return a->i < b->i ? -1 : 1;
    if (a->j != b->j) return a->j < b->j ? -1 : 1;
    if (a->bsum != b->bsum) return a->bsum < b->bsum ? -1 : 1;
    if (a->e != b->e) return a->e < b->e ? -1 : 1;
    return 0;
}

/* Alg. 2 Step 2 / Alg. 5: for every pair of cells joined by at least one
 * cross-cell edge (a,b), d'1(s_i,s_j) = min over those edges of
 * dist[a] + w + dist[b], and E_N keeps the minimising edge.  Every undirected
 * edge is looked at once, from its smaller endpoint a.  Output sorted by
 * (i, j); `cap` must be at least the number of pairs.  EOVERFLOW if some
 * cross-cell sum does not fit in 32 bits. */
int oracle_boundary(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, const uint32_t *w,
                    const uint64_t *dist, const uint32_t *src, uint64_t cap, uint32_t *pi,
                    uint32_t *pj, uint64_t *pbsum, uint32_t *pe, uint64_t *count) {
    uint64_t ncand = 0;
    for (uint32_t a = 0; a < n; a++)
        for (uint64_t e = row_ptr[a]; e < row_ptr[a + 1]; e++) {
            uint32_t b = col[e];
            if (a < b && dist[a] != DIST_INF && dist[b] != DIST_INF && src[a] != src[b]) ncand++;
        }
    cross *c = (cross *)malloc((ncand ? ncand : 1) * sizeof(cross));
    if (!c) return ORACLE_ENOMEM;
    uint64_t t = 0;
    int overflow = 0;
    for (uint32_t a = 0; a < n; a++)
        for (uint64_t e = row_ptr[a]; e < row_ptr[a + 1]; e++) {
            uint32_t b = col[e];
            if (!(a < b && dist[a] != DIST_INF && dist[b] != DIST_INF && src[a] != src[b])) continue;
            cross x;
            x.i = src[a] < src[b] ? src[a] : src[b];
            x.j = src[a] < src[b] ? src[b] : src[a];
            x.bsum = dist[a] + (uint64_t)w[e] + dist[b];
            x.e = (uint32_t)e;
            if (x.bsum >= (1ULL << 32)) overflow = 1;
            c[t++] = x;
        }
    if (overflow) { free(c); return ORACLE_EOVERFLOW; }
    qsort(c, ncand, sizeof(cross), cmp_cross_pair);
    uint64_t m = 0;
    for (uint64_t q = 0; q < ncand; q++) {
        if (q > 0 && c[q].i == c[q - 1].i && c[q].j == c[q - 1].j) continue; /* not the pair's minimum */
        if (m >= cap) { free(c); return ORACLE_ENOMEM; }
        pi[m] = c[q].i;
        pj[m] = c[q].j;
        pbsum[m] = c[q].bsum;
        pe[m] = c[q].e;
        m++;
    }
    free(c);
    *count = m;
    return ORACLE_OK;
}

/* --------------------------------------------------- Step 3: MST of G'1 -- */

typedef struct {
    uint64_t bsum;
    uint32_t i, j, pos;
} gedge;

static int cmp_gedge(const void *x, const void *y) {
    const gedge *a = (const gedge *)x, *b = (const gedge *)y;
    if (a->bsum != b->bsum) return a->bsum < b->bsum ? -1 : 1;
    if (a->i != b->i) return a->i < b->i ? -1 : 1;
    if (a->j != b->j) return a->j < b->j ? -1 : 1;
    return 0;
}

static uint32_t dsu_find(uint32_t *p, uint32_t x) {
    while (p[x] != x) {
        p[x] = p[p[x]];
        x = p[x];
    }
    return x;
}

/* Kruskal over G'1 in the strict order (d'1, i, j); the chosen list positions
 * are written to `chosen` in the order Kruskal accepts them.  EDISCONNECTED if
 * fewer than k-1 edges join the k seeds into one tree. */
int oracle_mst(uint32_t k, uint64_t count, const uint32_t *pi, const uint32_t *pj,
               const uint64_t *pbsum, uint32_t *chosen, uint32_t *nchosen) {
    gedge *g = (gedge *)malloc((count ? count : 1) * sizeof(gedge));
    uint32_t *par = (uint32_t *)malloc((size_t)(k ? k : 1) * sizeof(uint32_t));
    if (!g || !par) { free(g); free(par); return ORACLE_ENOMEM; }
    for (uint64_t q = 0; q < count; q++) g[q] = (gedge){pbsum[q], pi[q], pj[q], (uint32_t)q};
    qsort(g, count, sizeof(gedge), cmp_gedge);
    for (uint32_t i = 0; i < k; i++) par[i] = i;
    uint32_t m = 0;
    for (uint64_t q = 0; q < count && m + 1 < k; q++) {
        uint32_t a = dsu_find(par, g[q].i), b = dsu_find(par, g[q].j);
        if (a == b) continue;
        par[a] = b;
        chosen[m++] = g[q].pos;
    }
    free(g);
    free(par);
    *nchosen = m;
    return m + 1 == k ? ORACLE_OK : ORACLE_EDISCONNECTED;
}

/* --------------------------------- Steps 4-7: prune, expand, total weight -- */

typedef struct {
    uint32_t a, b, w;
} tedge;

static int cmp_tedge(const void *x, const void *y) {
    const tedge *p = (const tedge *)x, *q = (const tedge *)y;
    if (p->a != q->a) return p->a < q->a ? -1 : 1;
    if (p->b != q->b) return p->b < q->b ? -1 : 1;
    if (p->w != q->w) return p->w < q->w ? -1 : 1;
    return 0;
}

/* Row that holds CSR offset e. */
static uint32_t row_of(uint32_t n, const uint64_t *row_ptr, uint64_t e) {
    uint32_t lo = 0, hi = n; /* row_ptr[lo] <= e < row_ptr[hi] */
    while (hi - lo > 1) {
        uint32_t mid = lo + (hi - lo) / 2;
        if (row_ptr[mid] <= e) lo = mid; else hi = mid;
    }
    return lo;
}

/* Alg. 2 Steps 4-7 (Alg. 5 pruning, Alg. 6 tree edges): the tree's edges are
 * the kept cross-cell edge of every MST pair plus, from both of its endpoints,
 * every edge (pred(x), x) up to the cell's seed.  E_S is a set, so duplicates
 * are dropped; the result is sorted by (a, b, w) with a < b, and D is the sum
 * of the weights.  `out_cap` must hold at least 2*(k-1) + sum of path lengths;
 * n is a safe bound. */
int oracle_expand(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, const uint32_t *w,
                  uint32_t k, const uint32_t *S, const uint64_t *dist, const uint32_t *src,
                  const uint32_t *pred, uint32_t nsel, const uint32_t *sel_e, uint64_t out_cap,
                  uint32_t *oa, uint32_t *ob, uint32_t *ow, uint64_t *out_count, uint64_t *total) {
    uint64_t cap = 16, len = 0;
    tedge *t = (tedge *)malloc(cap * sizeof(tedge));
    if (!t) return ORACLE_ENOMEM;
#define ADD_EDGE(x, y, wt)                                                            \
    do {                                                                              \
        if (len == cap) {                                                             \
            cap *= 2;                                                                 \
            tedge *nt = (tedge *)realloc(t, cap * sizeof(tedge));                     \
            if (!nt) { free(t); return ORACLE_ENOMEM; }                               \
            t = nt;                                                                   \
        }                                                                             \
        t[len].a = (x) < (y) ? (x) : (y);                                             \
        t[len].b = (x) < (y) ? (y) : (x);                                             \
        t[len].w = (wt);                                                              \
        len++;                                                                        \
    } while (0)
    for (uint32_t q = 0; q < nsel; q++) {
        uint64_t e = sel_e[q];
        uint32_t a = row_of(n, row_ptr, e), b = col[e];
        ADD_EDGE(a, b, w[e]);
        uint32_t ends[2] = {a, b};
        for (int s = 0; s < 2; s++) {
            uint32_t x = ends[s];
            while (S[src[x]] != x) { /* x is not its cell's seed */
                uint32_t p = pred[x];
                ADD_EDGE(x, p, (uint32_t)(dist[x] - dist[p]));
                x = p;
            }
        }
    }
#undef ADD_EDGE
    qsort(t, len, sizeof(tedge), cmp_tedge);
    uint64_t m = 0, D = 0;
    for (uint64_t q = 0; q < len; q++) {
        if (m > 0 && t[q].a == t[m - 1].a && t[q].b == t[m - 1].b && t[q].w == t[m - 1].w) continue;
        t[m++] = t[q];
    }
    if (m > out_cap) { free(t); return ORACLE_ENOMEM; }
    for (uint64_t q = 0; q < m; q++) {
        oa[q] = t[q].a;
        ob[q] = t[q].b;
        ow[q] = t[q].w;
        D += t[q].w;
    }
    free(t);
    *out_count = m;
    *total = D;
    (void)k;
    return ORACLE_OK;
}

/* ------------------------------------------------------- whole method -- */

/* Alg. 2 end to end.  Outputs (caller-allocated): dist u64[n], src u32[n],
 * pred u32[n], edge arrays of capacity n, edge count and D.  k == 1 (after
 * deduplication) gives an empty tree with D = 0 without further checks. */
int oracle_solve(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, const uint32_t *w,
                 const uint32_t *seeds, uint32_t k_in, uint64_t *dist, uint32_t *src, uint32_t *pred,
                 uint32_t *oa, uint32_t *ob, uint32_t *ow, uint64_t *out_count, uint64_t *total) {
    *out_count = 0;
    *total = 0;
    int rc = oracle_check_graph(n, row_ptr[n], row_ptr, col, w);
    if (rc) return rc;
    uint32_t *S = (uint32_t *)malloc((size_t)(k_in ? k_in : 1) * sizeof(uint32_t));
    uint32_t k = 0;
    if (!S) return ORACLE_ENOMEM;
    rc = oracle_canon_seeds(n, seeds, k_in, S, &k);
    if (rc) { free(S); return rc; }
    if (k == 1) { free(S); return ORACLE_OK; }
    rc = oracle_voronoi(n, row_ptr, col, w, k, S, dist, src);
    if (!rc) rc = oracle_check_dist(n, dist);
    if (rc) { free(S); return rc; }
    oracle_pred(n, row_ptr, col, w, k, S, dist, src, pred);
    uint64_t cap = (uint64_t)k * (k - 1) / 2, half = row_ptr[n] / 2 + 1;
    if (half < cap) cap = half;
    uint32_t *pi = (uint32_t *)malloc(cap * sizeof(uint32_t)), *pj = (uint32_t *)malloc(cap * sizeof(uint32_t));
    uint32_t *pe = (uint32_t *)malloc(cap * sizeof(uint32_t)), *ch = (uint32_t *)malloc((size_t)k * sizeof(uint32_t));
    uint32_t *sel = (uint32_t *)malloc((size_t)k * sizeof(uint32_t));
    uint64_t *pb = (uint64_t *)malloc(cap * sizeof(uint64_t));
    uint64_t cnt = 0;
    uint32_t nch = 0;
    if (!pi || !pj || !pe || !ch || !sel || !pb) rc = ORACLE_ENOMEM;
    if (!rc) rc = oracle_boundary(n, row_ptr, col, w, dist, src, cap, pi, pj, pb, pe, &cnt);
    if (!rc) rc = oracle_mst(k, cnt, pi, pj, pb, ch, &nch);
    if (!rc) {
        for (uint32_t q = 0; q < nch; q++) sel[q] = pe[ch[q]];
        rc = oracle_expand(n, row_ptr, col, w, k, S, dist, src, pred, nch, sel, n, oa, ob, ow, out_count, total);
    }
    free(pi); free(pj); free(pe); free(ch); free(sel); free(pb); free(S);
    return rc;
}
