/*
 * Seeded synthetic workload generators: Erdos-Renyi G(n,m), 4-neighbour 2D
 * grids, R-MAT, largest-connected-component extraction and seed sampling.
 *
 * This module holds only input generation.  It computes nothing of the
 * Steiner-tree method itself and is shared by the GPU library's tests, the
 * benchmark and the CPU oracle's tests, so that every side sees the same
 * bytes.
 *
 * Randomness is counter based: the i-th draw of a stream is the i-th output
 * of a SplitMix64 generator (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) whose seed is the stream key.
 * A draw therefore depends only on (stream, index), never on thread count or
 * scheduling, and every generated graph is bit-identical on every machine.
 *
 * Output graphs are undirected and stored as a symmetric CSR: row_ptr u64[n+1],
 * col u32[nnz] sorted ascending within each row, w u32[nnz] with
 * w(a,b) == w(b,a) >= 1.  Self-loops are removed and parallel edges merged.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define GOLDEN_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t sm_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* i-th output (0-based) of SplitMix64 seeded with `key`. */
uint64_t wl_draw(uint64_t key, uint64_t i) { return sm_mix(key + (i + 1) * GOLDEN_GAMMA); }

/* Key of stream `stream_id` under master seed `master`. */
uint64_t wl_stream_key(uint64_t master, uint64_t stream_id) {
    return sm_mix(sm_mix(master + GOLDEN_GAMMA) ^ (stream_id * 0xD1B54A32D192ED03ULL));
}

/* Uniform integer in [0, range) from the top 32 bits of a draw (range < 2^32). */
static inline uint32_t below(uint64_t r, uint32_t range) {
    return (uint32_t)(((r >> 32) * (uint64_t)range) >> 32);
}

/* Weight of the undirected edge {a,b}: uniform in [lo,hi], keyed by the
 * unordered pair so that both CSR halves carry the same value. */
static inline uint32_t edge_weight(uint64_t wkey, uint32_t a, uint32_t b, uint32_t lo, uint32_t hi) {
    uint32_t x = a < b ? a : b, y = a < b ? b : a;
    return lo + below(wl_draw(wkey, ((uint64_t)x << 32) | y), hi - lo + 1);
}

typedef struct {
    uint32_t n;
    uint64_t nnz;
    uint64_t *row_ptr;
    uint32_t *col;
    uint32_t *w;
} wl_graph;

void wl_graph_free(wl_graph *g) {
    if (!g) return;
    free(g->row_ptr);
    free(g->col);
    free(g->w);
    free(g);
}

static int cmp_u32(const void *a, const void *b) {
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return (x > y) - (x < y);
}

static void sort_u32(uint32_t *p, uint64_t len) {
    if (len <= 24) {
        for (uint64_t i = 1; i < len; i++) {
            uint32_t x = p[i];
            uint64_t j = i;
            while (j > 0 && p[j - 1] > x) { p[j] = p[j - 1]; j--; }
            p[j] = x;
        }
    } else {
        qsort(p, len, sizeof(uint32_t), cmp_u32);
    }
}

/* Build a symmetric, deduplicated, self-loop-free CSR from m undirected pairs
 * (src[i], dst[i]).  Consumes nothing; the caller frees src/dst. */
static wl_graph *build_csr(uint32_t n, uint64_t m, const uint32_t *src, const uint32_t *dst,
                           uint64_t wkey, uint32_t wlo, uint32_t whi) {
    uint64_t *deg = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
    if (!deg) return NULL;
#pragma omp parallel for schedule(static)
    for (uint64_t i = 0; i < m; i++) {
        uint32_t a = src[i], b = dst[i];
        if (a == b) continue;
        __atomic_fetch_add(&deg[a], 1, __ATOMIC_RELAXED);
        __atomic_fetch_add(&deg[b], 1, __ATOMIC_RELAXED);
    }
    /* exclusive prefix sum -> start offsets of the raw (duplicated) rows */
    uint64_t *start = (uint64_t *)malloc(((size_t)n + 1) * sizeof(uint64_t));
    if (!start) { free(deg); return NULL; }
    uint64_t acc = 0;
    for (uint32_t v = 0; v < n; v++) { start[v] = acc; acc += deg[v]; }
    start[n] = acc;
    uint64_t raw = acc;
    uint32_t *buf = (uint32_t *)malloc((raw ? raw : 1) * sizeof(uint32_t));
    if (!buf) { free(deg); free(start); return NULL; }
    /* deg[] becomes the per-row fill cursor */
    memcpy(deg, start, (size_t)n * sizeof(uint64_t));
#pragma omp parallel for schedule(static)
    for (uint64_t i = 0; i < m; i++) {
        uint32_t a = src[i], b = dst[i];
        if (a == b) continue;
        buf[__atomic_fetch_add(&deg[a], 1, __ATOMIC_RELAXED)] = b;
        buf[__atomic_fetch_add(&deg[b], 1, __ATOMIC_RELAXED)] = a;
    }
    /* sort + unique each row in place; deg[v] becomes the unique count */
#pragma omp parallel for schedule(dynamic, 1024)
    for (uint32_t v = 0; v < n; v++) {
        uint32_t *p = buf + start[v];
        uint64_t len = start[v + 1] - start[v];
        sort_u32(p, len);
        uint64_t u = 0;
        for (uint64_t i = 0; i < len; i++)
            if (u == 0 || p[u - 1] != p[i]) p[u++] = p[i];
        deg[v] = u;
    }
    wl_graph *g = (wl_graph *)calloc(1, sizeof(wl_graph));
    if (!g) { free(buf); free(start); free(deg); return NULL; }
    g->n = n;
    g->row_ptr = (uint64_t *)malloc(((size_t)n + 1) * sizeof(uint64_t));
    if (!g->row_ptr) { free(g); free(buf); free(start); free(deg); return NULL; }
    acc = 0;
    for (uint32_t v = 0; v < n; v++) { g->row_ptr[v] = acc; acc += deg[v]; }
    g->row_ptr[n] = acc;
    g->nnz = acc;
    g->col = (uint32_t *)malloc((acc ? acc : 1) * sizeof(uint32_t));
    g->w = (uint32_t *)malloc((acc ? acc : 1) * sizeof(uint32_t));
    if (!g->col || !g->w) { wl_graph_free(g); free(buf); free(start); free(deg); return NULL; }
#pragma omp parallel for schedule(dynamic, 1024)
    for (uint32_t v = 0; v < n; v++) {
        uint64_t o = g->row_ptr[v], len = g->row_ptr[v + 1] - o;
        memcpy(g->col + o, buf + start[v], len * sizeof(uint32_t));
        for (uint64_t i = 0; i < len; i++) g->w[o + i] = edge_weight(wkey, v, g->col[o + i], wlo, whi);
    }
    free(buf);
    free(start);
    free(deg);
    return g;
}

/* Erdos-Renyi G(n, m): m distinct unordered pairs {u,v}, u != v, drawn
 * uniformly by rejection (sequential; intended for small graphs). */
wl_graph *wl_gen_er(uint32_t n, uint64_t m, uint32_t wlo, uint32_t whi, uint64_t master) {
    if (n < 2 || m > (uint64_t)n * (n - 1) / 2 || wlo < 1 || whi < wlo) return NULL;
    uint64_t gkey = wl_stream_key(master, 1), wkey = wl_stream_key(master, 2);
    uint64_t cap = 1;
    while (cap < 4 * m + 16) cap <<= 1;
    uint64_t *set = (uint64_t *)malloc(cap * sizeof(uint64_t));
    uint32_t *src = (uint32_t *)malloc((m ? m : 1) * sizeof(uint32_t));
    uint32_t *dst = (uint32_t *)malloc((m ? m : 1) * sizeof(uint32_t));
    memset(set, 0xff, cap * sizeof(uint64_t));
    uint64_t have = 0;
    for (uint64_t i = 0; have < m; i++) {
        uint64_t r = wl_draw(gkey, i);
        uint32_t u = (uint32_t)(((r & 0xffffffffULL) * n) >> 32), v = (uint32_t)(((r >> 32) * n) >> 32);
        if (u == v) continue;
        uint32_t x = u < v ? u : v, y = u < v ? v : u;
        uint64_t key = ((uint64_t)x << 32) | y, h = sm_mix(key) & (cap - 1);
        int dup = 0;
        while (set[h] != UINT64_MAX) {
            if (set[h] == key) { dup = 1; break; }
            h = (h + 1) & (cap - 1);
        }
        if (dup) continue;
        set[h] = key;
        src[have] = x;
        dst[have] = y;
        have++;
    }
    wl_graph *g = build_csr(n, m, src, dst, wkey, wlo, whi);
    free(set);
    free(src);
    free(dst);
    return g;
}

/* rows x cols 4-neighbour grid, vertex id = r*cols + c. */
wl_graph *wl_gen_grid(uint32_t rows, uint32_t cols, uint32_t wlo, uint32_t whi, uint64_t master) {
    if (rows == 0 || cols == 0 || (uint64_t)rows * cols >= 0xFFFFFFFFULL || wlo < 1 || whi < wlo) return NULL;
    uint64_t wkey = wl_stream_key(master, 2);
    uint32_t n = rows * cols;
    uint64_t m = (uint64_t)rows * (cols - 1) + (uint64_t)(rows - 1) * cols;
    uint32_t *src = (uint32_t *)malloc((m ? m : 1) * sizeof(uint32_t));
    uint32_t *dst = (uint32_t *)malloc((m ? m : 1) * sizeof(uint32_t));
    uint64_t e = 0;
    for (uint32_t r = 0; r < rows; r++)
        for (uint32_t c = 0; c < cols; c++) {
            uint32_t id = r * cols + c;
            if (c + 1 < cols) { src[e] = id; dst[e] = id + 1; e++; }
            if (r + 1 < rows) { src[e] = id; dst[e] = id + cols; e++; }
        }
    wl_graph *g = build_csr(n, m, src, dst, wkey, wlo, whi);
    free(src);
    free(dst);
    return g;
}

/* R-MAT (Chakrabarti, Zhan, Faloutsos 2004): edgefactor * 2^scale pairs; at
 * each of `scale` levels a quadrant is chosen with probabilities
 * (a, b, c, 1-a-b-c) from a 16-bit uniform, most significant bit first.
 * Vertex ids are then relabelled by a uniform random permutation (the
 * Graph500 convention); self-loops and duplicates are removed. */
wl_graph *wl_gen_rmat(uint32_t scale, uint32_t edgefactor, double a, double b, double c,
                      uint32_t wlo, uint32_t whi, int permute, uint64_t master) {
    if (scale < 1 || scale > 31 || edgefactor == 0 || wlo < 1 || whi < wlo) return NULL;
    if (a < 0 || b < 0 || c < 0 || a + b + c > 1.0) return NULL;
    uint64_t gkey = wl_stream_key(master, 1), wkey = wl_stream_key(master, 2), pkey = wl_stream_key(master, 3);
    uint32_t n = 1u << scale;
    uint64_t m = (uint64_t)edgefactor << scale;
    uint32_t ta = (uint32_t)(a * 65536.0 + 0.5), tb = ta + (uint32_t)(b * 65536.0 + 0.5),
             tc = tb + (uint32_t)(c * 65536.0 + 0.5);
    uint32_t words = (scale + 3) / 4; /* 4 levels of 16 bits per 64-bit draw */
    uint32_t *src = (uint32_t *)malloc(m * sizeof(uint32_t));
    uint32_t *dst = (uint32_t *)malloc(m * sizeof(uint32_t));
    uint32_t *perm = NULL;
    if (!src || !dst) { free(src); free(dst); return NULL; }
    if (permute) {
        perm = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
        for (uint32_t v = 0; v < n; v++) perm[v] = v;
        for (uint32_t i = n - 1; i > 0; i--) { /* Fisher-Yates */
            uint32_t j = below(wl_draw(pkey, i), i + 1);
            uint32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
        }
    }
#pragma omp parallel for schedule(static)
    for (uint64_t i = 0; i < m; i++) {
        uint32_t u = 0, v = 0, level = 0;
        for (uint32_t wd = 0; wd < words; wd++) {
            uint64_t r = wl_draw(gkey, i * words + wd);
            for (int q = 0; q < 4 && level < scale; q++, level++) {
                uint32_t x = (uint32_t)((r >> (16 * q)) & 0xffff);
                uint32_t bit = 1u << (scale - 1 - level);
                if (x < ta) {
                } else if (x < tb) {
                    v |= bit;
                } else if (x < tc) {
                    u |= bit;
                } else {
                    u |= bit;
                    v |= bit;
                }
            }
        }
        src[i] = perm ? perm[u] : u;
        dst[i] = perm ? perm[v] : v;
    }
    free(perm);
    wl_graph *g = build_csr(n, m, src, dst, wkey, wlo, whi);
    free(src);
    free(dst);
    return g;
}

/* Root of x with path halving; safe under concurrent hooking. */
static uint32_t uf_find(uint32_t *p, uint32_t x) {
    for (;;) {
        uint32_t y = __atomic_load_n(&p[x], __ATOMIC_RELAXED);
        if (y == x) return x;
        uint32_t z = __atomic_load_n(&p[y], __ATOMIC_RELAXED);
        if (z != y) __atomic_compare_exchange_n(&p[x], &y, z, 0, __ATOMIC_RELAXED, __ATOMIC_RELAXED);
        x = z;
    }
}

/* Connected-component label of every vertex: the smallest vertex id of its
 * component (lock-free union-find, larger root hooked under smaller). */
void wl_components(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, uint32_t *label) {
    for (uint32_t v = 0; v < n; v++) label[v] = v;
#pragma omp parallel for schedule(dynamic, 4096)
    for (uint32_t u = 0; u < n; u++) {
        for (uint64_t e = row_ptr[u]; e < row_ptr[u + 1]; e++) {
            uint32_t v = col[e];
            if (v <= u) continue;
            for (;;) {
                uint32_t ru = uf_find(label, u), rv = uf_find(label, v);
                if (ru == rv) break;
                uint32_t hi = ru > rv ? ru : rv, lo = ru > rv ? rv : ru;
                uint32_t expect = hi;
                if (__atomic_compare_exchange_n(&label[hi], &expect, lo, 0, __ATOMIC_RELAXED, __ATOMIC_RELAXED))
                    break;
            }
        }
    }
#pragma omp parallel for schedule(static)
    for (uint32_t v = 0; v < n; v++) label[v] = uf_find(label, v);
}

/* Vertices of the largest connected component (ties: smallest label),
 * ascending, written to out (capacity n).  Returns the count. */
uint32_t wl_lcc(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, uint32_t *out) {
    uint32_t *label = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
    uint32_t *size = (uint32_t *)calloc((size_t)n, sizeof(uint32_t));
    wl_components(n, row_ptr, col, label);
    for (uint32_t v = 0; v < n; v++) size[label[v]]++;
    uint32_t best = 0;
    for (uint32_t v = 1; v < n; v++)
        if (size[v] > size[best]) best = v;
    uint32_t cnt = 0;
    for (uint32_t v = 0; v < n; v++)
        if (label[v] == best) out[cnt++] = v;
    free(label);
    free(size);
    return cnt;
}

/* k distinct elements of cand[0..nc) chosen uniformly (partial Fisher-Yates
 * on a private copy), in draw order.  Returns 0, or -1 if k > nc. */
int wl_sample(const uint32_t *cand, uint32_t nc, uint32_t k, uint64_t key, uint32_t *out) {
    if (k > nc) return -1;
    uint32_t *c = (uint32_t *)malloc(((size_t)nc ? nc : 1) * sizeof(uint32_t));
    memcpy(c, cand, (size_t)nc * sizeof(uint32_t));
    for (uint32_t i = 0; i < k; i++) {
        uint32_t j = i + below(wl_draw(key, i), nc - i);
        uint32_t t = c[i]; c[i] = c[j]; c[j] = t;
        out[i] = c[i];
    }
    free(c);
    return 0;
}

int wl_num_threads(void) { return omp_get_max_threads(); }

/* Hop counts from src (breadth-first levels); UINT32_MAX where unreached. */
void wl_bfs_levels(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, uint32_t src, uint32_t *level) {
    for (uint32_t v = 0; v < n; v++) level[v] = UINT32_MAX;
    if (src >= n) return;
    uint32_t *queue = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
    uint64_t head = 0, tail = 0;
    level[src] = 0;
    queue[tail++] = src;
    while (head < tail) {
        uint32_t v = queue[head++];
        for (uint64_t e = row_ptr[v]; e < row_ptr[v + 1]; e++) {
            uint32_t u = col[e];
            if (level[u] == UINT32_MAX) {
                level[u] = level[v] + 1;
                queue[tail++] = u;
            }
        }
    }
    free(queue);
}

/* Seeds by the k-BFS heuristic of the paper's seed-selection study
 * (Section V): the first seed is `first`; each further seed is the candidate
 * not yet chosen whose sum of BFS levels from all seeds chosen so far is the
 * largest (mode 0, "eccentric": seeds far apart) or the smallest (mode 1,
 * "proximate": seeds close together); ties go to the smaller vertex id.
 * cand must lie in one connected component.  Returns 0, or -1 if k > nc. */
int wl_kbfs_seeds(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, const uint32_t *cand, uint32_t nc,
                  uint32_t first, uint32_t k, int mode, uint32_t *out) {
    if (k > nc) return -1;
    if (k == 0) return 0;
    uint64_t *acc = (uint64_t *)calloc((size_t)nc, sizeof(uint64_t));
    uint8_t *chosen = (uint8_t *)calloc((size_t)nc, 1);
    uint32_t *level = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
    uint32_t cur = first;
    for (uint32_t i = 0; i < nc; i++)
        if (cand[i] == first) chosen[i] = 1;
    out[0] = first;
    for (uint32_t s = 1; s < k; s++) {
        wl_bfs_levels(n, row_ptr, col, cur, level);
        int64_t best = -1;
        for (uint32_t i = 0; i < nc; i++) {
            acc[i] += level[cand[i]];
            if (chosen[i]) continue;
            if (best < 0) { best = i; continue; }
            const uint64_t a = acc[i], b = acc[best];
            const int better = mode == 0 ? (a > b || (a == b && cand[i] < cand[best]))
                                         : (a < b || (a == b && cand[i] < cand[best]));
            if (better) best = i;
        }
        chosen[best] = 1;
        cur = cand[best];
        out[s] = cur;
    }
    free(acc);
    free(chosen);
    free(level);
    return 0;
}
