/* Test-side property verifier (test infrastructure, shares nothing with the library):
 * properties that pin the unique results of Alg. 2 Steps 1 and 2 at sizes
 * where the oracle's full solve is too slow.  Keys are (dist << 32) | seed
 * index, all ones = unreached, as in the library's output. */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define KEY_INF UINT64_MAX

/* Step 1 (Alg. 4's relaxation, ties to the smaller seed index): with
 * positive weights the relaxation has exactly one fixed point, so key is the
 * result iff key[S[i]] = (0, i) and every other vertex holds the minimum over
 * its neighbours u of ((dist(u) + w) << 32 | src(u)) among candidates whose
 * distance fits below 2^32 - 1 (unreached if none).  Returns -1, or the first
 * vertex that breaks this. */
int64_t chk_voronoi_fixed_point(uint32_t n, const uint64_t *rp, const uint32_t *col, const uint32_t *w, uint32_t k,
                                const uint32_t *S, const uint64_t *key) {
    uint8_t *is_seed = (uint8_t *)calloc(n ? n : 1, 1);
    for (uint32_t i = 0; i < k; i++) is_seed[S[i]] = 1;
    int64_t bad = -1;
    for (uint32_t i = 0; i < k && bad < 0; i++)
        if (key[S[i]] != (uint64_t)i) bad = S[i];
#pragma omp parallel for schedule(dynamic, 4096)
    for (uint32_t v = 0; v < n; v++) {
        if (is_seed[v] || bad >= 0) continue;
        uint64_t best = KEY_INF;
        for (uint64_t e = rp[v]; e < rp[v + 1]; e++) {
            const uint64_t ku = key[col[e]];
            if (ku == KEY_INF) continue;
            const uint64_t d = (ku >> 32) + w[e];
            if (d >= 0xFFFFFFFFull) continue;
            const uint64_t c = (d << 32) | (ku & 0xFFFFFFFFull);
            if (c < best) best = c;
        }
        if (best != key[v]) {
#pragma omp critical
            if (bad < 0 || (int64_t)v < bad) bad = v;
        }
    }
    free(is_seed);
    return bad;
}

/* Step 2 (Alg. 5, ties to the smaller edge id): pt holds, for every pair
 * (i, j), i < j, at index j(j-1)/2 + i, the minimum of (bsum << 32 | e) over
 * the edges a -> b, a < b, at CSR offset e joining cells i and j (bsum =
 * dist(a) + w + dist(b)), all ones if there is none.  Verified as: no
 * candidate is below its pair's entry, and every finite entry equals some
 * candidate.  Returns 0, 1 (a candidate below its entry), 2 (a finite entry
 * no edge attains) or 3 (a sum of 2^32 or more). */
int chk_boundary(uint32_t n, const uint64_t *rp, const uint32_t *col, const uint32_t *w, const uint64_t *key, uint32_t k,
                 const uint64_t *pt) {
    const uint64_t P = (uint64_t)k * (k - 1) / 2;
    uint8_t *hit = (uint8_t *)calloc(P ? P : 1, 1);
    int status = 0;
#pragma omp parallel for schedule(dynamic, 4096)
    for (uint32_t a = 0; a < n; a++) {
        const uint64_t ka = key[a];
        if (ka == KEY_INF) continue;
        for (uint64_t e = rp[a]; e < rp[a + 1]; e++) {
            const uint32_t b = col[e];
            if (b <= a) continue;
            const uint64_t kb = key[b];
            if (kb == KEY_INF) continue;
            const uint32_t i1 = (uint32_t)ka, i2 = (uint32_t)kb;
            if (i1 == i2) continue;
            const uint64_t bsum = (ka >> 32) + w[e] + (kb >> 32);
            if (bsum >= (1ull << 32)) {
#pragma omp atomic write
                status = 3;
                continue;
            }
            const uint32_t i = i1 < i2 ? i1 : i2, j = i1 < i2 ? i2 : i1;
            const uint64_t p = (uint64_t)j * (j - 1) / 2 + i;
            const uint64_t val = (bsum << 32) | e;
            if (val < pt[p]) {
#pragma omp atomic write
                status = 1;
            } else if (val == pt[p]) {
#pragma omp atomic write
                hit[p] = 1;
            }
        }
    }
    if (status == 0)
        for (uint64_t p = 0; p < P; p++)
            if (pt[p] != KEY_INF && !hit[p]) {
                status = 2;
                break;
            }
    free(hit);
    return status;
}
