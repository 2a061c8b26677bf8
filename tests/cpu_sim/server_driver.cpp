// Drives the library's host code against the simulated runtime: graph upload
// and validation, batched solves, and the server under concurrent clients.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <thread>
#include <vector>

#include "engine.h"
#include "steiner.h"

long hipsim_live_allocs();
long hipsim_live_device_bytes();
void hipsim_stall(bool on);
void hipsim_freeze(bool on);

// The renumbering's maps against the caller's CSR: perm is a permutation by
// non-increasing degree and inv its inverse; every internal entry is a caller
// entry under perm; its edge id is the caller offset of the edge's entry that
// leaves the smaller caller id, with the same weight, shared by exactly the
// two entries of that edge; onew maps the id back to the entry leaving the
// smaller internal id.  (Simulated device memory is host memory.)
static bool renumbering_ok(const steiner_graph *g, const std::vector<uint64_t> &rp, const std::vector<uint32_t> &col,
                           const std::vector<uint32_t> &w) {
    const uint32_t n = g->n;
    const uint64_t nnz = g->nnz;
    if (!g->reordered || g->h_perm.size() != n || g->h_inv.size() != n) return false;
    std::vector<int> seen(n, 0);
    for (uint32_t i = 0; i < n; i++) {
        const uint32_t v = g->h_perm[i];
        if (v >= n || seen[v]++ || g->h_inv[v] != i) return false;
        if (i && rp[v + 1] - rp[v] > rp[g->h_perm[i - 1] + 1] - rp[g->h_perm[i - 1]]) return false;
    }
    std::vector<int> uses(nnz, 0);
    for (uint32_t i = 0; i < n; i++) {
        const uint32_t v = g->h_perm[i];
        const uint64_t b = g->d_rp[i], d = g->d_rp[i + 1] - b;
        if (d != rp[v + 1] - rp[v] || g->h_rp[i] != b) return false;
        for (uint64_t t = 0; t < d; t++) {
            const uint2 a = g->d_adj[b + t];
            if (t && a.x < g->d_adj[b + t - 1].x) return false;  // rows sorted by the new ids
            const uint32_t u = g->h_perm[a.x], f = g->d_eo[b + t];
            if (u == v) {
                if (f != stn::NONE) return false;
                continue;
            }
            const uint32_t lo = std::min(u, v), hi = std::max(u, v);
            if (f < rp[lo] || f >= rp[lo + 1] || col[f] != hi || w[f] != a.y) return false;
            uses[f]++;
            if (i < a.x && g->d_onew[f] != b + t) return false;
        }
    }
    for (uint32_t v = 0; v < n; v++)
        for (uint64_t f = rp[v]; f < rp[v + 1]; f++)
            if (uses[f] != (col[f] > v ? 2 : 0)) return false;
    return true;
}

// The fixed-stride copy of a graph whose rows all have at most ELL_W entries: row i of the internal CSR, two
// (col, w) pairs per 16 bytes, ELL_NONE past the row's end; no copy for any other graph.
static bool ell_ok(const steiner_graph *g) {
    if (g->max_deg > stn::ELL_W) return g->d_ell == nullptr && g->dg.ell == nullptr;
    if (!g->d_ell || g->dg.ell != g->d_ell) return false;
    for (uint32_t i = 0; i < g->n; i++) {
        const uint32_t b = g->d_rp[i], d = g->d_rp[i + 1] - b;
        const uint4 r0 = g->d_ell[2 * (size_t)i], r1 = g->d_ell[2 * (size_t)i + 1];
        const uint32_t c[4] = {r0.x, r0.z, r1.x, r1.z}, ww[4] = {r0.y, r0.w, r1.y, r1.w};
        for (uint32_t t = 0; t < stn::ELL_W; t++) {
            if (t < d && (c[t] != g->d_adj[b + t].x || ww[t] != g->d_adj[b + t].y)) return false;
            if (t >= d && c[t] != stn::ELL_NONE) return false;
        }
    }
    return true;
}

#define CHECK(c)                                                            \
    do {                                                                    \
        if (!(c)) {                                                         \
            fprintf(stderr, "FAILED %s:%d %s (%s)\n", __FILE__, __LINE__, #c, \
                    steiner_last_error());                                  \
            return 1;                                                       \
        }                                                                   \
    } while (0)

// Everything a server holds on the device is its budget: fixed + slots * slot_bytes + pool, allocated exactly.
// A waiter past its timeout gets ETIMEDOUT and can wait again; a waiter blocked at destroy gets ECANCELED.
static int server_memory_and_waits(steiner_graph *g) {
    const long before = hipsim_live_device_bytes();
    steiner_server *srv = nullptr;
    const uint64_t budget = 5ull << 20;
    CHECK(steiner_server_create(g, budget, 7, nullptr, &srv) == STEINER_OK);
    uint64_t fixed = 0, slot = 0, pool = 0;
    uint32_t slots = 0;
    CHECK(steiner_server_memory(srv, &fixed, &slot, &slots, &pool) == STEINER_OK);
    CHECK(slots == 7 && fixed + slots * slot + pool == budget);
    CHECK((uint64_t)(hipsim_live_device_bytes() - before) <= budget);
    CHECK(steiner_server_query_bytes(srv, 5) > slot);
    // a request whose pool region exceeds the pool is refused at submit
    std::vector<uint32_t> all(g->n);
    for (uint32_t v = 0; v < g->n; v++) all[v] = v;
    uint64_t t = 0;
    {
        steiner_server *small = nullptr;
        const uint64_t one = steiner_server_query_bytes(srv, 2) + fixed;
        CHECK(steiner_server_create(g, one + 4096, 3, nullptr, &small) == STEINER_OK);
        CHECK(steiner_server_submit(small, all.data(), g->n, &t) == STEINER_ENOMEM);
        CHECK(steiner_server_destroy(small) == STEINER_OK);
    }
    hipsim_stall(true);
    const uint32_t s1[] = {3, 9, 27};
    CHECK(steiner_server_submit(srv, s1, 3, &t) == STEINER_OK);
    steiner_result *r = nullptr;
    CHECK(steiner_server_wait(srv, t, 2000, &r) == STEINER_ETIMEDOUT && r == nullptr);
    hipsim_stall(false);
    CHECK(steiner_server_wait(srv, t, -1, &r) == STEINER_OK && r != nullptr);
    steiner_result_free(r);
    CHECK(steiner_server_wait(srv, t, 0, &r) == STEINER_EINVAL);  // a ticket is consumed by its result
    hipsim_stall(true);
    uint64_t t2 = 0, t3 = 0;
    const uint32_t s2[] = {1, 2, 40}, s3[] = {5, 6};
    CHECK(steiner_server_submit(srv, s2, 3, &t2) == STEINER_OK);
    CHECK(steiner_server_submit(srv, s3, 2, &t3) == STEINER_OK);
    int rc2 = 0, rc3 = 0;
    std::thread w2([&] {
        steiner_result *x = nullptr;
        rc2 = steiner_server_wait(srv, t2, -1, &x);
    });
    std::thread w3([&] {
        steiner_result *x = nullptr;
        rc3 = steiner_server_wait(srv, t3, 60000000, &x);
    });
    std::this_thread::sleep_for(std::chrono::milliseconds(100));
    CHECK(steiner_server_destroy(srv) == STEINER_OK);
    w2.join();
    w3.join();
    hipsim_stall(false);
    CHECK(rc2 == STEINER_ECANCELED && rc3 == STEINER_ECANCELED);
    // a pass whose round counter stops moving fails the resident and the waiting requests instead of
    // relaunching rounds for ever
    CHECK(steiner_server_create(g, budget, 1, nullptr, &srv) == STEINER_OK);
    hipsim_freeze(true);
    CHECK(steiner_server_submit(srv, s2, 3, &t2) == STEINER_OK);
    CHECK(steiner_server_submit(srv, s3, 2, &t3) == STEINER_OK);
    steiner_result *x = nullptr;
    CHECK(steiner_server_wait(srv, t2, 20000000, &x) == STEINER_EDEVICE && x == nullptr);
    CHECK(steiner_server_wait(srv, t3, 20000000, &x) == STEINER_EDEVICE && x == nullptr);
    hipsim_freeze(false);
    CHECK(steiner_server_destroy(srv) == STEINER_OK);
    CHECK(hipsim_live_device_bytes() == before);
    return 0;
}

// A query holds at most STEINER_MAX_SEEDS distinct seeds: one more is EINVAL for solves and for the server.
static int max_seeds(uint32_t) {
    const uint32_t n = STEINER_MAX_SEEDS + 10;
    std::vector<uint64_t> rp(n + 1);
    std::vector<uint32_t> col, w;
    for (uint32_t v = 0; v < n; v++) {
        rp[v] = col.size();
        if (v > 0) { col.push_back(v - 1); w.push_back(1); }
        if (v + 1 < n) { col.push_back(v + 1); w.push_back(1); }
    }
    rp[n] = col.size();
    steiner_graph *g = nullptr;
    CHECK(steiner_graph_upload(n, col.size(), rp.data(), col.data(), w.data(), 0, nullptr, 0, &g) == STEINER_OK);
    std::vector<uint32_t> seeds(STEINER_MAX_SEEDS + 1);
    for (uint32_t i = 0; i < seeds.size(); i++) seeds[i] = i;
    steiner_result *r = nullptr;
    CHECK(steiner_solve(g, seeds.data(), (uint32_t)seeds.size(), nullptr, &r) == STEINER_EINVAL && r == nullptr);
    std::vector<uint32_t> dup = seeds;  // duplicates do not count
    dup.back() = 0;
    steiner_server *srv = nullptr;
    CHECK(steiner_server_create(g, 64ull << 20, 2, nullptr, &srv) == STEINER_OK);
    uint64_t t = 0;
    CHECK(steiner_server_submit(srv, seeds.data(), (uint32_t)seeds.size(), &t) == STEINER_EINVAL);
    CHECK(steiner_server_destroy(srv) == STEINER_OK);
    CHECK(steiner_graph_free(g) == STEINER_OK);
    CHECK(hipsim_live_allocs() == 0);
    return 0;
}

// Every device or pinned-host allocation of an upload, a solve, a batch and a server start fails in turn
// (stn::set_fault_alloc_after): the call returns ENOMEM and, once the graph is freed, nothing is left allocated.
static int injected_allocation_failures(const std::vector<uint64_t> &rp, const std::vector<uint32_t> &col,
                                        const std::vector<uint32_t> &w) {
    const uint32_t n = (uint32_t)rp.size() - 1;
    const uint32_t seeds[] = {1, 30, 50, 7};
    std::vector<std::vector<uint32_t>> sets = {{1, 5, 9}, {2, 30}, {0, 63, 10, 20, 40}};
    std::vector<const uint32_t *> ptrs;
    std::vector<uint32_t> ks;
    for (auto &x : sets) { ptrs.push_back(x.data()); ks.push_back((uint32_t)x.size()); }
    for (int what = 0; what < 4; what++) {  // upload, solve, batch, server
        long points = -1;
        for (long lim = 0; lim < 400 && points < 0; lim++) {
            steiner_graph *g = nullptr;
            stn::set_fault_alloc_after(what == 0 ? lim : -1);
            int rc = steiner_graph_upload(n, col.size(), rp.data(), col.data(), w.data(), 0, nullptr, 0, &g);
            if (what == 0) {
                CHECK(rc == STEINER_OK || rc == STEINER_ENOMEM);
                if (rc == STEINER_OK) points = lim;
            } else {
                CHECK(rc == STEINER_OK);
                stn::set_fault_alloc_after(lim);
                if (what == 1) {
                    steiner_result *r = nullptr;
                    rc = steiner_solve(g, seeds, 4, nullptr, &r);
                    if (rc == STEINER_OK) steiner_result_free(r);
                } else if (what == 2) {
                    std::vector<steiner_result *> outs(sets.size(), nullptr);
                    std::vector<int> st(sets.size());
                    rc = steiner_solve_batch(g, (uint32_t)sets.size(), ptrs.data(), ks.data(), nullptr, outs.data(),
                                             st.data());
                    for (size_t i = 0; i < sets.size(); i++)
                        if (rc == STEINER_OK) {
                            CHECK(st[i] == STEINER_OK);
                            steiner_result_free(outs[i]);
                        }
                } else {
                    steiner_server *srv = nullptr;
                    rc = steiner_server_create(g, 4ull << 20, 3, nullptr, &srv);
                    if (rc == STEINER_OK) {
                        uint64_t t = 0;
                        steiner_result *r = nullptr;
                        CHECK(steiner_server_submit(srv, seeds, 4, &t) == STEINER_OK);
                        rc = steiner_server_wait(srv, t, -1, &r);
                        if (rc == STEINER_OK) steiner_result_free(r);
                        CHECK(steiner_server_destroy(srv) == STEINER_OK);
                    }
                }
                CHECK(rc == STEINER_OK || rc == STEINER_ENOMEM);
                if (rc == STEINER_OK) points = lim;
            }
            stn::set_fault_alloc_after(-1);
            if (g) CHECK(steiner_graph_free(g) == STEINER_OK);
            CHECK(hipsim_live_allocs() == 0);
        }
        CHECK(points > 0);
        printf("injected allocation failures: operation %d fails cleanly at each of its %ld allocations\n", what,
               points);
    }
    return 0;
}

int main() {
    const uint32_t n = 64;
    std::vector<uint64_t> rp(n + 1);
    std::vector<uint32_t> col, w;
    for (uint32_t v = 0; v < n; v++) {  // path graph
        rp[v] = col.size();
        if (v > 0) { col.push_back(v - 1); w.push_back(2); }
        if (v + 1 < n) { col.push_back(v + 1); w.push_back(2); }
    }
    rp[n] = col.size();
    steiner_graph *g = nullptr;
    CHECK(steiner_graph_upload(n, col.size(), rp.data(), col.data(), w.data(), 0, nullptr, 1, &g) == STEINER_OK);
    CHECK(ell_ok(g));
    {
        // fixed-stride rows of a renumbered graph (built from the internal CSR), with a parallel edge and a
        // self-loop: every row still has at most four entries
        std::vector<std::vector<std::pair<uint32_t, uint32_t>>> rows(n);  // (col, w)
        auto edge = [&](uint32_t a, uint32_t b, uint32_t wt) {
            rows[a].push_back({b, wt});
            rows[b].push_back({a, wt});  // a self-loop gets both entries in its own row
        };
        for (uint32_t v = 0; v + 1 < n; v++) edge(v, v + 1, 2);
        edge(20, 21, 1);
        edge(9, 9, 4);
        std::vector<uint64_t> rp3(n + 1);
        std::vector<uint32_t> col3, w3;
        for (uint32_t v = 0; v < n; v++) {
            std::sort(rows[v].begin(), rows[v].end());
            rp3[v] = col3.size();
            for (auto &e : rows[v]) { col3.push_back(e.first); w3.push_back(e.second); }
        }
        rp3[n] = col3.size();
        steiner_graph *g3 = nullptr;
        CHECK(steiner_graph_upload(n, col3.size(), rp3.data(), col3.data(), w3.data(), 0, nullptr,
                                   STEINER_UPLOAD_REORDER | 1u, &g3) == STEINER_OK);
        CHECK(g3->reordered && g3->max_deg <= stn::ELL_W && ell_ok(g3));
        CHECK(steiner_graph_free(g3) == STEINER_OK);
    }
    std::vector<uint32_t> badw = w;
    badw[3] = 0;
    steiner_graph *bad = nullptr;
    CHECK(steiner_graph_upload(n, col.size(), rp.data(), col.data(), badw.data(), 0, nullptr, 0, &bad) == STEINER_EINVAL);
    CHECK(steiner_graph_upload(n, col.size(), rp.data(), col.data(), w.data(), 0, nullptr,
                               STEINER_UPLOAD_REORDER | STEINER_UPLOAD_KEEP_ORDER, &bad) == STEINER_EINVAL);
    {
        // the internal renumbering (host side: radix sort, twin matching and per-row sorts on worker
        // threads, offset maps) on a path plus a hub joined to every vertex, which the automatic rule
        // renumbers; every 7th path edge is doubled with weights 5 then 1 on one side and 1 then 5 on
        // the other, every 11th vertex has a self-loop
        const uint32_t n2 = 4096;
        std::vector<uint64_t> rp2(n2 + 1);
        std::vector<uint32_t> col2, w2;
        for (uint32_t v = 0; v < n2; v++) {
            rp2[v] = col2.size();
            if (v == 0) {
                for (uint32_t u = 1; u < n2; u++) { col2.push_back(u); w2.push_back(3); }
                continue;
            }
            col2.push_back(0);
            w2.push_back(3);
            if (v > 1) {
                col2.push_back(v - 1);
                w2.push_back(1);
                if ((v - 1) % 7 == 0) { col2.push_back(v - 1); w2.push_back(5); }
            }
            if (v % 11 == 0) { col2.push_back(v); w2.push_back(2); }
            if (v + 1 < n2) {
                if (v % 7 == 0) { col2.push_back(v + 1); w2.push_back(5); }
                col2.push_back(v + 1);
                w2.push_back(1);
            }
        }
        rp2[n2] = col2.size();
        for (uint32_t fl : {0u, (uint32_t)STEINER_UPLOAD_REORDER}) {
            steiner_graph *g2 = nullptr;
            CHECK(steiner_graph_upload(n2, col2.size(), rp2.data(), col2.data(), w2.data(), 0, nullptr, fl | 1u, &g2) ==
                  STEINER_OK);
            CHECK(renumbering_ok(g2, rp2, col2, w2));
            CHECK(ell_ok(g2));  // a hub: no fixed-stride copy
            const uint32_t seeds2[] = {4095, 17, 900, 17};
            steiner_result *r2 = nullptr;
            CHECK(steiner_solve(g2, seeds2, 4, nullptr, &r2) == STEINER_OK);
            uint64_t m2 = 0;
            CHECK(steiner_result_edges(r2, &m2, nullptr, nullptr, nullptr) == STEINER_OK && m2 == 2);
            steiner_result_free(r2);
            CHECK(steiner_graph_free(g2) == STEINER_OK);
        }
        // an asymmetric CSR keeps the caller's order, or is refused when renumbering is forced
        std::vector<uint32_t> w3 = w2;
        w3[rp2[5] + 1] = 9;
        steiner_graph *g3 = nullptr;
        CHECK(steiner_graph_upload(n2, col2.size(), rp2.data(), col2.data(), w3.data(), 0, nullptr, 0, &g3) == STEINER_OK);
        CHECK(!g3->reordered);
        CHECK(steiner_graph_free(g3) == STEINER_OK);
        CHECK(steiner_graph_upload(n2, col2.size(), rp2.data(), col2.data(), w3.data(), 0, nullptr, STEINER_UPLOAD_REORDER,
                                   &g3) == STEINER_EINVAL);
    }

    // the graph-captured driver: same trees as the host-stepped one
    {
        steiner_options go{};
        go.driver = 4;
        const uint32_t sd[] = {3, 44, 20, 61};
        steiner_result *r1 = nullptr, *r2 = nullptr;
        for (int rep = 0; rep < 3; rep++) {
            CHECK(steiner_solve(g, sd, 4, &go, &r1) == STEINER_OK);
            CHECK(steiner_solve(g, sd, 4, nullptr, &r2) == STEINER_OK);
            uint64_t m1 = 0, m2 = 0;
            CHECK(steiner_result_edges(r1, &m1, nullptr, nullptr, nullptr) == STEINER_OK);
            CHECK(steiner_result_edges(r2, &m2, nullptr, nullptr, nullptr) == STEINER_OK);
            CHECK(m1 == m2 && steiner_result_total(r1) == steiner_result_total(r2));
            steiner_result_free(r1);
            steiner_result_free(r2);
        }
    }

    // batch through the pass driver
    std::vector<std::vector<uint32_t>> sets = {{1, 5, 9}, {7}, {2, 2, 30}, {0, 63, 10, 20, 40}};
    std::vector<const uint32_t *> ptrs;
    std::vector<uint32_t> ks;
    for (auto &s : sets) { ptrs.push_back(s.data()); ks.push_back((uint32_t)s.size()); }
    std::vector<steiner_result *> outs(sets.size());
    std::vector<int> st(sets.size());
    CHECK(steiner_solve_batch(g, (uint32_t)sets.size(), ptrs.data(), ks.data(), nullptr, outs.data(), st.data()) == STEINER_OK);
    const uint64_t want[] = {2, 0, 1, 4};
    for (size_t i = 0; i < sets.size(); i++) {
        uint64_t m = 0;
        CHECK(st[i] == STEINER_OK);
        CHECK(steiner_result_edges(outs[i], &m, nullptr, nullptr, nullptr) == STEINER_OK);
        CHECK(m == want[i]);
        steiner_result_free(outs[i]);
    }

    // the allocation-free solve: same tree as steiner_solve, twice in a row (the second smaller), no allocation
    {
        const uint32_t s1[] = {40, 3, 17, 3, 60, 25}, s2[] = {9, 2};
        for (int rep = 0; rep < 2; rep++) {
            const uint32_t *sd = rep ? s2 : s1;
            const uint32_t kk = rep ? 2 : 6;
            steiner_result *r = nullptr;
            CHECK(steiner_solve(g, sd, kk, nullptr, &r) == STEINER_OK);
            uint64_t m = 0;
            const uint32_t *ra, *rb, *rw;
            CHECK(steiner_result_edges(r, &m, &ra, &rb, &rw) == STEINER_OK);
            const long live = hipsim_live_allocs();
            std::vector<uint32_t> a(n), b(n), ww(n);
            uint64_t m2 = 0, tot = 0;
            CHECK(steiner_solve_noalloc(g, sd, kk, nullptr, n, &m2, a.data(), b.data(), ww.data(), &tot) == STEINER_OK);
            CHECK(hipsim_live_allocs() == live);
            CHECK(m2 == m && tot == steiner_result_total(r));
            for (uint64_t t = 0; t < m; t++) CHECK(a[t] == ra[t] && b[t] == rb[t] && ww[t] == rw[t]);
            if (m) {
                uint64_t m3 = 0;
                CHECK(steiner_solve_noalloc(g, sd, kk, nullptr, m - 1, &m3, a.data(), b.data(), ww.data(), &tot) ==
                      STEINER_ENOMEM);
                CHECK(m3 == m);
            }
            steiner_result_free(r);
        }
        std::vector<uint32_t> many(9000, 1);
        uint64_t m = 0, tot = 0;
        CHECK(steiner_solve_noalloc(g, many.data(), 9000, nullptr, 0, &m, nullptr, nullptr, nullptr, &tot) ==
              STEINER_ENOMEM);
        const uint32_t bad[] = {1, 64};
        CHECK(steiner_solve_noalloc(g, bad, 2, nullptr, 0, &m, nullptr, nullptr, nullptr, &tot) == STEINER_EINVAL);
    }

    // server: budget for 3 queries, 5 slots, 4 client threads
    steiner_server *srv = nullptr;
    CHECK(steiner_server_create(g, 10, 4, nullptr, &srv) == STEINER_EINVAL);
    uint64_t fixed5 = 0, one = 0;
    {
        steiner_server *probe = nullptr;
        CHECK(steiner_server_create(g, 64ull << 20, 5, nullptr, &probe) == STEINER_OK);
        CHECK(steiner_server_memory(probe, &fixed5, nullptr, nullptr, nullptr) == STEINER_OK);
        one = steiner_server_query_bytes(probe, 9);
        CHECK(steiner_server_destroy(probe) == STEINER_OK);
    }
    CHECK(steiner_server_create(g, fixed5 + 3 * one + 4096, 5, nullptr, &srv) == STEINER_OK);
    uint64_t t = 0;
    CHECK(steiner_server_submit(srv, nullptr, 0, &t) == STEINER_EINVAL);
    std::vector<uint32_t> too_many(n);
    for (uint32_t v = 0; v < n; v++) too_many[v] = v;
    CHECK(steiner_server_query_bytes(srv, 40) > one && steiner_server_query_bytes(srv, 2) <= one);
    {
        uint32_t slots = 0;
        CHECK(steiner_server_memory(srv, nullptr, nullptr, &slots, nullptr) == STEINER_OK);
        CHECK(slots >= 3 && slots <= 5);
    }
    int failures = 0;
    std::vector<std::thread> clients;
    for (int c = 0; c < 4; c++) {
        clients.emplace_back([&, c] {
            for (int i = 0; i < 40; i++) {
                std::vector<uint32_t> s;
                const uint32_t k = 1 + (uint32_t)((c * 7 + i * 3) % 9);
                for (uint32_t j = 0; j < k; j++) s.push_back((c * 5 + i + j * 11) % n);
                uint64_t tk = 0;
                if (steiner_server_submit(srv, s.data(), (uint32_t)s.size(), &tk) != STEINER_OK) { failures++; continue; }
                steiner_result *r = nullptr;
                if (steiner_server_wait(srv, tk, -1, &r) != STEINER_OK) { failures++; continue; }
                uint64_t m = 0;
                steiner_result_edges(r, &m, nullptr, nullptr, nullptr);
                std::vector<uint32_t> u = s;
                std::sort(u.begin(), u.end());
                u.erase(std::unique(u.begin(), u.end()), u.end());
                if (m != u.size() - 1) failures++;
                steiner_result_free(r);
            }
        });
    }
    for (auto &th : clients) th.join();
    CHECK(failures == 0);
    // pending work is canceled at destroy
    for (int i = 0; i < 6; i++) {
        uint32_t s[3] = {1, 2, (uint32_t)(3 + i)};
        CHECK(steiner_server_submit(srv, s, 3, &t) == STEINER_OK);
    }
    CHECK(steiner_server_destroy(srv) == STEINER_OK);
    CHECK(server_memory_and_waits(g) == 0);
    CHECK(steiner_graph_free(g) == STEINER_OK);
    CHECK(hipsim_live_allocs() == 0);
    CHECK(max_seeds(n) == 0);
    CHECK(injected_allocation_failures(rp, col, w) == 0);
    printf("cpu_sim ok\n");
    return 0;
}
