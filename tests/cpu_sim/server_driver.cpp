// Drives the library's host code against the simulated runtime: graph upload
// and validation, batched solves, and the server under concurrent clients.
#include <algorithm>
#include <cstdio>
#include <thread>
#include <vector>

#include "steiner.h"

long hipsim_live_allocs();

#define CHECK(c)                                                            \
    do {                                                                    \
        if (!(c)) {                                                         \
            fprintf(stderr, "FAILED %s:%d %s (%s)\n", __FILE__, __LINE__, #c, \
                    steiner_last_error());                                  \
            return 1;                                                       \
        }                                                                   \
    } while (0)

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
    std::vector<uint32_t> badw = w;
    badw[3] = 0;
    steiner_graph *bad = nullptr;
    CHECK(steiner_graph_upload(n, col.size(), rp.data(), col.data(), badw.data(), 0, nullptr, 0, &bad) == STEINER_EINVAL);

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

    // server: budget for 3 queries, 5 slots, 4 client threads
    steiner_server *srv = nullptr;
    const uint64_t one = 13ull * n;
    CHECK(steiner_server_create(g, 10, 4, nullptr, &srv) == STEINER_EINVAL);
    CHECK(steiner_server_create(g, 3 * (one + 4096), 5, nullptr, &srv) == STEINER_OK);
    uint64_t t = 0;
    CHECK(steiner_server_submit(srv, nullptr, 0, &t) == STEINER_EINVAL);
    std::vector<uint32_t> too_many(n);
    for (uint32_t v = 0; v < n; v++) too_many[v] = v;
    CHECK(steiner_server_query_bytes(srv, 10) > one);
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
    CHECK(steiner_graph_free(g) == STEINER_OK);
    CHECK(hipsim_live_allocs() == 0);
    printf("cpu_sim ok\n");
    return 0;
}
