// One multi-query pass over a resident graph: Alg. 2 Steps 1-7 for every
// query of the batch, sharing the relaxation rounds and the boundary scan.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <tuple>

#include "engine.h"

namespace stn {

// Chunks of the rows above small_max (sizes the chunk lists); one O(n) host
// pass per (small_max, chunk) and graph, remembered unless `remember` is false.
uint64_t big_row_chunks(const steiner_graph *g, uint32_t small_max, uint32_t chunk, bool remember) {
    const uint64_t memo_key = ((uint64_t)small_max << 32) | chunk;
    {
        std::lock_guard<std::mutex> lk(g->memo_mu);
        auto it = g->chunk_memo.find(memo_key);
        if (it != g->chunk_memo.end()) return it->second;
    }
    uint64_t t = 0;
    for (uint32_t v = 0; v < g->n; v++) {
        uint64_t d = g->h_rp[v + 1] - g->h_rp[v];
        if (d > small_max) t += (d + chunk - 1) / chunk;
    }
    if (!remember) return t;
    std::lock_guard<std::mutex> lk(g->memo_mu);
    g->chunk_memo[memo_key] = t;
    return t;
}

const ChunkTable *chunk_table(steiner_graph *g, uint32_t small_max, uint32_t chunk, int *rc) {
    *rc = STEINER_OK;
    const uint64_t memo_key = ((uint64_t)small_max << 32) | chunk;
    auto it = g->chunk_tables.find(memo_key);
    if (it != g->chunk_tables.end()) return it->second.get();
    std::unique_ptr<ChunkTable> t(new ChunkTable());
    const uint32_t n = g->n;
    uint32_t nx = 0;
    while (nx < n && g->h_rp[nx + 1] - g->h_rp[nx] > small_max) nx++;
    bool prefix = true;
    for (uint32_t v = nx; v < n && prefix; v++) prefix = g->h_rp[v + 1] - g->h_rp[v] <= small_max;
    if (!prefix || nx == 0) {
        g->chunk_tables[memo_key] = nullptr;  // remembered: no chunk memory on this graph
        return nullptr;
    }
    std::vector<uint32_t> start(nx + 1, 0);
    uint64_t total = 0;
    for (uint32_t v = 0; v < nx; v++) {
        start[v] = (uint32_t)total;
        total += (g->h_rp[v + 1] - g->h_rp[v] + chunk - 1) / chunk;
    }
    if (total >= (1ull << 32)) {
        g->chunk_tables[memo_key] = nullptr;
        return nullptr;
    }
    start[nx] = (uint32_t)total;
    if ((*rc = t->start.ensure(((size_t)nx + 1) * 4))) return nullptr;
    *rc = hip_check(hipMemcpyAsync(t->start.ptr, start.data(), ((size_t)nx + 1) * 4, hipMemcpyHostToDevice, g->stream),
                    "H2D chunk table");
    if (!*rc) *rc = hip_check(hipStreamSynchronize(g->stream), "chunk table");
    if (*rc) {
        t->start.release();
        return nullptr;
    }
    t->nxrow = nx;
    t->xchunks = (uint32_t)total;
    ChunkTable *raw = t.get();
    g->chunk_tables[memo_key] = std::move(t);
    return raw;
}

int bind_chunk_memory(VorParams &P, steiner_graph *g, const Options &o, uint32_t Q, DevBuf &xkey) {
    // The large rows' chunk memory: not with the light/heavy split, where a chunk is expanded once per edge
    // class, and only when the rows above small_max are a prefix of the ids.
    int rc = STEINER_OK;
    const ChunkTable *ct = P.split ? nullptr : chunk_table(g, o.small_max, o.chunk, &rc);
    if (rc || !ct) return rc;
    if ((rc = xkey.ensure((size_t)Q * ct->xchunks * 8))) return rc;
    P.xkey = xkey.as<uint64_t>();
    P.xchunk = ct->start.as<uint32_t>();
    P.nxrow = ct->nxrow;
    P.xchunks = ct->xchunks;
    return STEINER_OK;
}

void bind_pass(VorParams &P, const DevGraph &dg, uint8_t *ctl, const Layout &L, uint32_t Q) {
    P.g = dg;
    P.cnt = (Counters *)(ctl + L.counters);
    P.pass = (PassCtl *)(ctl + L.pass);
    P.far_min = (uint32_t *)(ctl + L.far_min);
    P.near_mark = (uint32_t *)(ctl + L.near_mark);
    P.settle_mark = (uint32_t *)(ctl + L.settle_mark);
    P.slot.thr = (uint64_t *)(ctl + L.thr);
    P.slot.thr_prev = (uint64_t *)(ctl + L.thr_prev);
    P.slot.carry = (uint32_t *)(ctl + L.carry);
    P.slot.active = (uint32_t *)(ctl + L.active);
    P.slot.adv = (uint32_t *)(ctl + L.adv);
    P.slot.done = (uint32_t *)(ctl + L.done);
    P.slot.advances = (uint32_t *)(ctl + L.advances);
    P.nslots = Q;
}

void bind_state(VorParams &P, const Options &o, uint64_t cap_s, uint64_t cap_b) {
    P.cap_s = (uint32_t)cap_s;
    P.cap_b = (uint32_t)cap_b;
    P.delta = o.delta;
    P.small_max = o.small_max;
    P.chunk = o.chunk;
    P.local_iters = o.local_iters;
    P.counting = o.counting ? 1u : 0u;
    P.split = (o.delta != 0xFFFFFFFFu && o.split) ? 1u : 0u;
    P.lq_mode = o.lq_mode;
    P.defer_min = (o.split || !o.defer_min) ? 0 : std::max(o.defer_min, o.small_max);
}

namespace {

struct Timer {
    bool on;
    hipStream_t s;
    std::vector<hipEvent_t> ev;
    Timer(bool on_, hipStream_t s_) : on(on_), s(s_) {}
    void mark() {
        if (!on) return;
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) { on = false; return; }
        (void)hipEventRecord(e, s);
        ev.push_back(e);
    }
    double ms(size_t a, size_t b) {
        if (!on || b >= ev.size()) return 0.0;
        float m = 0.f;
        (void)hipEventSynchronize(ev[b]);
        (void)hipEventElapsedTime(&m, ev[a], ev[b]);
        return m;
    }
    ~Timer() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
};

}  // namespace

// From each vertex not yet clustered, in id order, a breadth-first search
// over unclustered vertices collects up to CLUSTER_MAX vertices holding at
// most CLUSTER_EDGES edge entries (a vertex with more is a cluster of its
// own); each member's edges are then split into internal ones (target's local
// index; self-loops dropped, they never improve a key) and external ones
// (target vertex).
int ClusterSet::build(steiner_graph *g) {
    if (built) return STEINER_OK;
    const uint32_t n = g->n;
    const uint64_t nnz = g->nnz;
    hipStream_t st = g->stream;
    int rc;
    std::vector<uint2> adj(nnz);
    if (nnz && (rc = hip_check(hipMemcpyAsync(adj.data(), g->d_adj, nnz * 8, hipMemcpyDeviceToHost, st), "D2H adjacency")))
        return rc;
    if ((rc = hip_check(hipStreamSynchronize(st), "D2H adjacency"))) return rc;
    const std::vector<uint64_t> &rp = g->h_rp;
    std::vector<uint32_t> cl(n, NONE), loc(n), mem, cs;
    mem.reserve(n);
    cs.push_back(0);
    for (uint32_t s0 = 0; s0 < n; s0++) {
        if (cl[s0] != NONE) continue;
        const uint32_t c = (uint32_t)cs.size() - 1, base = (uint32_t)mem.size();
        uint64_t edges = rp[s0 + 1] - rp[s0];
        cl[s0] = c;
        loc[s0] = 0;
        mem.push_back(s0);
        for (size_t head = base; head < mem.size() && mem.size() - base < CLUSTER_MAX; head++) {
            const uint32_t v = mem[head];
            for (uint64_t e = rp[v]; e < rp[v + 1] && mem.size() - base < CLUSTER_MAX; e++) {
                const uint32_t u = adj[e].x;
                const uint64_t du = rp[u + 1] - rp[u];
                if (cl[u] != NONE || edges + du > CLUSTER_EDGES) continue;
                cl[u] = c;
                loc[u] = (uint32_t)(mem.size() - base);
                mem.push_back(u);
                edges += du;
            }
        }
        cs.push_back((uint32_t)mem.size());
    }
    nclusters = (uint32_t)cs.size() - 1;
    std::vector<uint32_t> irp_h((size_t)n + 1, 0), erp_h((size_t)n + 1, 0);
    std::vector<uint2> ie_h, ee_h;
    ie_h.reserve(nnz);
    for (uint32_t p = 0; p < n; p++) {
        const uint32_t v = mem[p];
        for (uint64_t e = rp[v]; e < rp[v + 1]; e++) {
            const uint32_t u = adj[e].x;
            if (u == v) continue;
            if (cl[u] == cl[v]) ie_h.push_back(make_uint2(loc[u], adj[e].y));
            else ee_h.push_back(make_uint2(u, adj[e].y));
        }
        irp_h[p + 1] = (uint32_t)ie_h.size();
        erp_h[p + 1] = (uint32_t)ee_h.size();
    }
    if ((rc = members.ensure((size_t)n * 4 + 4)) || (rc = cstart.ensure(cs.size() * 4)) ||
        (rc = cl_of.ensure((size_t)n * 4 + 4)) || (rc = irp.ensure(irp_h.size() * 4)) ||
        (rc = erp.ensure(erp_h.size() * 4)) || (rc = ie.ensure(ie_h.size() * 8 + 8)) ||
        (rc = ee.ensure(ee_h.size() * 8 + 8)) || (rc = expanded.ensure((size_t)n * 8 + 8)) ||
        (rc = lists.ensure((size_t)nclusters * 8 + 8)) || (rc = stamp.ensure((size_t)nclusters * 4 + 4)) ||
        (rc = ctl.ensure(sizeof(ClusterCtl))))
        return rc;
    rc = hip_check(hipMemcpyAsync(members.ptr, mem.data(), (size_t)n * 4, hipMemcpyHostToDevice, st), "H2D clusters");
    if (!rc) rc = hip_check(hipMemcpyAsync(cstart.ptr, cs.data(), cs.size() * 4, hipMemcpyHostToDevice, st), "H2D clusters");
    if (!rc) rc = hip_check(hipMemcpyAsync(cl_of.ptr, cl.data(), (size_t)n * 4, hipMemcpyHostToDevice, st), "H2D clusters");
    if (!rc) rc = hip_check(hipMemcpyAsync(irp.ptr, irp_h.data(), irp_h.size() * 4, hipMemcpyHostToDevice, st), "H2D clusters");
    if (!rc) rc = hip_check(hipMemcpyAsync(erp.ptr, erp_h.data(), erp_h.size() * 4, hipMemcpyHostToDevice, st), "H2D clusters");
    if (!rc && !ie_h.empty())
        rc = hip_check(hipMemcpyAsync(ie.ptr, ie_h.data(), ie_h.size() * 8, hipMemcpyHostToDevice, st), "H2D clusters");
    if (!rc && !ee_h.empty())
        rc = hip_check(hipMemcpyAsync(ee.ptr, ee_h.data(), ee_h.size() * 8, hipMemcpyHostToDevice, st), "H2D clusters");
    if (!rc) rc = hip_check(hipStreamSynchronize(st), "H2D clusters");
    if (rc) return rc;
    built = true;
    return STEINER_OK;
}

int RoundGraph::get(const VorParams &P, uint32_t grid, uint32_t block, uint32_t rounds, hipGraphExec_t *out) {
    std::vector<uint8_t> want(sizeof(VorParams) + 12);
    memcpy(want.data(), &P, sizeof(VorParams));
    const uint32_t shape[3] = {grid, block, rounds};
    memcpy(want.data() + sizeof(VorParams), shape, 12);
    if (!exec || want != key) {
        release();
        int rc = hip_check(build_round_graph(P, grid, block, rounds, &exec), "round graph");
        if (rc) return rc;
        key.swap(want);
    }
    *out = exec;
    return STEINER_OK;
}

size_t mst_scratch_bytes(uint32_t k, uint64_t m) {
    const size_t k4 = ((size_t)k * 4 + 255) & ~(size_t)255, m4 = ((size_t)m * 4 + 255) & ~(size_t)255;
    return 256 + 5 * k4 + 2 * m4;
}

int TailScratch::prepare(uint32_t n, uint32_t k, uint64_t m, bool own_mst, hipStream_t st) {
    int rc;
    if (own_mst && (rc = mst.ensure(mst_scratch_bytes(k, m)))) return rc;
    if ((rc = out.ensure((size_t)n * 12 + 16))) return rc;
    if ((rc = host.ensure(64))) return rc;
    const size_t mark_bytes = ((size_t)n + 3) / 4 * 4;
    if (mark_n != n || mark.bytes < mark_bytes) {
        if ((rc = mark.ensure(mark_bytes))) return rc;
        if ((rc = hip_check(launch_fill_u32(mark.as<uint32_t>(), mark_bytes / 4, 0u, st), "mark clear"))) return rc;
        mark_n = n;
    }
    for (hipEvent_t &e : ev)
        if (!e && (rc = hip_check(hipEventCreate(&e), "hipEventCreate"))) return rc;
    return STEINER_OK;
}

void TailScratch::release() {
    mst.release();
    mark.release();
    out.release();
    host.release();
    for (hipEvent_t &e : ev)
        if (e) {
            (void)hipEventDestroy(e);
            e = nullptr;
        }
    mark_n = 0;
}

int launch_tree(const steiner_graph *g, hipStream_t st, const uint64_t *key, uint32_t *pred, uint32_t k,
                const uint64_t *pt, const uint32_t *tr, const uint32_t *g1_idx, uint32_t m, bool pred_ready,
                const TreeBufs &tb, hipEvent_t ev_mid) {
    const uint32_t n = g->n;
    const size_t k4 = ((size_t)k * 4 + 255) & ~(size_t)255, m4 = ((size_t)m * 4 + 255) & ~(size_t)255;
    uint8_t *base = tb.mst;
    MstParams M{};
    M.pt = pt;
    M.tr = tr;
    M.k = k;
    M.hdr = (uint32_t *)base;
    M.par = (uint32_t *)(base + 256);
    M.hook = (uint32_t *)(base + 256 + k4);
    M.sel = (uint32_t *)(base + 256 + 2 * k4);
    M.best = (unsigned long long *)(base + 256 + 3 * k4);
    M.edges[0] = (uint32_t *)(base + 256 + 5 * k4);
    M.edges[1] = (uint32_t *)(base + 256 + 5 * k4 + m4);
    M.block = tb.mst_block;
    ExpandParams EP{};
    EP.g = g->dg;
    EP.key = key;
    EP.pred = pred;
    EP.sel_e = M.sel;
    EP.nsel = M.hdr + 2;
    EP.nsel_max = k - 1;
    EP.mark = tb.mark;
    EP.oa = tb.out;
    EP.ob = EP.oa + n;
    EP.ow = EP.oa + 2 * (size_t)n;
    EP.ocnt = M.hdr + 3;
    EP.pred_ready = pred_ready ? 1u : 0u;
    const uint32_t emit_grid = (uint32_t)std::max<uint64_t>(
        1, std::min<uint64_t>((uint64_t)std::max(1, g->cu_count) * 8, (((uint64_t)n + 3) / 4 + 255) / 256));
    // Step 3 (MST of G'1), Step 4 (its kept cross-cell edges), Steps 5-6 (pred walks)
    int rc = hip_check(launch_mst(M, g1_idx, m, st), "mst");
    if (!rc && ev_mid) rc = hip_check(hipEventRecord(ev_mid, st), "event");
    if (!rc) rc = hip_check(launch_expand(EP, emit_grid, st), "expand");
    return rc;
}

int tree_from_g1(steiner_graph *g, hipStream_t st, const uint64_t *key, uint32_t *pred, uint32_t k,
                 const uint64_t *pt, const uint32_t *tr, const uint32_t *g1_idx, uint32_t m, bool pred_ready,
                 TailScratch &ts, uint8_t *mst_buf, std::unique_ptr<steiner_result> &out, double *ms_mst,
                 double *ms_expand, uint32_t mst_block) {
    const uint32_t n = g->n;
    int rc;
    if ((rc = ts.prepare(n, k, m, mst_buf == nullptr, st))) return rc;
    TreeBufs tb{mst_buf ? mst_buf : ts.mst.as<uint8_t>(), ts.mark.as<uint32_t>(), ts.out.as<uint32_t>(), mst_block};
    const uint32_t *hdr = (const uint32_t *)tb.mst;
    const bool timed = ms_mst || ms_expand;
    rc = timed ? hip_check(hipEventRecord(ts.ev[0], st), "event") : STEINER_OK;
    if (!rc) rc = launch_tree(g, st, key, pred, k, pt, tr, g1_idx, m, pred_ready, tb, timed ? ts.ev[1] : nullptr);
    if (!rc && timed) rc = hip_check(hipEventRecord(ts.ev[2], st), "event");
    uint32_t *h = ts.host.as<uint32_t>();
    if (!rc) rc = hip_check(hipMemcpyAsync(h, hdr, 16, hipMemcpyDeviceToHost, st), "D2H counts");
    if (!rc) rc = hip_check(hipStreamSynchronize(st), "tail sync");
    if (rc) {
        ts.mark_n = 0;  // the marks may be left set
        return rc;
    }
    const uint32_t nsel = h[2], m_out = h[3];
    if (nsel < k - 1) return fail(STEINER_EDISCONNECTED, "seeds are not connected");
    if (nsel > k - 1 || m_out > n) {
        ts.mark_n = 0;
        return fail(STEINER_EDEVICE, "tree expansion overflow (%u MST edges, %u tree edges)", nsel, m_out);
    }
    if (timed) {
        float t_mst = 0.f, t_exp = 0.f;
        (void)hipEventElapsedTime(&t_mst, ts.ev[0], ts.ev[1]);
        (void)hipEventElapsedTime(&t_exp, ts.ev[1], ts.ev[2]);
        if (ms_mst) *ms_mst += t_mst;
        if (ms_expand) *ms_expand += t_exp;
    }
    // the edge arrays into pinned memory, one synchronisation
    if ((rc = ts.host.ensure(((size_t)m_out * 3 + 16) * 4))) return rc;
    uint32_t *ha = ts.host.as<uint32_t>() + 16, *hb = ha + m_out, *hw = hb + m_out;
    rc = hip_check(hipMemcpyAsync(ha, tb.out, (size_t)m_out * 4, hipMemcpyDeviceToHost, st), "D2H edges");
    if (!rc) rc = hip_check(hipMemcpyAsync(hb, tb.out + n, (size_t)m_out * 4, hipMemcpyDeviceToHost, st), "D2H edges");
    if (!rc) rc = hip_check(hipMemcpyAsync(hw, tb.out + 2 * (size_t)n, (size_t)m_out * 4, hipMemcpyDeviceToHost, st),
                            "D2H edges");
    if (!rc) rc = hip_check(hipStreamSynchronize(st), "D2H edges");
    if (rc) return rc;
    // Step 7: canonical order (a, b, w) and D.  A tree has one edge per vertex
    // pair, so (a, b) decides the order: LSD radix sort of (a << 32 | b), w
    // riding along, 11-bit digits within each half, constant digits skipped.
    std::unique_ptr<steiner_result> res(new steiner_result());
    std::vector<uint64_t> ek(m_out), ek2(m_out);
    std::vector<uint32_t> val(hw, hw + m_out), val2(m_out);
    for (uint32_t t = 0; t < m_out; t++) ek[t] = ((uint64_t)ha[t] << 32) | hb[t];
    std::vector<uint32_t> hist(2048);
    for (uint32_t pass = 0; pass < 6 && m_out > 1; pass++) {
        const uint32_t shift = (pass / 3) * 32 + (pass % 3) * 11;
        const uint32_t width = pass % 3 == 2 ? 10 : 11;
        const uint64_t mask = (1ull << width) - 1;
        std::fill(hist.begin(), hist.end(), 0u);
        for (uint32_t t = 0; t < m_out; t++) hist[(ek[t] >> shift) & mask]++;
        if (hist[(ek[0] >> shift) & mask] == m_out) continue;  // one digit value: already in order
        uint32_t sum = 0;
        for (uint32_t &h : hist) {
            const uint32_t c = h;
            h = sum;
            sum += c;
        }
        for (uint32_t t = 0; t < m_out; t++) {
            const uint32_t at = hist[(ek[t] >> shift) & mask]++;
            ek2[at] = ek[t];
            val2[at] = val[t];
        }
        ek.swap(ek2);
        val.swap(val2);
    }
    res->a.resize(m_out);
    res->b.resize(m_out);
    res->w.resize(m_out);
    uint64_t D = 0;
    for (uint32_t t = 0; t < m_out; t++) {
        res->a[t] = (uint32_t)(ek[t] >> 32);
        res->b[t] = (uint32_t)ek[t];
        res->w[t] = val[t];
        D += val[t];
    }
    res->total = D;
    res->stats.tree_edges = m_out;
    out = std::move(res);
    return STEINER_OK;
}

int run_pass(steiner_graph *g, const Options &o, std::vector<Query> &qs) {
    const auto t_start = std::chrono::steady_clock::now();
    hipStream_t st = g->stream;
    Workspace &ws = g->ws;
    const uint32_t n = g->n;
    int rc;

    // Queries that need the device: status OK and at least two seeds.
    std::vector<uint32_t> act;
    for (uint32_t i = 0; i < qs.size(); i++) {
        if (qs[i].status) continue;
        if (qs[i].S.size() < 2) {  // k == 1: empty tree, D = 0
            qs[i].result.reset(new steiner_result());
            continue;
        }
        act.push_back(i);
    }
    const uint32_t Q = (uint32_t)act.size();
    if (Q == 0) return STEINER_OK;

    // ---------------------------------------------------------- allocation
    // a vertex is listed at most once per round as a light item and once as a heavy item
    const uint64_t cap_s = 2ull * Q * n + 64;
    const uint64_t cap_b = 2ull * Q * big_row_chunks(g, o.small_max, o.chunk) + 64;
    if (cap_s >= (1ull << 32) || cap_b >= (1ull << 32))
        return fail(STEINER_ENOMEM, "batch too large for 32-bit frontier counters");
    std::vector<uint64_t> pt_off(Q + 1, 0), oc_off(Q + 1, 0), sd_off(Q + 1, 0);
    uint64_t half = g->nnz / 2 + 1;
    for (uint32_t s = 0; s < Q; s++) {
        const uint64_t k = qs[act[s]].S.size();
        const uint64_t P = k * (k - 1) / 2;
        pt_off[s + 1] = pt_off[s] + P;
        oc_off[s + 1] = oc_off[s] + std::min(P, half);
        sd_off[s + 1] = sd_off[s] + k;
    }
    const Layout L(Q);
    const size_t QN = (size_t)Q * n;
    if ((rc = ws.key.ensure(QN * 8)) || (rc = ws.aux.ensure(QN * 4)) || (rc = ws.dirty.ensure(QN)) ||
        (rc = ws.settled.ensure(QN)) ||
        (rc = ws.items_s[0].ensure(cap_s * 8)) || (rc = ws.items_s[1].ensure(cap_s * 8)) ||
        (rc = ws.items_b[0].ensure(cap_b * 8)) || (rc = ws.items_b[1].ensure(cap_b * 8)) ||
        (rc = ws.ctl.ensure(L.total)) || (rc = ws.heavy_pe.ensure((size_t)Q * g->nheavy * 4 + 4)) ||
        (rc = ws.seeds.ensure(sd_off[Q] * 12 + 4)) || (rc = ws.pt.ensure(pt_off[Q] * 8)) ||
        (rc = ws.cidx.ensure(oc_off[Q] * 4)) || (rc = ws.cval.ensure(oc_off[Q] * 8)) ||
        (rc = ws.host.ensure(std::max<size_t>(L.total, sd_off[Q] * 12) + 4096)))
        return rc;
    // seeds of every slot, then their table ranks and the inverse (renumbered graphs), concatenated
    const bool ranked = g->reordered;
    uint32_t *d_tr = ws.seeds.as<uint32_t>() + sd_off[Q], *d_ts = d_tr + sd_off[Q];
    uint8_t *ctl = ws.ctl.as<uint8_t>();
    uint8_t *hctl = ws.host.as<uint8_t>();

    VorParams P{};
    bind_pass(P, g->dg, ctl, L, Q);
    P.key = ws.key.as<uint64_t>();
    P.aux = ws.aux.as<uint32_t>();
    P.dirty = ws.dirty.as<uint8_t>();
    P.settled = ws.settled.as<uint8_t>();
    P.items_s[0] = ws.items_s[0].as<uint64_t>();
    P.items_s[1] = ws.items_s[1].as<uint64_t>();
    P.items_b[0] = ws.items_b[0].as<uint64_t>();
    P.items_b[1] = ws.items_b[1].as<uint64_t>();
    bind_state(P, o, cap_s, cap_b);
    if ((rc = bind_chunk_memory(P, g, o, Q, ws.xkey))) return rc;

    // Per-slot pointer tables (host image, then one copy).
    {
        uint64_t *h_ptr = (uint64_t *)(hctl + L.pt_ptr);
        uint64_t *h_len = (uint64_t *)(hctl + L.pt_len);
        uint64_t *h_oi = (uint64_t *)(hctl + L.oidx_ptr);
        uint64_t *h_ov = (uint64_t *)(hctl + L.oval_ptr);
        uint64_t *h_oc = (uint64_t *)(hctl + L.ocap);
        uint64_t *h_tr = (uint64_t *)(hctl + L.tr_ptr);
        uint64_t *h_ts = (uint64_t *)(hctl + L.ts_ptr);
        uint32_t *h_ids = (uint32_t *)(hctl + L.slot_ids);
        for (uint32_t s = 0; s < Q; s++) {
            h_tr[s] = (uint64_t)(uintptr_t)(d_tr + sd_off[s]);
            h_ts[s] = (uint64_t)(uintptr_t)(d_ts + sd_off[s]);
            h_ptr[s] = (uint64_t)(uintptr_t)(ws.pt.as<uint64_t>() + pt_off[s]);
            h_len[s] = pt_off[s + 1] - pt_off[s];
            h_oi[s] = (uint64_t)(uintptr_t)(ws.cidx.as<uint32_t>() + oc_off[s]);
            h_ov[s] = (uint64_t)(uintptr_t)(ws.cval.as<uint64_t>() + oc_off[s]);
            h_oc[s] = oc_off[s + 1] - oc_off[s];
            h_ids[s] = s;
        }
        memset(hctl + L.slot_err, 0, 4ull * Q);
        memset(hctl + L.out_cnt, 0, 4ull * Q);
        if ((rc = hip_check(hipMemcpyAsync(ctl + L.pt_ptr, hctl + L.pt_ptr, L.far_min - L.pt_ptr, hipMemcpyHostToDevice, st),
                            "H2D tables")))
            return rc;
        if ((rc = hip_check(hipMemcpyAsync(ctl + L.slot_err, hctl + L.slot_err, L.total - L.slot_err,
                                           hipMemcpyHostToDevice, st), "H2D tables")))
            return rc;
        if ((rc = hip_check(hipStreamSynchronize(st), "tables"))) return rc;
    }
    // Seeds of every slot, concatenated (then the ranks).
    {
        uint32_t *hs = ws.host.as<uint32_t>();
        std::vector<uint32_t> rk;
        for (uint32_t s = 0; s < Q; s++) {
            const std::vector<uint32_t> &S = qs[act[s]].S;
            memcpy(hs + sd_off[s], S.data(), S.size() * 4);
            if (ranked) {
                seed_ranks(g, S, rk);
                memcpy(hs + sd_off[Q] + sd_off[s], rk.data(), S.size() * 4);
                memcpy(hs + 2 * sd_off[Q] + sd_off[s], rk.data() + S.size(), S.size() * 4);
            }
        }
        if ((rc = hip_check(hipMemcpyAsync(ws.seeds.ptr, hs, sd_off[Q] * (ranked ? 12 : 4), hipMemcpyHostToDevice, st),
                            "H2D seeds")))
            return rc;
        if ((rc = hip_check(hipStreamSynchronize(st), "seeds"))) return rc;
    }

    Timer tm(o.timing, st);
    tm.mark();  // 0
    if ((rc = hip_check(launch_pass_reset(P, st), "pass reset"))) return rc;
    if ((rc = hip_check(launch_fill_u64(ws.pt.as<uint64_t>(), pt_off[Q], KEY_INF, st), "pair table init"))) return rc;
    for (uint32_t s = 0; s < Q; s++) {
        rc = hip_check(launch_slot_start(P, s, ws.seeds.as<uint32_t>() + sd_off[s], (uint32_t)qs[act[s]].S.size(),
                                         ws.heavy_pe.as<uint32_t>() + (size_t)s * g->nheavy, g->nheavy, st),
                       "slot start");
        if (rc) return rc;
    }
    tm.mark();  // 1

    // ------------------------------------------------- Step 1: Voronoi cells
    PassCtl *hpass = (PassCtl *)(hctl + L.pass);
    // event pairs around each chunk of relaxation launches (timing mode only);
    // the gaps between the launches of a chunk count as kernel time
    size_t nkev = 0;
    auto kmark = [&]() {
        if (!o.timing) return;
        if (nkev == ws.events.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return;
            ws.events.push_back(e);
        }
        (void)hipEventRecord(ws.events[nkev++], st);
    };
    uint32_t relax_launches = 0;
    const uint32_t round_cap = 1u << 26;
    const uint32_t rounds_per_launch = 4096;
    const double wall_cap_s = 120.0;
    auto wall = [&]() {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    };
    // cluster-local relaxation (one query): rounds over clusters instead of frontier lists
    const bool clustered = o.driver == 3 && Q == 1;
    uint32_t cluster_rounds = 0;
    if (clustered) {
        ClusterSet &cs = g->clusters;
        if ((rc = cs.build(g))) return rc;
        ClusterParams C{};
        C.n = n;
        C.nclusters = cs.nclusters;
        C.members = cs.members.as<uint32_t>();
        C.cstart = cs.cstart.as<uint32_t>();
        C.cl_of = cs.cl_of.as<uint32_t>();
        C.irp = cs.irp.as<uint32_t>();
        C.ie = cs.ie.as<uint2>();
        C.erp = cs.erp.as<uint32_t>();
        C.ee = cs.ee.as<uint2>();
        C.key = P.key;
        C.expanded = cs.expanded.as<uint64_t>();
        C.list[0] = cs.lists.as<uint32_t>();
        C.list[1] = cs.lists.as<uint32_t>() + cs.nclusters;
        C.stamp = cs.stamp.as<uint32_t>();
        C.ctl = cs.ctl.as<ClusterCtl>();
        rc = hip_check(launch_fill_u64(C.expanded, n, KEY_INF, st), "cluster reset");
        if (!rc) rc = hip_check(launch_fill_u32(C.stamp, cs.nclusters, 0u, st), "cluster reset");
        if (!rc) rc = hip_check(launch_fill_u32((uint32_t *)C.ctl, sizeof(ClusterCtl) / 4, 0u, st), "cluster reset");
        if (!rc) rc = hip_check(launch_cluster_start(C, ws.seeds.as<uint32_t>(), (uint32_t)qs[act[0]].S.size(), st),
                                "cluster start");
        if (rc) return rc;
        const uint32_t cgrid = (uint32_t)std::max(1, cluster_max_grid());
        ClusterCtl *hc = (ClusterCtl *)(hctl + L.pass);  // pinned scratch; the frontier pass control is unused here
        // the previous pass's rounds plus the deciding round and one spare, then small growing chunks
        uint32_t chunk_rounds = std::min<uint32_t>(std::max<uint32_t>(g->last_rounds + 2, 4), 256), launched = 0;
        uint32_t next_chunk = 4;
        for (;;) {
            kmark();
            for (uint32_t i = 0; i < chunk_rounds; i++) {
                rc = hip_check(launch_cluster_round(C, cgrid, st), "cluster round");
                relax_launches++;
                if (rc) return rc;
            }
            kmark();
            launched += chunk_rounds;
            if ((rc = hip_check(hipMemcpyAsync(hc, C.ctl, sizeof(ClusterCtl), hipMemcpyDeviceToHost, st), "D2H clusters")))
                return rc;
            if ((rc = hip_check(hipStreamSynchronize(st), "cluster sync"))) return rc;
            if (hc->err) return fail(STEINER_EDEVICE, "cluster list overflow");
            if (hc->done) break;
            if (launched >= round_cap || wall() > wall_cap_s)
                return fail(STEINER_EDEVICE, "relaxation did not converge (%u rounds)", hc->round);
            chunk_rounds = next_chunk;
            next_chunk = std::min<uint32_t>(next_chunk * 2, 64);
        }
        cluster_rounds = hc->round;
        hpass->round = 0;  // the frontier pass did not run
    }
    bool persistent = !clustered && o.driver == 2 && Q <= 256;
    uint32_t pgrid = 0;
    if (persistent) {
        int mg = persistent_max_grid(o.block);
        pgrid = std::min<uint32_t>(o.grid, (uint32_t)std::max(mg, 0));
        if (pgrid == 0) persistent = false;
    }
    if (persistent) {
        for (;;) {
            kmark();
            rc = hip_check(launch_persistent(P, pgrid, o.block, rounds_per_launch, st), "persistent pass");
            kmark();
            relax_launches++;
            if (rc) return rc;
            if ((rc = hip_check(hipMemcpyAsync(hpass, P.pass, sizeof(PassCtl), hipMemcpyDeviceToHost, st), "D2H pass")))
                return rc;
            if ((rc = hip_check(hipStreamSynchronize(st), "persistent sync"))) return rc;
            if (hpass->err & (ERR_LIST_OVERFLOW | ERR_BARRIER_TIMEOUT))
                return fail(STEINER_EDEVICE, "relaxation pass failed (err bits 0x%x)", hpass->err);
            if (hpass->all_done) break;
            if (hpass->round >= round_cap || wall() > wall_cap_s)
                return fail(STEINER_EDEVICE, "relaxation did not converge (%u rounds)", hpass->round);
        }
    } else if (!clustered) {
        // the previous pass's rounds plus the deciding round and one spare, then small growing chunks
        uint32_t chunk_rounds = std::min<uint32_t>(std::max<uint32_t>(g->last_rounds + 2, 4), 256), launched = 0;
        uint32_t next_chunk = 4;
        // a batch's frontier is larger: at least half the resident workgroups
        const uint32_t grid = Q == 1 ? o.grid_tuned : std::max(o.grid_tuned, o.grid / 2);
        // graph-captured driver: the chunk is whole replays of one graph of GRAPH_ROUNDS launches
        hipGraphExec_t gexec = nullptr;
        if (o.driver == 4 && (rc = ws.rgraph.get(P, grid, o.block, GRAPH_ROUNDS, &gexec))) return rc;
        for (;;) {
            kmark();
            if (gexec) {
                const uint32_t reps = (chunk_rounds + GRAPH_ROUNDS - 1) / GRAPH_ROUNDS;
                for (uint32_t i = 0; i < reps; i++) {
                    rc = hip_check(hipGraphLaunch(gexec, st), "round graph launch");
                    relax_launches += GRAPH_ROUNDS;
                    if (rc) return rc;
                }
                chunk_rounds = reps * GRAPH_ROUNDS;
            } else {
                for (uint32_t i = 0; i < chunk_rounds; i++) {
                    rc = hip_check(launch_round(P, grid, o.block, st), "round");
                    relax_launches++;
                    if (rc) return rc;
                }
            }
            kmark();
            launched += chunk_rounds;
            if ((rc = hip_check(hipMemcpyAsync(hpass, P.pass, sizeof(PassCtl), hipMemcpyDeviceToHost, st), "D2H pass")))
                return rc;
            if ((rc = hip_check(hipStreamSynchronize(st), "round sync"))) return rc;
            if (hpass->err & ERR_LIST_OVERFLOW) return fail(STEINER_EDEVICE, "frontier overflow");
            if (hpass->all_done) break;
            if (launched >= round_cap || wall() > wall_cap_s)
                return fail(STEINER_EDEVICE, "relaxation did not converge (%u rounds)", hpass->round);
            chunk_rounds = next_chunk;
            next_chunk = std::min<uint32_t>(next_chunk * 2, 64);
        }
    }
    const uint32_t rounds = clustered ? cluster_rounds : hpass->round;
    g->last_rounds = rounds;
    double ms_relax = 0.0;
    for (size_t i = 0; i + 1 < nkev; i += 2) {
        float m = 0.f;
        (void)hipEventSynchronize(ws.events[i + 1]);
        if (hipEventElapsedTime(&m, ws.events[i], ws.events[i + 1]) == hipSuccess) ms_relax += m;
    }
    tm.mark();  // 2

    // ------------------------------ canonical pred + Step 2 boundary scan
    ScanParams SP{};
    SP.g = g->dg;
    SP.key = P.key;
    SP.aux = P.aux;
    SP.heavy_pe = ws.heavy_pe.as<uint32_t>();
    SP.pt = (uint64_t *const *)(ctl + L.pt_ptr);
    SP.tr = ranked ? (const uint32_t *const *)(ctl + L.tr_ptr) : nullptr;
    SP.slot_ids = (const uint32_t *)(ctl + L.slot_ids);
    SP.nscan = Q;
    SP.slot_err = (uint32_t *)(ctl + L.slot_err);
    SP.with_pred = o.lazy_pred ? 0 : 1;
    SP.ev = o.counting ? P.cnt->scan_ev : nullptr;
    for (uint32_t a : act)
        if (qs[a].want_key) SP.with_pred = 1;
    const uint32_t sgrid = (uint32_t)std::max(1, g->cu_count) * 8;
    if ((rc = hip_check(launch_scan(SP, sgrid, 256, st), "scan"))) return rc;
    tm.mark();  // 3

    // ------------------------------------------------- G'1 compaction
    CompactParams CP{};
    CP.pt = SP.pt;
    CP.ts = ranked ? (const uint32_t *const *)(ctl + L.ts_ptr) : nullptr;
    CP.pt_len = (const uint64_t *)(ctl + L.pt_len);
    CP.out_idx = (uint32_t *const *)(ctl + L.oidx_ptr);
    CP.out_val = (uint64_t *const *)(ctl + L.oval_ptr);
    CP.out_cap = (const uint64_t *)(ctl + L.ocap);
    CP.out_cnt = (uint32_t *)(ctl + L.out_cnt);
    CP.slot_ids = SP.slot_ids;
    CP.nscan = Q;
    CP.pass = P.pass;
    if ((rc = hip_check(launch_compact(CP, sgrid, 256, st), "compact"))) return rc;
    tm.mark();  // 4
    // errors, counts, per-slot advances
    if ((rc = hip_check(hipMemcpyAsync(hctl + L.advances, ctl + L.advances, L.total - L.advances, hipMemcpyDeviceToHost, st),
                        "D2H counts")))
        return rc;
    if ((rc = hip_check(hipMemcpyAsync(hpass, P.pass, sizeof(PassCtl), hipMemcpyDeviceToHost, st), "D2H pass"))) return rc;
    Counters hcnt{};
    if (o.counting &&
        (rc = hip_check(hipMemcpyAsync(&hcnt, P.cnt, sizeof(Counters), hipMemcpyDeviceToHost, st), "D2H counters")))
        return rc;
    if ((rc = hip_check(hipStreamSynchronize(st), "compact sync"))) return rc;
    if (hpass->err & ERR_LIST_OVERFLOW) return fail(STEINER_EDEVICE, "compaction overflow");
    const uint32_t *h_err = (const uint32_t *)(hctl + L.slot_err);
    const uint32_t *h_cnt = (const uint32_t *)(hctl + L.out_cnt);
    const uint32_t *h_adv = (const uint32_t *)(hctl + L.advances);
    std::vector<uint32_t> slot_err(h_err, h_err + Q), out_cnt(h_cnt, h_cnt + Q), slot_adv(h_adv, h_adv + Q);

    // debug: key / pred of the single slot, indexed and valued by caller ids
    for (uint32_t s = 0; s < Q; s++) {
        Query &qq = qs[act[s]];
        if (qq.want_key && !slot_err[s]) {
            std::vector<uint64_t> ik;
            std::vector<uint32_t> ip;
            if (g->reordered) {
                ik.resize(n);
                ip.resize(n);
            }
            uint64_t *kd = g->reordered ? ik.data() : qq.want_key;
            uint32_t *pd = g->reordered ? ip.data() : qq.want_pred;
            rc = hip_check(hipMemcpyAsync(kd, P.key + (size_t)s * n, (size_t)n * 8, hipMemcpyDeviceToHost, st), "D2H key");
            if (!rc) rc = hip_check(hipMemcpyAsync(pd, P.aux + (size_t)s * n, (size_t)n * 4, hipMemcpyDeviceToHost, st), "D2H pred");
            if (!rc) rc = hip_check(hipStreamSynchronize(st), "D2H");
            if (rc) return rc;
            if (g->reordered) {
                for (uint32_t v = 0; v < n; v++) {
                    const uint32_t i = g->h_inv[v], p = ip[i];
                    qq.want_key[v] = ik[i];
                    qq.want_pred[v] = p < n ? g->h_perm[p] : p;
                }
            }
        }
    }

    // ---------------------------------------- Steps 3-7 per query
    double ms_mst = 0.0, ms_expand = 0.0;
    for (uint32_t s = 0; s < Q; s++) {
        Query &qq = qs[act[s]];
        const uint32_t k = (uint32_t)qq.S.size();
        if (slot_err[s] & (ERR_DIST_OVERFLOW | ERR_SUM_OVERFLOW)) {
            qq.status = fail(STEINER_EOVERFLOW, "distance or cross-cell sum does not fit in 32 bits");
            continue;
        }
        if (qq.stop_after == STOP_AFTER_SCAN) continue;
        const uint32_t m = out_cnt[s];
        if (qq.stop_after == STOP_AFTER_COMPACT) {
            qq.pidx.resize(m);
            qq.pval.resize(m);
            if (m) {
                rc = hip_check(hipMemcpyAsync(qq.pidx.data(), ws.cidx.as<uint32_t>() + oc_off[s], (size_t)m * 4,
                                              hipMemcpyDeviceToHost, st), "D2H G'1");
                if (!rc) rc = hip_check(hipMemcpyAsync(qq.pval.data(), ws.cval.as<uint64_t>() + oc_off[s], (size_t)m * 8,
                                                       hipMemcpyDeviceToHost, st), "D2H G'1");
                if (!rc) rc = hip_check(hipStreamSynchronize(st), "D2H G'1");
                if (rc) return rc;
            }
            continue;
        }
        int trc = tree_from_g1(g, st, P.key + (size_t)s * n, P.aux + (size_t)s * n, k, ws.pt.as<uint64_t>() + pt_off[s],
                               ranked ? d_tr + sd_off[s] : nullptr,
                               ws.cidx.as<uint32_t>() + oc_off[s], m, SP.with_pred != 0, ws.tail, nullptr, qq.result,
                               o.timing ? &ms_mst : nullptr, o.timing ? &ms_expand : nullptr);
        if (trc == STEINER_EDISCONNECTED) {
            qq.status = trc;
            continue;
        }
        if (trc) return trc;
        steiner_stats &x = qq.result->stats;
        x.rounds = rounds;
        x.advances = slot_adv[s];
        x.pairs = m;
    }
    const auto t_end = std::chrono::steady_clock::now();
    const double ms_total = std::chrono::duration<double, std::milli>(t_end - t_start).count();
    for (uint32_t s = 0; s < Q; s++) {
        Query &qq = qs[act[s]];
        if (!qq.result) continue;
        steiner_stats &x = qq.result->stats;
        x.ms_init = tm.ms(0, 1);
        x.ms_voronoi = tm.ms(1, 2);
        x.ms_scan = tm.ms(2, 3);
        x.ms_compact = tm.ms(3, 4);
        x.ms_mst = ms_mst;
        x.ms_expand = ms_expand;
        x.ms_total = ms_total;
        x.ms_relax_kernels = ms_relax;
        x.relax_launches = relax_launches;
        x.relax_attempts = hcnt.ev[EV_ATTEMPT];
        x.relax_atomics = hcnt.ev[EV_ATOMIC];
        x.relax_improved = hcnt.ev[EV_IMPROVED];
        x.pushes_local = hcnt.ev[EV_LOCAL];
        x.pushes_next = hcnt.ev[EV_GLOBAL];
        x.parked = hcnt.ev[EV_PARK];
        x.items = hcnt.ev[EV_ITEMS];
        x.relax_attempts_large = hcnt.ev[EV_LARGE];
        x.scan_entries = hcnt.scan_ev[SCAN_EV_ENTRIES];
        x.scan_gathers = hcnt.scan_ev[SCAN_EV_GATHERS];
        x.scan_candidates = hcnt.scan_ev[SCAN_EV_CANDIDATES];
        x.scan_atomics = hcnt.scan_ev[SCAN_EV_ATOMICS];
    }
    return STEINER_OK;
}

}  // namespace stn
