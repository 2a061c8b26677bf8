// Continuous-batching Steiner query server over one resident graph.
//
// One multi-query relaxation pass runs for the server's lifetime.  Between
// short chunks of rounds the scheduler thread admits waiting requests into
// free slots (a slot is the per-query vertex state: key, stamp/pred and park
// byte and settled byte, 14 bytes per vertex) when the request's device bytes fit the memory
// budget; a new query's seeds join the pass at the next round, so queries at
// different bucket depths share every relaxation launch.  A query whose cells
// have converged is handed to the tail thread, which runs its boundary scan,
// G'1 compaction, MST, pruning and expansion on a second stream while the
// pass keeps relaxing the other queries, then frees the slot.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <thread>
#include <unordered_map>

#include "engine.h"

using namespace stn;

namespace {

struct Request {
    uint64_t ticket = 0;
    std::vector<uint32_t> S;
    std::vector<uint32_t> rk;  // pair-table ranks of the seeds and their inverse (empty: identity)
    int status = STEINER_OK;
    bool done = false;
    int slot = -1;
    uint64_t pool_off = 0, pool_bytes = 0, charge = 0;
    uint64_t pt_len = 0, oc_cap = 0;
    std::unique_ptr<steiner_result> result;
    std::chrono::steady_clock::time_point t_submit;
};

enum SlotState { SLOT_FREE = 0, SLOT_ACTIVE = 1, SLOT_TAIL = 2 };

// First-fit allocator over a device pool (host-side bookkeeping only).
struct PoolAlloc {
    std::map<uint64_t, uint64_t> free_;  // offset -> bytes
    void init(uint64_t bytes) {
        free_.clear();
        free_[0] = bytes;
    }
    bool alloc(uint64_t bytes, uint64_t *off) {
        bytes = (bytes + 255) & ~255ull;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const uint64_t rest = it->second - bytes, at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes) {
        bytes = (bytes + 255) & ~255ull;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

__global__ void k_set_slot_tables(uint64_t *pt_ptr, uint64_t *pt_len, uint64_t *oidx, uint64_t *oval, uint64_t *ocap,
                                  uint64_t *tr_ptr, uint64_t *ts_ptr, uint32_t *slot_err, uint32_t *out_cnt,
                                  uint32_t slot, uint64_t pt, uint64_t len, uint64_t oi, uint64_t ov, uint64_t cap,
                                  uint64_t tr, uint64_t ts) {
    pt_ptr[slot] = pt;
    tr_ptr[slot] = tr;
    ts_ptr[slot] = ts;
    pt_len[slot] = len;
    oidx[slot] = oi;
    oval[slot] = ov;
    ocap[slot] = cap;
    slot_err[slot] = 0;
    out_cnt[slot] = 0;
}

// Starts the pass at round r (a long-lived pass runs through the wrap of the round numbers).
__global__ void k_set_round(PassCtl *pass, uint32_t r) {
    pass->round = r;
    pass->word = pass_word(r, 0, 1, NO_LAUNCH);
}

__global__ void k_iota(uint32_t *p, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = i;
}

}  // namespace

struct steiner_server {
    steiner_graph *g = nullptr;
    Options o{};
    // Device memory: fixed_bytes (control region, tail output and marks, list headroom) + S * slot_bytes
    // (per-slot vertex state and frontier lists) + the pool (per-request regions) = budget.
    uint64_t budget = 0, fixed_bytes = 0, slot_bytes = 0, pool_bytes = 0, used = 0;
    uint32_t S = 0;  // slots
    uint32_t round_base = 0;  // the pass's first round (0 unless STEINER_SERVER_ROUND_BASE says otherwise)
    hipStream_t s_main = nullptr, s_tail = nullptr;
    DevBuf key, aux, dirty, settled, items_s[2], items_b[2], ctl, heavy_pe, pool, xkey;
    TailScratch tail;
    RoundGraph rgraph;  // the graph-captured driver's chunk of rounds
    HostPinned hbuf;
    Layout L{1};
    VorParams P{};
    PoolAlloc pa;
    uint64_t half = 0;

    std::mutex mu;
    std::condition_variable cv_sched, cv_done, cv_tail;
    std::deque<Request *> pending;
    std::unordered_map<uint64_t, Request *> reqs;
    std::vector<Request *> slot_req;
    std::vector<int> slot_state;
    std::deque<int> tail_q;
    uint64_t next_ticket = 1;
    uint32_t waiters = 0;  // threads inside steiner_server_wait (destroy waits for them to leave)
    bool stopping = false;
    int fatal = STEINER_OK;
    std::thread sched, tailer;

    // A request's pool region: pair table (8 B per pair), G'1 pair indices (4 B per entry, at most one per
    // pair and one per edge), the MST's scratch over that G'1, then its seeds, their table ranks and the
    // inverse ranks (k entries each).
    static uint64_t al(uint64_t b) { return (b + 255) & ~255ull; }
    uint64_t g1_cap(uint32_t k) const { return std::min<uint64_t>((uint64_t)k * (k - 1) / 2, half); }
    uint64_t pool_need(uint32_t k) const {
        const uint64_t P_ = (uint64_t)k * (k - 1) / 2, oc = g1_cap(k);
        return al(8 * P_) + al(4 * oc) + al(mst_scratch_bytes(k, oc)) + al(12ull * k);
    }
    uint8_t *region(const Request *r, int part) const {  // 0 pair table, 1 G'1 indices, 2 MST, 3 seeds
        const uint64_t k = r->S.size(), P_ = k * (k - 1) / 2, oc = g1_cap((uint32_t)k);
        const uint64_t off[4] = {0, al(8 * P_), al(8 * P_) + al(4 * oc),
                                 al(8 * P_) + al(4 * oc) + al(mst_scratch_bytes((uint32_t)k, oc))};
        return pool.as<uint8_t>() + r->pool_off + off[part];
    }
    uint32_t *seeds_of(const Request *r) const { return (uint32_t *)region(r, 3); }

    void run_sched();
    void run_tail();
    int admit(Request *r, int slot);
    void free_device() {
        DevBuf *bufs[] = {&key, &aux, &dirty, &settled, &items_s[0], &items_s[1], &items_b[0], &items_b[1], &ctl,
                          &heavy_pe, &pool, &xkey};
        for (DevBuf *b : bufs) b->release();
        hbuf.release();
        tail.release();
        rgraph.release();
        if (s_main) (void)hipStreamDestroy(s_main);
        if (s_tail) (void)hipStreamDestroy(s_tail);
        s_main = s_tail = nullptr;
    }
};

// ---------------------------------------------------------------- helpers

static double ms_since(std::chrono::steady_clock::time_point t) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t).count();
}

int steiner_server::admit(Request *r, int slot) {
    const uint32_t k = (uint32_t)r->S.size();
    const uint64_t P_ = (uint64_t)k * (k - 1) / 2;
    const uint64_t oc = g1_cap(k);
    uint64_t *pt = (uint64_t *)region(r, 0);
    uint32_t *oi = (uint32_t *)region(r, 1);
    uint32_t *seeds = seeds_of(r);
    uint8_t *c = ctl.as<uint8_t>();
    int rc = hip_check(hipMemcpyAsync(seeds, r->S.data(), 4ull * k, hipMemcpyHostToDevice, s_main), "H2D seeds");
    if (!rc && !r->rk.empty())
        rc = hip_check(hipMemcpyAsync(seeds + k, r->rk.data(), 8ull * k, hipMemcpyHostToDevice, s_main), "H2D ranks");
    if (rc) return rc;
    const bool ranked = !r->rk.empty();
    hipLaunchKernelGGL(k_set_slot_tables, dim3(1), dim3(1), 0, s_main, (uint64_t *)(c + L.pt_ptr),
                       (uint64_t *)(c + L.pt_len), (uint64_t *)(c + L.oidx_ptr), (uint64_t *)(c + L.oval_ptr),
                       (uint64_t *)(c + L.ocap), (uint64_t *)(c + L.tr_ptr), (uint64_t *)(c + L.ts_ptr),
                       (uint32_t *)(c + L.slot_err), (uint32_t *)(c + L.out_cnt), (uint32_t)slot,
                       (uint64_t)(uintptr_t)pt, P_, (uint64_t)(uintptr_t)oi, 0ull, oc,
                       ranked ? (uint64_t)(uintptr_t)(seeds + k) : 0ull, ranked ? (uint64_t)(uintptr_t)(seeds + 2 * k) : 0ull);
    if ((rc = hip_check(hipGetLastError(), "slot tables"))) return rc;
    if ((rc = hip_check(launch_fill_u64(pt, P_, KEY_INF, s_main), "pair table"))) return rc;
    rc = hip_check(launch_slot_start(P, (uint32_t)slot, seeds, k, heavy_pe.as<uint32_t>() + (size_t)slot * g->nheavy,
                                     g->nheavy, s_main),
                   "slot start");
    r->pt_len = P_;
    r->oc_cap = oc;
    return rc;
}

void steiner_server::run_sched() {
    (void)hipSetDevice(g->device);
    uint8_t *hc = hbuf.as<uint8_t>();
    const uint32_t rounds_per_chunk = 4;
    // every launch with a query resident takes its round's decision and advances the round counter; a chunk
    // that leaves it unchanged, or a query resident for more rounds than any pass may take, means the pass
    // state is broken: every request then fails instead of the scheduler relaunching rounds for ever
    const uint32_t round_cap = 1u << 26;
    uint32_t round_seen = round_base;
    auto rounds_since = [](uint32_t now, uint32_t then) { return (now + ROUND_WRAP - then) % ROUND_WRAP; };
    std::vector<uint32_t> admitted_at(S, 0);
    std::unique_lock<std::mutex> lk(mu);
    while (!stopping) {
        // admission, first come first served
        while (!pending.empty() && !fatal) {
            Request *r = pending.front();
            int slot = -1;
            for (uint32_t s = 0; s < S; s++)
                if (slot_state[s] == SLOT_FREE) { slot = (int)s; break; }
            if (slot < 0) break;
            const uint64_t need = pool_need((uint32_t)r->S.size());
            if (used + need > pool_bytes) break;
            uint64_t off = 0;
            if (!pa.alloc(need, &off)) break;
            pending.pop_front();
            r->pool_off = off;
            r->pool_bytes = need;
            r->charge = need;
            r->slot = slot;
            used += need;
            slot_state[slot] = SLOT_ACTIVE;
            slot_req[slot] = r;
            admitted_at[slot] = round_seen;
            const int rc = admit(r, slot);
            if (rc) fatal = rc;
        }
        bool any_active = false;
        for (uint32_t s = 0; s < S; s++) any_active |= slot_state[s] == SLOT_ACTIVE;
        if (fatal) {
            for (uint32_t s = 0; s < S; s++)
                if (slot_state[s] == SLOT_ACTIVE) {
                    Request *r = slot_req[s];
                    slot_state[s] = SLOT_FREE;
                    slot_req[s] = nullptr;
                    used -= r->charge;
                    pa.release(r->pool_off, r->pool_bytes);
                    r->status = fatal;
                    r->done = true;
                }
            while (!pending.empty()) {
                Request *r = pending.front();
                pending.pop_front();
                r->status = fatal;
                r->done = true;
            }
            cv_done.notify_all();
            any_active = false;
        }
        if (!any_active) {
            cv_sched.wait(lk);
            continue;
        }
        lk.unlock();
        int rc = STEINER_OK;
        if (o.driver == 4) {  // the chunk as one captured graph
            hipGraphExec_t ge = nullptr;
            rc = rgraph.get(P, o.grid, o.block, rounds_per_chunk, &ge);
            if (!rc) rc = hip_check(hipGraphLaunch(ge, s_main), "round graph launch");
        } else {
            for (uint32_t i = 0; i < rounds_per_chunk && !rc; i++)
                rc = hip_check(launch_round(P, o.grid, o.block, s_main), "round");
        }
        if (!rc)
            rc = hip_check(hipMemcpyAsync(hc + L.pass, P.pass, sizeof(PassCtl), hipMemcpyDeviceToHost, s_main), "D2H pass");
        if (!rc)
            rc = hip_check(hipMemcpyAsync(hc + L.done, ctl.as<uint8_t>() + L.done, 4ull * S, hipMemcpyDeviceToHost, s_main),
                           "D2H done");
        if (!rc) rc = hip_check(hipStreamSynchronize(s_main), "chunk sync");
        lk.lock();
        const PassCtl *hpass = (const PassCtl *)(hc + L.pass);
        if (!rc && (hpass->err & ERR_LIST_OVERFLOW)) rc = fail(STEINER_EDEVICE, "frontier overflow");
        if (!rc && hpass->round == round_seen)
            rc = fail(STEINER_EDEVICE, "relaxation stalled at round %u", hpass->round);
        if (!rc) round_seen = hpass->round;
        for (uint32_t s = 0; s < S && !rc; s++)
            if (slot_state[s] == SLOT_ACTIVE && rounds_since(round_seen, admitted_at[s]) > round_cap)
                rc = fail(STEINER_EDEVICE, "relaxation did not converge (%u rounds)",
                          rounds_since(round_seen, admitted_at[s]));
        if (rc) {
            fatal = rc;
            continue;
        }
        const uint32_t *done = (const uint32_t *)(hc + L.done);
        for (uint32_t s = 0; s < S; s++) {
            if (slot_state[s] == SLOT_ACTIVE && done[s]) {
                slot_state[s] = SLOT_TAIL;
                tail_q.push_back((int)s);
                cv_tail.notify_one();
            }
        }
    }
}

void steiner_server::run_tail() {
    (void)hipSetDevice(g->device);
    uint8_t *c = ctl.as<uint8_t>();
    const uint32_t n = g->n;
    const uint32_t *ids = (const uint32_t *)(c + L.slot_ids);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        while (tail_q.empty() && !stopping) cv_tail.wait(lk);
        if (stopping) return;
        const int slot = tail_q.front();
        tail_q.pop_front();
        Request *r = slot_req[slot];
        lk.unlock();
        // boundary scan and compaction of this query only
        ScanParams SP{};
        SP.g = g->dg;
        SP.key = P.key;
        SP.aux = P.aux;
        SP.heavy_pe = heavy_pe.as<uint32_t>();
        SP.pt = (uint64_t *const *)(c + L.pt_ptr);
        SP.tr = g->reordered ? (const uint32_t *const *)(c + L.tr_ptr) : nullptr;
        SP.slot_ids = ids + slot;
        SP.nscan = 1;
        SP.slot_err = (uint32_t *)(c + L.slot_err);
        SP.with_pred = o.lazy_pred ? 0 : 1;
        CompactParams CP{};
        CP.pt = SP.pt;
        CP.ts = g->reordered ? (const uint32_t *const *)(c + L.ts_ptr) : nullptr;
        CP.pt_len = (const uint64_t *)(c + L.pt_len);
        CP.out_idx = (uint32_t *const *)(c + L.oidx_ptr);
        CP.out_val = (uint64_t *const *)(c + L.oval_ptr);
        CP.out_cap = (const uint64_t *)(c + L.ocap);
        CP.out_cnt = (uint32_t *)(c + L.out_cnt);
        CP.slot_ids = SP.slot_ids;
        CP.nscan = 1;
        CP.pass = P.pass;
        const uint32_t grid = (uint32_t)std::max(1, g->cu_count) * 8;
        uint32_t err = 0, cnt = 0;
        int rc = hip_check(launch_scan(SP, grid, 256, s_tail), "scan");
        if (!rc) rc = hip_check(launch_compact(CP, grid, 256, s_tail), "compact");
        if (!rc) rc = hip_check(hipMemcpyAsync(&err, SP.slot_err + slot, 4, hipMemcpyDeviceToHost, s_tail), "D2H err");
        if (!rc) rc = hip_check(hipMemcpyAsync(&cnt, CP.out_cnt + slot, 4, hipMemcpyDeviceToHost, s_tail), "D2H count");
        if (!rc) rc = hip_check(hipStreamSynchronize(s_tail), "tail sync");
        int status = rc;
        std::unique_ptr<steiner_result> res;
        if (!rc) {
            if (err & (ERR_DIST_OVERFLOW | ERR_SUM_OVERFLOW)) {
                status = fail(STEINER_EOVERFLOW, "distance or cross-cell sum does not fit in 32 bits");
            } else {
                const uint32_t k = (uint32_t)r->S.size();
                const uint32_t *oi = (const uint32_t *)region(r, 1);
                const uint32_t *tr = r->rk.empty() ? nullptr : seeds_of(r) + k;
                if (cnt > r->oc_cap) {
                    status = fail(STEINER_EDEVICE, "G'1 overflow (%u entries)", cnt);
                } else {
                    status = tree_from_g1(g, s_tail, P.key + (size_t)slot * n, P.aux + (size_t)slot * n, k,
                                          (const uint64_t *)region(r, 0), tr, oi, cnt, SP.with_pred != 0, tail,
                                          region(r, 2), res, nullptr, nullptr, 256);
                }
                if (!status) res->stats.pairs = cnt;
            }
        }
        lk.lock();
        r->status = status;
        if (!status) {
            res->stats.ms_total = ms_since(r->t_submit);
            r->result = std::move(res);
        }
        r->done = true;
        used -= r->charge;
        pa.release(r->pool_off, r->pool_bytes);
        slot_state[slot] = SLOT_FREE;
        slot_req[slot] = nullptr;
        cv_done.notify_all();
        cv_sched.notify_one();
    }
}

// ---------------------------------------------------------------- C ABI

extern "C" uint64_t steiner_server_query_bytes(const steiner_server *s, uint32_t k) {
    if (!s) return 0;
    return s->slot_bytes + s->pool_need(std::max<uint32_t>(k, 2));
}

extern "C" int steiner_server_memory(const steiner_server *s, uint64_t *fixed_bytes, uint64_t *slot_bytes,
                                     uint32_t *slots, uint64_t *pool_bytes) {
    if (!s) return fail(STEINER_EINVAL, "NULL server");
    if (fixed_bytes) *fixed_bytes = s->fixed_bytes;
    if (slot_bytes) *slot_bytes = s->slot_bytes;
    if (slots) *slots = s->S;
    if (pool_bytes) *pool_bytes = s->pool_bytes;
    return STEINER_OK;
}

extern "C" int steiner_server_create(steiner_graph *g, uint64_t mem_budget_bytes, uint32_t max_slots,
                                     const steiner_options *opt, steiner_server **out) {
    if (!g || !out) return fail(STEINER_EINVAL, "NULL argument");
    if (max_slots == 0 || max_slots > MAX_SLOTS) return fail(STEINER_EINVAL, "max_slots must be in [1, %u]", MAX_SLOTS);
    int rc = hip_check(hipSetDevice(g->device), "hipSetDevice");
    if (rc) return rc;
    std::unique_ptr<steiner_server> s(new steiner_server());
    struct Cleanup {  // device memory and streams of a server that failed to start
        std::unique_ptr<steiner_server> &s;
        ~Cleanup() {
            if (s) s->free_device();
        }
    } cleanup{s};
    s->g = g;
    s->o = resolve_options(g, opt);
    if (s->o.driver != 4) s->o.driver = 1;  // host-stepped chunks (or their captured graphs)
    // the relaxation leaves a few workgroup slots free, so the tails' kernels (second stream) start at once
    // instead of waiting for a gap between round kernels
    if (!(opt && opt->grid)) s->o.grid = std::max<uint32_t>(1, s->o.grid - s->o.grid / 32);
    s->o.timing = false;
    s->o.counting = false;
    const uint32_t n = g->n;
    const uint64_t chunks = big_row_chunks(g, s->o.small_max, s->o.chunk);
    const ChunkTable *ct = nullptr;  // chunk memory of the large rows (not with the light/heavy split)
    if (!s->o.split || s->o.delta == 0xFFFFFFFFu) {
        std::lock_guard<std::mutex> lk(g->mu);
        ct = chunk_table(g, s->o.small_max, s->o.chunk, &rc);
        if (rc) return rc;
    }
    const uint64_t xchunks = ct ? ct->xchunks : 0;
    // per slot: key 8 + stamp/pred 4 + park 1 + settled 1 bytes per vertex, the heavy rows' pred minima, the
    // slot's share of the two S lists (two entries of 8 bytes per vertex each) and of the two B lists, and the
    // large rows' chunk memory
    s->slot_bytes = 14ull * n + 4ull * g->nheavy + 32ull * n + 32ull * chunks + 8ull * xchunks;
    s->half = g->nnz / 2 + 1;
    const uint64_t mark_bytes = ((uint64_t)n + 3) / 4 * 4, out_bytes = 12ull * n + 16;
    s->fixed_bytes = steiner_server::al(Layout(max_slots).total) + steiner_server::al(mark_bytes) +
                     steiner_server::al(out_bytes) + 4 * steiner_server::al(64 * 8) + 4;
    s->budget = mem_budget_bytes;
    const uint64_t one = s->fixed_bytes + s->slot_bytes + s->pool_need(2);
    if (s->budget < one)
        return fail(STEINER_EINVAL, "memory budget below one query's state (%llu bytes)", (unsigned long long)one);
    s->S = (uint32_t)std::min<uint64_t>(max_slots, (s->budget - s->fixed_bytes) / (s->slot_bytes + s->pool_need(2)));
    const uint32_t S = s->S;
    s->pool_bytes = s->budget - s->fixed_bytes - (uint64_t)S * s->slot_bytes;
    const uint64_t cap_s = 2ull * S * n + 64;
    const uint64_t cap_b = 2ull * S * chunks + 64;
    if (cap_s >= (1ull << 32) || cap_b >= (1ull << 32)) return fail(STEINER_ENOMEM, "too many slots for this graph");
    s->L = Layout(S);
    const size_t SN = (size_t)S * n;
    // exact sizes: everything the server holds on the device stays within the budget
    if ((rc = s->key.ensure(SN * 8, true)) || (rc = s->aux.ensure(SN * 4, true)) || (rc = s->dirty.ensure(SN, true)) ||
        (rc = s->settled.ensure(SN, true)) ||
        (rc = s->items_s[0].ensure(cap_s * 8, true)) || (rc = s->items_s[1].ensure(cap_s * 8, true)) ||
        (rc = s->items_b[0].ensure(cap_b * 8, true)) || (rc = s->items_b[1].ensure(cap_b * 8, true)) ||
        (rc = s->ctl.ensure(s->L.total, true)) || (rc = s->heavy_pe.ensure((size_t)S * g->nheavy * 4 + 4, true)) ||
        (rc = s->tail.mark.ensure(mark_bytes, true)) || (rc = s->tail.out.ensure(out_bytes, true)) ||
        (rc = s->pool.ensure(s->pool_bytes, true)) || (rc = s->hbuf.ensure(s->L.total + 4096)) ||
        (xchunks && (rc = s->xkey.ensure((size_t)S * xchunks * 8, true))))
        return rc;
    s->pa.init(s->pool_bytes);
    if ((rc = hip_check(hipStreamCreateWithFlags(&s->s_main, hipStreamNonBlocking), "stream"))) return rc;
    if ((rc = hip_check(hipStreamCreateWithFlags(&s->s_tail, hipStreamNonBlocking), "stream"))) return rc;
    VorParams &P = s->P;
    bind_pass(P, g->dg, s->ctl.as<uint8_t>(), s->L, S);
    P.key = s->key.as<uint64_t>();
    P.aux = s->aux.as<uint32_t>();
    P.dirty = s->dirty.as<uint8_t>();
    P.settled = s->settled.as<uint8_t>();
    P.items_s[0] = s->items_s[0].as<uint64_t>();
    P.items_s[1] = s->items_s[1].as<uint64_t>();
    P.items_b[0] = s->items_b[0].as<uint64_t>();
    P.items_b[1] = s->items_b[1].as<uint64_t>();
    bind_state(P, s->o, cap_s, cap_b);
    {
        std::lock_guard<std::mutex> lk(g->mu);
        if ((rc = bind_chunk_memory(P, g, s->o, S, s->xkey))) return rc;  // the exact buffer made above
    }
    if ((rc = hip_check(launch_pass_reset(P, s->s_main), "pass reset"))) return rc;
    if (const char *e = getenv("STEINER_SERVER_ROUND_BASE")) {  // testing the wrap of the round numbers
        s->round_base = (uint32_t)(strtoull(e, nullptr, 10) % ROUND_WRAP);
        hipLaunchKernelGGL(k_set_round, dim3(1), dim3(1), 0, s->s_main, P.pass, s->round_base);
        if ((rc = hip_check(hipGetLastError(), "round base"))) return rc;
    }
    if ((rc = hip_check(launch_fill_u32(s->tail.mark.as<uint32_t>(), mark_bytes / 4, 0u, s->s_main), "mark clear")))
        return rc;
    s->tail.mark_n = n;
    hipLaunchKernelGGL(k_iota, dim3((S + 255) / 256), dim3(256), 0, s->s_main,
                       (uint32_t *)(s->ctl.as<uint8_t>() + s->L.slot_ids), S);
    if ((rc = hip_check(hipStreamSynchronize(s->s_main), "server init"))) return rc;
    s->slot_req.assign(S, nullptr);
    s->slot_state.assign(S, SLOT_FREE);
    steiner_server *raw = s.release();
    raw->sched = std::thread([raw] { raw->run_sched(); });
    raw->tailer = std::thread([raw] { raw->run_tail(); });
    *out = raw;
    return STEINER_OK;
}

extern "C" int steiner_server_submit(steiner_server *s, const uint32_t *seeds, uint32_t k, uint64_t *ticket) {
    if (!s || !ticket) return fail(STEINER_EINVAL, "NULL argument");
    std::unique_ptr<Request> r(new Request());
    int rc = canon_seeds(s->g, seeds, k, r->S);
    if (!rc) seed_ranks(s->g, r->S, r->rk);
    if (rc) return rc;
    r->t_submit = std::chrono::steady_clock::now();
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) return fail(STEINER_ECANCELED, "server is shutting down");
    r->ticket = s->next_ticket++;
    if (r->S.size() < 2) {  // k == 1: empty tree, D = 0
        r->result.reset(new steiner_result());
        r->done = true;
    } else if (s->pool_need((uint32_t)r->S.size()) > s->pool_bytes) {
        return fail(STEINER_ENOMEM, "a query with %zu seeds needs more than the server's memory budget", r->S.size());
    } else {
        s->pending.push_back(r.get());
        s->cv_sched.notify_one();
    }
    *ticket = r->ticket;
    Request *raw = r.release();  // (the right operand of = is evaluated first)
    s->reqs[raw->ticket] = raw;
    return STEINER_OK;
}

extern "C" int steiner_server_wait(steiner_server *s, uint64_t ticket, int64_t timeout_us, steiner_result **out) {
    if (!s || !out) return fail(STEINER_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(STEINER_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    Request *r = it->second;
    auto ready = [&] { return r->done; };
    s->waiters++;
    bool in_time = true;
    if (timeout_us < 0) {
        s->cv_done.wait(lk, ready);
    } else {
        // the deadline is on the steady clock; each sleep is bounded through the system clock, whose
        // timed wait every threading tool understands
        const auto deadline = std::chrono::steady_clock::now() + std::chrono::microseconds(timeout_us);
        for (;;) {
            if (ready()) break;
            const auto now = std::chrono::steady_clock::now();
            if (now >= deadline) break;
            s->cv_done.wait_until(lk, std::chrono::system_clock::now() + (deadline - now));
        }
        in_time = ready();
    }
    s->waiters--;
    if (s->stopping) s->cv_done.notify_all();  // destroy waits for the waiters to leave
    if (!in_time) return fail(STEINER_ETIMEDOUT, "request %llu still running", (unsigned long long)ticket);
    const int status = r->status;
    std::unique_ptr<steiner_result> res = std::move(r->result);
    s->reqs.erase(r->ticket);
    delete r;
    if (status) return fail(status, "request failed: %s", steiner_strerror(status));
    if (!res) return fail(STEINER_EDEVICE, "missing result");
    *out = res.release();
    return STEINER_OK;
}

extern "C" int steiner_server_destroy(steiner_server *s) {
    if (!s) return STEINER_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
        s->cv_sched.notify_all();
        s->cv_tail.notify_all();
    }
    if (s->sched.joinable()) s->sched.join();
    if (s->tailer.joinable()) s->tailer.join();
    {
        std::unique_lock<std::mutex> lk(s->mu);
        for (auto &kv : s->reqs)
            if (!kv.second->done) {
                kv.second->status = STEINER_ECANCELED;
                kv.second->done = true;
            }
        s->cv_done.notify_all();
        // threads blocked in steiner_server_wait take their (canceled) results and leave first
        s->cv_done.wait(lk, [&] { return s->waiters == 0; });
    }
    (void)hipSetDevice(s->g->device);
    (void)hipStreamSynchronize(s->s_main);
    (void)hipStreamSynchronize(s->s_tail);
    for (auto &kv : s->reqs) delete kv.second;
    s->reqs.clear();
    s->free_device();
    delete s;
    return STEINER_OK;
}
