// gfx950 (MI355X) kernels of the Voronoi-cell Steiner tree hot path
// (arXiv:2205.14503, Alg. 2 Steps 1, 2, 4-6).
//
// Step 1, the Voronoi cells (Alg. 4's relaxation), runs as rounds of a
// distance-bucketed label-correcting pass over a frontier of improved
// vertices.  A vertex key packs (dist << 32) | seed index, so one 64-bit
// atomicMin applies the lexicographic (distance, seed index) order; the pass
// converges to the unique fixed point key[v] = min_i (d(s_i, v), i) whatever
// the processing order.  Improved vertices whose distance is inside the
// query's current bucket go to the next round's frontier; the others are
// parked with a dirty byte until their bucket comes up (Section IV's message
// prioritisation, realised as distance buckets instead of a priority queue).
//
// Frontier rows of degree <= small_max are expanded wave-cooperatively: a
// wave takes 64 items, prefix-sums their degrees and walks the combined edge
// range 64 edges per step (coalesced 8-byte (col, w) loads).  Larger rows are
// pushed as fixed chunks that any wave can take, so hubs spread over the GPU.
//
// Step 2 (Alg. 5) is one streaming pass over the CSR that gathers each edge's
// far key from its smaller endpoint only.  The canonical predecessor is found
// where it is needed: by the tree walks for ordinary rows, by the scan for
// rows above scan_heavy (and for every row when the caller asks for pred).
#include <algorithm>

#include "kernels.h"

namespace stn {

#define DEVI __device__ __forceinline__

constexpr uint32_t PERSIST_SLOTS = 256;

DEVI uint32_t lane() { return __lane_id(); }

DEVI uint64_t ld_agent(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
DEVI uint32_t ld_agent(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
DEVI void st_agent(uint64_t *p, uint64_t v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }


// Orders LDS traffic between the lanes of one wave.
DEVI void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

DEVI uint32_t wave_incl_scan(uint32_t x) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t y = __shfl_up(x, d, 64);
        if (lane() >= (uint32_t)d) x += y;
    }
    return x;
}

DEVI uint32_t wave_min(uint32_t x) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) x = min(x, (uint32_t)__shfl_xor(x, d, 64));
    return x;
}

DEVI uint32_t lanes_below(uint64_t mask) { return (uint32_t)__popcll(mask & ((1ull << lane()) - 1ull)); }

struct RoundIdx {
    uint32_t r;      // round number
    uint32_t cur;    // list read this round
    uint32_t nxt;    // list filled this round
    uint32_t c_nxt;  // counter set filled this round
    uint32_t b;      // near_mark / far_min buffer written this round
};

DEVI RoundIdx round_idx(uint32_t r) { return RoundIdx{r, r & 1u, (r + 1) & 1u, (r + 1) % 3u, r % 3u}; }

// Wave-aggregated append of S items (one atomic per wave).
DEVI void append_s(const VorParams &P, uint32_t list, uint32_t cidx, bool pred, uint64_t item) {
    uint64_t m = __ballot(pred);
    if (m == 0) return;
    uint32_t leader = (uint32_t)__ffsll((unsigned long long)m) - 1;
    uint32_t base = 0;
    if (lane() == leader) base = atomicAdd(&P.cnt->s[cidx], (uint32_t)__popcll(m));
    base = __shfl(base, leader, 64);
    if (pred) {
        uint32_t pos = base + lanes_below(m);
        if (pos < P.cap_s)
            P.items_s[list][pos] = item;
        else
            atomicOr(&P.pass->err, ERR_LIST_OVERFLOW);
    }
}

// Wave-aggregated append of the chunks of rows larger than small_max.
DEVI void append_b(const VorParams &P, uint32_t list, uint32_t cidx, bool pred, uint32_t slot, uint32_t v,
                   uint32_t deg, bool heavy = false) {
    uint64_t m = __ballot(pred);
    if (m == 0) return;
    uint32_t nch = pred ? (deg + P.chunk - 1) / P.chunk : 0;
    uint32_t incl = wave_incl_scan(nch);
    uint32_t total = __shfl(incl, 63, 64);
    uint32_t base = 0;
    if (lane() == 0) base = atomicAdd(&P.cnt->b[cidx], total);
    base = __shfl(base, 0, 64);
    if (pred) {
        uint32_t pos = base + incl - nch;
        for (uint32_t c = 0; c < nch; c++) {
            if (pos + c < P.cap_b) {
                P.items_b[list][pos + c] = b_item(slot, c, v, heavy);
            } else {
                atomicOr(&P.pass->err, ERR_LIST_OVERFLOW);
                break;
            }
        }
    }
}

// Per-wave LDS queue of improved small-degree vertices that the wave expands
// itself within the same round, so one round advances many hops along
// long shortest paths (high-diameter graphs otherwise need a global round per
// hop).  Anything the queue cannot hold goes to the next round's list.
constexpr uint32_t LQ_CAP = 128;
constexpr uint32_t OUT_CAP = 128;
constexpr uint32_t PEND_CAP = 256;
static_assert(LQ_CAP == 128, "lq_select holds two queue entries per lane");

struct WaveScratch {
    uint32_t incl[64];
    uint32_t beg[64];
    uint32_t slot[64];
    uint32_t pad[64];
    uint64_t key[64];
    // local queue: item (slot << 32 | v), the key it was improved to, its row extent
    uint64_t lq_item[LQ_CAP];
    uint64_t lq_key[LQ_CAP];
    uint32_t lq_beg[LQ_CAP];
    uint32_t lq_deg[LQ_CAP];
    // staging for the next round's S list: one global atomicAdd per flush
    // instead of one per 64-edge step (the list counter is a single address)
    uint64_t out[OUT_CAP];
    uint32_t out_n;
    // fixed-stride rows: improved vertices the local queue could not hold,
    // claimed for the next round's list together at the end of the unit
    uint64_t pend[PEND_CAP];
    uint32_t pend_n;
    uint32_t ev[EV_N];  // per-wave event counts (counting mode)
};

DEVI void count(const VorParams &P, WaveScratch *L, int which, bool pred) {
    if (!P.counting) return;
    const uint64_t m = __ballot(pred);
    if (lane() == 0 && m) L->ev[which] += (uint32_t)__popcll(m);
}

// Moves the wave's staged S items to the next round's list.
DEVI void flush_out(const VorParams &P, const RoundIdx &R, WaveScratch *L) {
    wave_sync();
    const uint32_t cnt = L->out_n;
    if (cnt == 0) return;
    uint32_t base = 0;
    if (lane() == 0) base = atomicAdd(&P.cnt->s[R.c_nxt], cnt);
    base = __shfl(base, 0, 64);
    for (uint32_t i = lane(); i < cnt; i += 64) {
        if (base + i < P.cap_s) P.items_s[R.nxt][base + i] = L->out[i];
        else atomicOr(&P.pass->err, ERR_LIST_OVERFLOW);
    }
    wave_sync();
    if (lane() == 0) L->out_n = 0;
    wave_sync();
}

// Stages S items of the lanes with `pred` (flushing first when full).
DEVI void stage_s(const VorParams &P, const RoundIdx &R, WaveScratch *L, bool pred, uint64_t item) {
    const uint64_t m = __ballot(pred);
    if (m == 0) return;
    const uint32_t cnt = (uint32_t)__popcll(m);
    wave_sync();
    if (L->out_n + cnt > OUT_CAP) flush_out(P, R, L);
    const uint32_t at = L->out_n;
    if (pred) L->out[at + lanes_below(m)] = item;
    wave_sync();
    if (lane() == 0) L->out_n = at + cnt;
    wave_sync();
}

constexpr int UNROLL = 4;  // independent 64-edge steps whose memory operations are issued together

// Relax UNROLL edges per lane (src key ksrc[i], target u[i], weight w[i] of
// query slot[i]; lanes/steps with valid[i] false do nothing) and schedule
// every improved target: into the wave's local queue (L != null, small row,
// room left) together with its improved key and row extent, else into the
// next round's list once per round (stamp), or park it if its distance is
// beyond the query's bucket.  The loads, atomics and row-offset reads of the
// UNROLL steps are independent and issued back to back, so one memory
// latency chain covers 64 * UNROLL edges.  Must be reached by every lane.
DEVI void relax_multi(const VorParams &P, const RoundIdx &R, const uint64_t *thr, const bool *valid,
                      const uint32_t *slot, const uint64_t *ksrc, const uint32_t *u, const uint32_t *w, WaveScratch *Lw,
                      bool use_lq, uint32_t &lq_head, uint32_t &lq_tail) {
    WaveScratch *L = use_lq ? Lw : nullptr;
    const uint32_t n = P.g.n;
    uint64_t cand[UNROLL], cur[UNROLL];
    uint32_t tv[UNROLL];  // bucket end, clamped: every stored distance is below 2^32 - 1
    bool live[UNROLL], tried[UNROLL], near[UNROLL];
    // All loads and atomics of the UNROLL steps are issued unconditionally (idle lanes read vertex 0
    // of their slot) and the atomics return nothing, so that they are in flight together; a branch
    // around an access, or a returned value, makes the compiler wait for it before the next one.
#pragma unroll
    for (int i = 0; i < UNROLL; i++) {
        const uint64_t d = (ksrc[i] >> 32) + (uint64_t)w[i];
        live[i] = valid[i] && d < DIST_INF;  // a distance of 2^32-1 or more is never stored
        cand[i] = (d << 32) | (ksrc[i] & 0xFFFFFFFFull);
        tv[i] = (uint32_t)min(thr[slot[i]], (uint64_t)DIST_INF);
    }
#pragma unroll
    for (int i = 0; i < UNROLL; i++)  // possibly stale (larger) values: filter only
        cur[i] = P.key[(size_t)slot[i] * n + (live[i] ? u[i] : 0u)];
    // A lane whose candidate beats its (possibly stale) read treats the edge as an improvement: the
    // lane whose atomic really lowers the key is always among them, and the others only add an
    // expansion that finds nothing, so no atomic has to return its old value.
    uint32_t beg[UNROLL], deg[UNROLL];
#pragma unroll
    for (int i = 0; i < UNROLL; i++) {
        tried[i] = live[i] && cand[i] < cur[i];
        near[i] = tried[i] && (uint32_t)(cand[i] >> 32) < tv[i];
        const uint32_t r = near[i] ? u[i] : 0u;
        beg[i] = P.g.rp[r];
        deg[i] = P.g.rp[r + 1];
    }
#pragma unroll
    for (int i = 0; i < UNROLL; i++) {
        count(P, Lw, EV_ATTEMPT, valid[i]);
        count(P, Lw, EV_ATOMIC, tried[i]);
    }
#pragma unroll
    for (int i = 0; i < UNROLL; i++)
        if (tried[i]) (void)atomicMin((unsigned long long *)(P.key + (size_t)slot[i] * n + u[i]), (unsigned long long)cand[i]);
#pragma unroll
    for (int i = 0; i < UNROLL; i++) {
        const uint32_t nd = (uint32_t)(cand[i] >> 32);
        if (!near[i]) beg[i] = deg[i] = 0;
        count(P, Lw, EV_PARK, tried[i] && !near[i]);
        if (tried[i] && !near[i]) {  // park until the query's bucket reaches it
            P.dirty[(size_t)slot[i] * n + u[i]] = 1;
            uint32_t *fm = P.far_min + (size_t)R.b * P.nslots + slot[i];
            if (nd < *fm) atomicMin(fm, nd);
        }
    }
    bool spill[UNROLL];  // near but not queued locally: claim for the next round's list
#pragma unroll
    for (int i = 0; i < UNROLL; i++) {
        deg[i] -= beg[i];
        // deferred large row: expanded once, at the bucket's advance, instead of at every improvement
        const bool defer = P.defer_min && near[i] && deg[i] > P.defer_min;
        if (defer) {
            P.settled[(size_t)slot[i] * n + u[i]] = 1;
            uint32_t *sm = P.settle_mark + (size_t)R.b * P.nslots + slot[i];
            if (*sm == 0) *sm = 1;
            near[i] = false;
        }
        bool local = false;
        if (L) {
            const bool want = near[i] && deg[i] <= P.small_max;
            const uint64_t m = __ballot(want);
            if (m) {
                const uint32_t space = LQ_CAP - (lq_tail - lq_head);
                const uint32_t rank = lanes_below(m);
                local = want && rank < space;
                if (local) {
                    const uint32_t at = (lq_tail + rank) % LQ_CAP;
                    L->lq_item[at] = s_item(slot[i], u[i]);
                    L->lq_key[at] = cand[i];
                    L->lq_beg[at] = beg[i];
                    L->lq_deg[at] = deg[i];
                }
                lq_tail += min((uint32_t)__popcll(m), space);
            }
        }
        count(P, Lw, EV_IMPROVED, tried[i]);
        count(P, Lw, EV_LOCAL, local);
        spill[i] = near[i] && !local;
    }
    // the claims of all steps are in flight together: the returned stamps are used only after the
    // last one is issued (an empty asm hides them from the compiler until then)
    uint32_t old[UNROLL];
#pragma unroll
    for (int i = 0; i < UNROLL; i++) {
        old[i] = R.r + 1;
        if (spill[i]) old[i] = atomicExch(P.aux + (size_t)slot[i] * n + u[i], R.r + 1);
    }
#pragma unroll
    for (int i = 0; i < UNROLL; i++) asm volatile("" : "+v"(old[i]));
#pragma unroll
    for (int i = 0; i < UNROLL; i++) {
        const bool claim = spill[i] && old[i] != R.r + 1;
        if (claim) {
            uint32_t *nm = P.near_mark + (size_t)R.b * P.nslots + slot[i];
            if (*nm == 0) *nm = 1;
        }
        count(P, Lw, EV_GLOBAL, claim);
        stage_s(P, R, Lw, claim && deg[i] <= P.small_max, s_item(slot[i], u[i]));
        append_b(P, R.nxt, R.c_nxt, claim && deg[i] > P.small_max, slot[i], u[i], deg[i]);
    }
}

// Expands one frontier item per lane: the row [beg, beg + deg) of a vertex
// with key kv in query `slot` (deg = 0 for idle lanes), 64 * UNROLL edges per
// step, balanced across the wave by a prefix sum of the degrees (coalesced
// 8-byte (col, w) loads within each row).
DEVI void expand_items(const VorParams &P, const RoundIdx &R, const uint64_t *thr, uint32_t slot, uint32_t v,
                       uint64_t kv, uint32_t beg, uint32_t deg, bool heavy, WaveScratch *L, bool use_lq,
                       uint32_t &lq_head, uint32_t &lq_tail) {
    const uint32_t ln = lane();
    count(P, L, EV_ITEMS, kv != KEY_INF);
    if (P.split && !heavy && kv != KEY_INF) {  // its heavy edges wait until the bucket closes
        P.settled[(size_t)slot * P.g.n + v] = 1;
        uint32_t *sm = P.settle_mark + (size_t)R.b * P.nslots + slot;
        if (*sm == 0) *sm = 1;
    }
    const uint32_t incl = wave_incl_scan(deg);
    const uint32_t total = __shfl(incl, 63, 64);
    wave_sync();
    L->incl[ln] = incl;
    L->beg[ln] = beg;
    L->slot[ln] = slot;
    L->pad[ln] = heavy ? 1u : 0u;
    L->key[ln] = kv;
    wave_sync();
    for (uint32_t base = 0; base < total; base += 64 * UNROLL) {
        bool valid[UNROLL], hv[UNROLL];
        uint32_t sl[UNROLL], uu[UNROLL], ww[UNROLL], e[UNROLL];
        uint64_t ks[UNROLL];
#pragma unroll
        for (int i = 0; i < UNROLL; i++) {
            const uint32_t t = base + 64 * i + ln;
            valid[i] = t < total;
            uint32_t j = 0;
            if (valid[i]) {
                uint32_t lo = 0, hi = 63;
                while (lo < hi) {
                    uint32_t mid = (lo + hi) >> 1;
                    if (L->incl[mid] > t) hi = mid; else lo = mid + 1;
                }
                j = lo;
            }
            const uint32_t ex = j ? L->incl[j - 1] : 0;
            e[i] = L->beg[j] + (t - ex);
            sl[i] = L->slot[j];
            ks[i] = L->key[j];
            hv[i] = L->pad[j] != 0;
        }
#pragma unroll
        for (int i = 0; i < UNROLL; i++) {  // unconditional loads (idle lanes read entry 0): all in flight together
            const uint2 a = P.g.adj[valid[i] ? e[i] : 0u];
            uu[i] = valid[i] ? a.x : 0u;
            ww[i] = a.y;
            if (P.split) valid[i] = valid[i] && (hv[i] ? a.y > P.delta : a.y <= P.delta);
        }
        relax_multi(P, R, thr, valid, sl, ks, uu, ww, L, use_lq, lq_head, lq_tail);
    }
}

// One wave expands one chunk of a large row.
DEVI void process_b_chunk(const VorParams &P, const RoundIdx &R, const uint64_t *thr, uint32_t idx, WaveScratch *L,
                          bool use_lq, uint32_t &lq_head, uint32_t &lq_tail) {
    const uint64_t it = P.items_b[R.cur][idx];
    const uint32_t slot = (uint32_t)(it >> 52);
    const bool heavy = ((it >> 51) & 1u) != 0;
    const uint32_t c = (uint32_t)(it >> 32) & ((1u << CHUNK_BITS) - 1);
    const uint32_t v = (uint32_t)it;
    const uint64_t kv = ld_agent(P.key + (size_t)slot * P.g.n + v);
    bool again = false;  // this chunk was already expanded with this very key: nothing new to push
    if (P.xkey && v < P.nxrow && kv != KEY_INF) {
        uint64_t *xk = P.xkey + (size_t)slot * P.xchunks + P.xchunk[v] + c;
        again = *xk == kv;
        if (!again && lane() == 0) *xk = kv;
    }
    if (P.split && !heavy && c == 0 && kv != KEY_INF) {  // heavy edges wait until the bucket closes
        if (lane() == 0) {
            P.settled[(size_t)slot * P.g.n + v] = 1;
            uint32_t *sm = P.settle_mark + (size_t)R.b * P.nslots + slot;
            if (*sm == 0) *sm = 1;
        }
    }
    const uint32_t beg = P.g.rp[v] + c * P.chunk;
    const uint32_t lim = P.g.rp[v + 1];
    uint32_t end = (lim - beg > P.chunk) ? beg + P.chunk : lim;
    if (kv == KEY_INF || again) end = beg;
    for (uint32_t e0 = beg; e0 < end; e0 += 64 * UNROLL) {
        bool valid[UNROLL];
        uint32_t sl[UNROLL], uu[UNROLL], ww[UNROLL];
        uint64_t ks[UNROLL];
#pragma unroll
        for (int i = 0; i < UNROLL; i++) {
            const uint64_t e = (uint64_t)e0 + 64 * i + lane();
            valid[i] = e < end;
            const uint2 a = P.g.adj[valid[i] ? e : (uint64_t)beg];
            uu[i] = valid[i] ? a.x : 0u;
            ww[i] = a.y;
            if (P.split) valid[i] = valid[i] && (heavy ? a.y > P.delta : a.y <= P.delta);
            sl[i] = slot;
            ks[i] = kv;
            count(P, L, EV_LARGE, valid[i]);
        }
        relax_multi(P, R, thr, valid, sl, ks, uu, ww, L, use_lq, lq_head, lq_tail);
    }
}

// A monotone 16-bit compression of a distance (a 5-bit exponent over an
// 11-bit mantissa; exact below 2048, relative step 2^-11 above): the local
// queue's order only needs nearly-smallest-first.
DEVI uint32_t order_key(uint32_t d) {
    if (d < 2048u) return d;
    const uint32_t t = 31u - (uint32_t)__builtin_clz(d);  // 11..31
    return ((t - 10u) << 11) | ((d >> (t - 11u)) & 0x7FFu);
}

// The 64 entries of smallest order key among the local queue's cnt > 64
// entries at ring positions [h, h + cnt) (equal keys in position order) are
// returned in the lanes' registers; the others move to [h + 64, h + cnt).  A
// radix search over the 16 key bits (two ballots per bit) finds the 64th
// smallest key x; the entries below x and the first ones equal to it are
// placed by ballot prefixes (one per lane, through LDS), and so is the rest.
// Order only steers the work, never the result.
DEVI void lq_select(WaveScratch *L, uint32_t h, uint32_t cnt, uint64_t &item, uint64_t &kv, uint32_t &beg,
                    uint32_t &deg) {
    const uint32_t ln = lane();
    constexpr uint32_t NONE = 1u << 16;  // above every order key
    uint32_t a[2], p[2];
#pragma unroll
    for (int j = 0; j < 2; j++) {
        const uint32_t i = ln + 64 * j;
        p[j] = (h + i) % LQ_CAP;
        a[j] = i < cnt ? order_key((uint32_t)(L->lq_key[p[j]] >> 32)) : NONE;
    }
    uint32_t x = 0;  // the largest value with at most 63 keys below it: the 64th smallest key
#pragma unroll
    for (int bit = 15; bit >= 0; bit--) {
        const uint32_t y = x | (1u << bit);
        const uint32_t below = (uint32_t)__popcll(__ballot(a[0] < y)) + (uint32_t)__popcll(__ballot(a[1] < y));
        x = below <= 63 ? y : x;
    }
    // fewer than 64 keys lie below x and at least 64 at or below it: the first `need` equal ones join
    const uint64_t b0 = __ballot(a[0] < x), b1 = __ballot(a[1] < x);
    const uint64_t e0 = __ballot(a[0] == x), e1 = __ballot(a[1] == x);
    const uint32_t need = 64u - (uint32_t)__popcll(b0) - (uint32_t)__popcll(b1);
    const bool s0 = a[0] < x || (a[0] == x && lanes_below(e0) < need);
    const bool s1 = a[1] < x || (a[1] == x && (uint32_t)__popcll(e0) + lanes_below(e1) < need);
    const bool q0 = !s0 && a[0] != NONE, q1 = !s1 && a[1] != NONE;
    const uint64_t m0 = __ballot(s0), m1 = __ballot(s1), n0 = __ballot(q0), n1 = __ballot(q1);
    uint32_t *slot = L->incl;  // free until the expansion rebuilds it
    if (s0) slot[lanes_below(m0)] = p[0];
    if (s1) slot[(uint32_t)__popcll(m0) + lanes_below(m1)] = p[1];
    // the rest: every entry is read before any is written
    uint64_t r_item[2] = {0, 0}, r_key[2] = {0, 0};
    uint32_t r_beg[2] = {0, 0}, r_deg[2] = {0, 0};
#pragma unroll
    for (int j = 0; j < 2; j++) {
        if (j ? q1 : q0) {
            r_item[j] = L->lq_item[p[j]];
            r_key[j] = L->lq_key[p[j]];
            r_beg[j] = L->lq_beg[p[j]];
            r_deg[j] = L->lq_deg[p[j]];
        }
    }
    wave_sync();
    const uint32_t pb = slot[ln];
    item = L->lq_item[pb];
    kv = L->lq_key[pb];
    beg = L->lq_beg[pb];
    deg = L->lq_deg[pb];
    wave_sync();
#pragma unroll
    for (int j = 0; j < 2; j++) {
        if (j ? q1 : q0) {
            const uint32_t at = (h + 64 + (j ? (uint32_t)__popcll(n0) + lanes_below(n1) : lanes_below(n0))) % LQ_CAP;
            L->lq_item[at] = r_item[j];
            L->lq_key[at] = r_key[j];
            L->lq_beg[at] = r_beg[j];
            L->lq_deg[at] = r_deg[j];
        }
    }
    wave_sync();
}

// Expand the wave's local queue for at most `budget` batches of 64 (each
// entry carries the key it was improved to: a later improvement of the same
// vertex queues or lists it again), then move what is left to the next
// round's list (once per vertex per round; that path re-reads the key).
DEVI void drain_local(const VorParams &P, const RoundIdx &R, const uint64_t *thr, WaveScratch *L, uint32_t budget,
                      uint32_t &h, uint32_t &t) {
    for (uint32_t it = 0; it < budget && h != t; it++) {
        const uint32_t cnt = t - h;
        const uint32_t take = min(cnt, 64u);
        wave_sync();
        uint64_t item = 0, kv = KEY_INF;
        uint32_t beg = 0, deg = 0;
        if ((P.lq_mode & 1u) && cnt > 64) {
            lq_select(L, h, cnt, item, kv, beg, deg);
        } else if (lane() < take) {
            const uint32_t at = (h + lane()) % LQ_CAP;
            item = L->lq_item[at];
            kv = L->lq_key[at];
            beg = L->lq_beg[at];
            deg = L->lq_deg[at];
        }
        h += take;
        if ((P.lq_mode & 2u) && kv != KEY_INF) {  // superseded: a smaller key of this vertex is queued elsewhere
            if (ld_agent(P.key + (size_t)s_slot(item) * P.g.n + (uint32_t)item) < kv) {
                deg = 0;
                kv = KEY_INF;
            }
        }
        expand_items(P, R, thr, s_slot(item), (uint32_t)item, kv, beg, deg, false, L, true, h, t);
    }
    while (h != t) {
        const uint32_t take = min(t - h, 64u);
        wave_sync();
        const bool has = lane() < take;
        const uint64_t item = has ? L->lq_item[(h + lane()) % LQ_CAP] : 0;
        h += take;
        bool claim = false;
        if (has) {
            const uint32_t slot = s_slot(item), v = (uint32_t)item;
            if (atomicExch(P.aux + (size_t)slot * P.g.n + v, R.r + 1) != R.r + 1) {
                claim = true;
                uint32_t *nm = P.near_mark + (size_t)R.b * P.nslots + slot;
                if (*nm == 0) *nm = 1;
            }
        }
        stage_s(P, R, L, claim, item);
    }
}


// ------------------------------------------- rows of at most ELL_W entries
//
// On a graph whose rows all fit the fixed-stride copy (a grid), a hop of the
// local queue is a chain of dependent device-memory accesses, so this path
// keeps it short: a row's address follows from the vertex id (no row-offset
// read), the superseded test reads the key together with the row, and the
// claims of spilled vertices wait until the end of the unit.

static_assert(UNROLL == (int)ELL_W, "one step per fixed-stride row entry");

// Claims the wave's pending spilled items for the next round's list (once per
// vertex per round, stamp R.r + 1), UNROLL exchanges per lane in flight, and
// stages the claimed ones.
DEVI void claim_pending(const VorParams &P, const RoundIdx &R, WaveScratch *L) {
    wave_sync();
    const uint32_t cnt = L->pend_n;
    const uint32_t n = P.g.n;
    for (uint32_t base = 0; base < cnt; base += 64 * UNROLL) {
        uint64_t it[UNROLL];
        uint32_t old[UNROLL];
        bool has[UNROLL];
#pragma unroll
        for (int j = 0; j < UNROLL; j++) {
            const uint32_t idx = base + 64 * j + lane();
            has[j] = idx < cnt;
            it[j] = has[j] ? L->pend[idx] : 0;
        }
#pragma unroll
        for (int j = 0; j < UNROLL; j++) {
            old[j] = R.r + 1;
            if (has[j]) old[j] = atomicExch(P.aux + (size_t)s_slot(it[j]) * n + (uint32_t)it[j], R.r + 1);
        }
#pragma unroll
        for (int j = 0; j < UNROLL; j++) asm volatile("" : "+v"(old[j]));  // all exchanges issued first
#pragma unroll
        for (int j = 0; j < UNROLL; j++) {
            const bool claim = has[j] && old[j] != R.r + 1;
            if (claim) P.near_mark[(size_t)R.b * P.nslots + s_slot(it[j])] = 1;  // no read: off the chain
            count(P, L, EV_GLOBAL, claim);
            stage_s(P, R, L, claim, it[j]);
        }
    }
    wave_sync();
    if (lane() == 0) L->pend_n = 0;
    wave_sync();
}

// Adds the items of the lanes with `pred` to the pending claims.
DEVI void pend_items(const VorParams &P, const RoundIdx &R, WaveScratch *L, bool pred, uint64_t item) {
    const uint64_t m = __ballot(pred);
    if (m == 0) return;
    const uint32_t cnt = (uint32_t)__popcll(m);
    wave_sync();
    if (L->pend_n + cnt > PEND_CAP) claim_pending(P, R, L);
    const uint32_t at = L->pend_n;
    if (pred) L->pend[at + lanes_below(m)] = item;
    wave_sync();
    if (lane() == 0) L->pend_n = at + cnt;
    wave_sync();
}

// relax_multi for one fixed-stride row per lane (source key ksrc of query
// slot; step i relaxes entry i): improved targets inside the bucket go to the
// local queue (key only: the row needs no extent) or, when it is full (or
// unused), to the pending claims; the others are parked.
DEVI void relax_narrow(const VorParams &P, const RoundIdx &R, const uint64_t *thr, const bool *valid,
                       uint32_t slot, uint64_t ksrc, const uint32_t *u, const uint32_t *w, WaveScratch *L,
                       bool use_lq, uint32_t &lq_head, uint32_t &lq_tail) {
    const uint32_t n = P.g.n;
    const uint32_t tv = (uint32_t)min(thr[slot], (uint64_t)DIST_INF);
    uint64_t cand[UNROLL], cur[UNROLL];
    bool live[UNROLL], tried[UNROLL], near[UNROLL];
#pragma unroll
    for (int i = 0; i < UNROLL; i++) {
        const uint64_t d = (ksrc >> 32) + (uint64_t)w[i];
        live[i] = valid[i] && d < DIST_INF;
        cand[i] = (d << 32) | (ksrc & 0xFFFFFFFFull);
    }
#pragma unroll
    for (int i = 0; i < UNROLL; i++)  // possibly stale (larger) values: filter only
        cur[i] = P.key[(size_t)slot * n + (live[i] ? u[i] : 0u)];
#pragma unroll
    for (int i = 0; i < UNROLL; i++) {
        tried[i] = live[i] && cand[i] < cur[i];
        near[i] = tried[i] && (uint32_t)(cand[i] >> 32) < tv;
        count(P, L, EV_ATTEMPT, valid[i]);
        count(P, L, EV_ATOMIC, tried[i]);
    }
#pragma unroll
    for (int i = 0; i < UNROLL; i++)
        if (tried[i]) (void)atomicMin((unsigned long long *)(P.key + (size_t)slot * n + u[i]), (unsigned long long)cand[i]);
#pragma unroll
    for (int i = 0; i < UNROLL; i++) {
        if (tried[i] && !near[i]) {  // park until the query's bucket reaches it
            P.dirty[(size_t)slot * n + u[i]] = 1;
            uint32_t *fm = P.far_min + (size_t)R.b * P.nslots + slot;
            const uint32_t nd = (uint32_t)(cand[i] >> 32);
            if (nd < *fm) atomicMin(fm, nd);
        }
    }
#pragma unroll
    for (int i = 0; i < UNROLL; i++) {
        bool local = false;
        if (use_lq) {
            const uint64_t m = __ballot(near[i]);
            if (m) {
                const uint32_t space = LQ_CAP - (lq_tail - lq_head);
                const uint32_t rank = lanes_below(m);
                local = near[i] && rank < space;
                if (local) {
                    const uint32_t at = (lq_tail + rank) % LQ_CAP;
                    L->lq_item[at] = s_item(slot, u[i]);
                    L->lq_key[at] = cand[i];
                }
                lq_tail += min((uint32_t)__popcll(m), space);
            }
        }
        count(P, L, EV_IMPROVED, tried[i]);
        count(P, L, EV_LOCAL, local);
        count(P, L, EV_PARK, tried[i] && !near[i]);
        pend_items(P, R, L, near[i] && !local, s_item(slot, u[i]));
    }
}

// Expands one fixed-stride row per lane (vertex v of query slot with key kv;
// lanes with `active` false do nothing).  check_sup: the items come from the
// local queue with the key they were queued with, and one whose vertex has
// been improved since is skipped (its key is read together with the row).
DEVI void expand_narrow(const VorParams &P, const RoundIdx &R, const uint64_t *thr, uint32_t slot, uint32_t v,
                        uint64_t kv, bool active, bool heavy, WaveScratch *L, bool use_lq, uint32_t &lq_head,
                        uint32_t &lq_tail, bool check_sup) {
    if (__ballot(active) == 0) return;
    // a plain read: a stale value is never below the current key, so it can only miss a skip
    uint64_t now = KEY_INF;
    if (check_sup) now = P.key[(size_t)slot * P.g.n + v];
    const uint4 r0 = P.g.ell[2 * (size_t)v], r1 = P.g.ell[2 * (size_t)v + 1];
    const uint32_t col[UNROLL] = {r0.x, r0.z, r1.x, r1.z}, wt[UNROLL] = {r0.y, r0.w, r1.y, r1.w};
    const bool on = active && kv != KEY_INF && !(check_sup && (P.lq_mode & 2u) && now < kv);
    count(P, L, EV_ITEMS, on);
    if (P.split && !heavy && on) {  // its heavy edges wait until the bucket closes
        P.settled[(size_t)slot * P.g.n + v] = 1;
        uint32_t *sm = P.settle_mark + (size_t)R.b * P.nslots + slot;
        if (*sm == 0) *sm = 1;
    }
    bool valid[UNROLL];
    uint32_t uu[UNROLL];
#pragma unroll
    for (int i = 0; i < UNROLL; i++) {
        valid[i] = on && col[i] != ELL_NONE;
        if (P.split) valid[i] = valid[i] && (heavy ? wt[i] > P.delta : wt[i] <= P.delta);
        uu[i] = valid[i] ? col[i] : 0u;
    }
    relax_narrow(P, R, thr, valid, slot, kv, uu, wt, L, use_lq, lq_head, lq_tail);
}

// drain_local for fixed-stride rows: up to `budget` batches of 64, smallest
// first; what is left joins the pending claims, which are then made.
DEVI void drain_narrow(const VorParams &P, const RoundIdx &R, const uint64_t *thr, WaveScratch *L, uint32_t budget,
                       uint32_t &h, uint32_t &t) {
    for (uint32_t it = 0; it < budget && h != t; it++) {
        const uint32_t cnt = t - h;
        const uint32_t take = min(cnt, 64u);
        wave_sync();
        uint64_t item = 0, kv = KEY_INF;
        if ((P.lq_mode & 1u) && cnt > 64) {
            uint32_t beg_unused, deg_unused;
            lq_select(L, h, cnt, item, kv, beg_unused, deg_unused);
        } else if (lane() < take) {
            const uint32_t at = (h + lane()) % LQ_CAP;
            item = L->lq_item[at];
            kv = L->lq_key[at];
        }
        h += take;
        expand_narrow(P, R, thr, s_slot(item), (uint32_t)item, kv, lane() < take, false, L, true, h, t, true);
    }
    while (h != t) {
        const uint32_t take = min(t - h, 64u);
        wave_sync();
        const bool has = lane() < take;
        const uint64_t item = has ? L->lq_item[(h + lane()) % LQ_CAP] : 0;
        h += take;
        pend_items(P, R, L, has, item);
    }
}

template <bool NARROW>
DEVI void relax_round_body(const VorParams &P, const RoundIdx &R, const uint64_t *thr, uint32_t cs, uint32_t cb,
                           WaveScratch *L, uint32_t wave_gid, uint32_t nwaves) {
    const uint32_t ng = (cs + 63) / 64;
    const uint32_t units = ng + cb;
    const bool use_lq = P.local_iters != 0;
    if (lane() == 0) {
        L->out_n = 0;
        L->pend_n = 0;
        for (int i = 0; i < EV_N; i++) L->ev[i] = 0;
    }
    wave_sync();
    for (uint32_t u = wave_gid; u < units; u += nwaves) {
        uint32_t h = 0, t = 0;
        if (NARROW && u < ng) {  // rows of at most ELL_W entries: every item is a small row
            const uint32_t idx = u * 64 + lane();
            uint32_t slot = 0, v = 0;
            uint64_t kv = KEY_INF;
            bool heavy = false;
            if (idx < cs) {
                const uint64_t it = P.items_s[R.cur][idx];
                slot = s_slot(it);
                heavy = s_heavy(it);
                v = (uint32_t)it;
                kv = ld_agent(P.key + (size_t)slot * P.g.n + v);
            }
            expand_narrow(P, R, thr, slot, v, kv, idx < cs, heavy, L, use_lq, h, t, false);
            if (use_lq) drain_narrow(P, R, thr, L, P.local_iters, h, t);
            claim_pending(P, R, L);
        } else {
            if (u < ng) {
                const uint32_t idx = u * 64 + lane();
                uint32_t slot = 0, beg = 0, deg = 0, v = 0;
                uint64_t kv = KEY_INF;
                bool heavy = false;
                if (idx < cs) {
                    const uint64_t it = P.items_s[R.cur][idx];
                    slot = s_slot(it);
                    heavy = s_heavy(it);
                    v = (uint32_t)it;
                    kv = ld_agent(P.key + (size_t)slot * P.g.n + v);
                    beg = P.g.rp[v];
                    deg = kv == KEY_INF ? 0 : P.g.rp[v + 1] - beg;
                }
                expand_items(P, R, thr, slot, v, kv, beg, deg, heavy, L, use_lq, h, t);
            } else {
                process_b_chunk(P, R, thr, u - ng, L, use_lq, h, t);
            }
            if (use_lq) drain_local(P, R, thr, L, P.local_iters, h, t);
        }
        flush_out(P, R, L);
    }
    if (P.counting && lane() < EV_N) {
        wave_sync();
        const uint32_t c = L->ev[lane()];
        if (c) atomicAdd(&P.cnt->ev[lane()], (unsigned long long)c);
    }
}

// Bucket decision for one query at the end of round r (identical inputs give
// identical outputs, so the persistent kernel can evaluate it redundantly in
// every workgroup).
DEVI void decide_slot(const VorParams &P, uint32_t r, uint32_t q, uint64_t *thr, uint64_t *thr_prev,
                      uint32_t *carry, uint32_t *active, uint32_t *adv, uint32_t *done, uint32_t *advances,
                      bool &any_adv, bool &any_active) {
    adv[q] = 0;
    if (!active[q]) return;
    const uint32_t b = r % 3u;
    uint32_t c = min(carry[q], ld_agent(P.far_min + (size_t)b * P.nslots + q));
    // vertices expanded in the open bucket still owe their heavy edges: work at >= thr
    if (ld_agent(P.settle_mark + (size_t)b * P.nslots + q)) c = min(c, (uint32_t)min(thr[q], (uint64_t)DIST_INF - 1));
    const bool has_near = ld_agent(P.near_mark + (size_t)b * P.nslots + q) != 0;
    if (!has_near) {
        if (c == DIST_INF) {
            active[q] = 0;
            done[q] = 1;
        } else {
            const uint64_t dl = P.delta;
            thr_prev[q] = thr[q];
            thr[q] = ((uint64_t)c / dl + 1) * dl;
            c = DIST_INF;
            adv[q] = 1;
            advances[q] += 1;
            any_adv = true;
        }
    }
    carry[q] = c;
    if (active[q]) any_active = true;
}

// Parked vertices of every advancing query whose distance falls below the new
// bucket end join list `list` (stamp `stamp`); stale marks are cleared; the
// minimum parked distance left over goes to far_min[fm_buf]; if nm_buf >= 0
// the query's near mark in that buffer is set when something was pushed.
DEVI void advance_body(const VorParams &P, const uint64_t *thr, const uint64_t *thr_prev, const uint32_t *adv,
                       uint32_t stamp, uint32_t list, uint32_t cidx, uint32_t fm_buf, int nm_buf, uint32_t wave_gid,
                       uint32_t nwaves, WaveScratch *L) {
    // S items go through the wave's staging buffer (one list atomic per flush)
    RoundIdx Rs;
    Rs.nxt = list;
    Rs.c_nxt = cidx;
    if (lane() == 0) L->out_n = 0;
    wave_sync();
    const uint32_t n = P.g.n;
    for (uint32_t q = 0; q < P.nslots; q++) {
        if (!adv[q]) continue;
        const uint64_t lo = thr_prev[q], hi = thr[q];
        uint32_t kept = DIST_INF;
        bool pushed = false;
        for (uint32_t base = wave_gid * 64; base < n; base += nwaves * 64) {
            const uint32_t v = base + lane();
            bool push = false, hpush = false;
            uint32_t deg = 0;
            if (v < n) {
                const size_t o = (size_t)q * n + v;
                if (P.split && P.settled[o]) {  // the closed bucket's vertices relax their heavy edges
                    P.settled[o] = 0;
                    deg = P.g.rp[v + 1] - P.g.rp[v];
                    hpush = true;
                } else if (!P.split && P.settled[o]) {  // a large row deferred to the bucket's end
                    P.settled[o] = 0;
                    P.aux[o] = stamp;
                    deg = P.g.rp[v + 1] - P.g.rp[v];
                    push = true;
                } else if (P.dirty[o]) {
                    const uint32_t d = (uint32_t)(ld_agent(P.key + o) >> 32);
                    if (d < lo) {
                        P.dirty[o] = 0;
                    } else if (d < hi) {
                        P.dirty[o] = 0;
                        P.aux[o] = stamp;
                        deg = P.g.rp[v + 1] - P.g.rp[v];
                        push = true;
                    } else {
                        kept = min(kept, d);
                    }
                }
            }
            pushed |= __ballot(push || hpush) != 0;
            stage_s(P, Rs, L, (push || hpush) && deg <= P.small_max, s_item(q, v, hpush));
            append_b(P, list, cidx, (push || hpush) && deg > P.small_max, q, v, deg, hpush);
        }
        flush_out(P, Rs, L);
        kept = wave_min(kept);
        if (lane() == 0) {
            if (kept != DIST_INF) atomicMin(P.far_min + (size_t)fm_buf * P.nslots + q, kept);
            if (pushed && nm_buf >= 0) P.near_mark[(size_t)nm_buf * P.nslots + q] = 1;
        }
    }
}

// ------------------------------------------------------------ host-stepped

// One round per launch: the advance scan decided at the end of the previous
// round (its pushes are processed one round later), the relaxation of this
// round's list, and, in the last workgroup to finish, the bucket decision.
// 256-thread workgroups (the host clamps the block size); the default grid is
// as many workgroups as fit on the device at once (round_max_grid).
template <bool NARROW>
__global__ void __launch_bounds__(256) k_round(VorParams P) {
    extern __shared__ __align__(16) unsigned char dyn_smem[];
    WaveScratch *s_wave = (WaveScratch *)dyn_smem;
    __shared__ int s_last, s_adv, s_act;
    // The pass state, all loads in flight together (the list counts of every buffer, selected after).  A
    // workgroup dispatched after this launch's decision (late, behind other kernels' workgroups) reads the next
    // round's control word; were it to take part in that round inside this launch it would count toward the
    // wrong launch.  The word carries the identity of the launch that decided last (its dispatch-packet address,
    // distinct for consecutive launches), so such a workgroup sees its own launch's identity and leaves.  A
    // workgroup that takes part is counted before any decision and never sees it.  The counts of this round's
    // list do not change during the launch.  (A stale identity equal to this launch's, after the queue's ring
    // has wrapped, makes every workgroup leave: the launch changes nothing and the next one does the round.)
    const uint64_t pw = ld_agent(&P.pass->word);
    uint32_t s3[3], b3[3];
#pragma unroll
    for (int i = 0; i < 3; i++) {
        s3[i] = ld_agent(&P.cnt->s[i]);
        b3[i] = ld_agent(&P.cnt->b[i]);
    }
    const uint32_t did = (uint32_t)(uintptr_t)__builtin_amdgcn_dispatch_ptr();
    if ((pw >> 63) || (uint32_t)pw == did) return;
    const uint32_t r = (uint32_t)(pw >> 32) & 0x3FFFFFFFu, any_adv = (uint32_t)(pw >> 62) & 1u;
    const uint32_t cur = r % 3u;  // this round's list (the advance below fills the next one)
    // uniform values: scalar registers
    const uint32_t cs = (uint32_t)__builtin_amdgcn_readfirstlane(
        (int)min(cur == 0 ? s3[0] : cur == 1 ? s3[1] : s3[2], P.cap_s));
    const uint32_t cb = (uint32_t)__builtin_amdgcn_readfirstlane(
        (int)min(cur == 0 ? b3[0] : cur == 1 ? b3[1] : b3[2], P.cap_b));
    const RoundIdx R = round_idx((uint32_t)__builtin_amdgcn_readfirstlane((int)r));
    const uint32_t wpb = blockDim.x / 64, w = threadIdx.x / 64;
    // Workgroups that take part in this round: all of them when parked vertices move (the advance scans every
    // vertex), else as many as the round's units need (one unit per wave).  The others leave at once and are not
    // counted, so a large grid costs little in rounds with a small frontier.
    const uint32_t units = (cs + 63) / 64 + cb;
    const uint32_t part = any_adv ? gridDim.x : max(1u, min(gridDim.x, (units + wpb - 1) / wpb));
    if (blockIdx.x >= part) return;
    const uint32_t wave_gid = blockIdx.x * wpb + w, nwaves = part * wpb;
    if (any_adv)
        advance_body(P, P.slot.thr, P.slot.thr_prev, P.slot.adv, R.r + 1, R.nxt, R.c_nxt, R.b, (int)R.b, wave_gid,
                     nwaves, &s_wave[w]);
    relax_round_body<NARROW>(P, R, P.slot.thr, cs, cb, &s_wave[w], wave_gid, nwaves);

    __syncthreads();
    if (threadIdx.x == 0) {  // the last workgroup of its group, then the last group, takes the decision
        __threadfence();
        const uint32_t ng = min(part, ROUND_GROUPS), grp = blockIdx.x % ng;
        const uint32_t gsize = (part - grp + ng - 1) / ng;  // workgroups with this residue
        uint32_t *gc = P.cnt->grp_done + grp * 32;
        s_last = 0;
        if (atomicAdd(gc, 1u) == gsize - 1) {
            *gc = 0;  // every workgroup of the group has counted: ready for the next round
            __threadfence();
            s_last = atomicAdd(&P.cnt->blocks_done, 1u) == ng - 1;
        }
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    if (threadIdx.x == 0) { s_adv = 0; s_act = 0; }
    __syncthreads();
    bool aa = false, act = false;
    const uint32_t nb = (r + 1) % 3u;
    for (uint32_t q = threadIdx.x; q < P.nslots; q += blockDim.x) {
        decide_slot(P, r, q, P.slot.thr, P.slot.thr_prev, P.slot.carry, P.slot.active, P.slot.adv, P.slot.done,
                    P.slot.advances, aa, act);
        P.near_mark[(size_t)nb * P.nslots + q] = 0;
        P.settle_mark[(size_t)nb * P.nslots + q] = 0;
        P.far_min[(size_t)nb * P.nslots + q] = DIST_INF;
    }
    if (aa) atomicOr(&s_adv, 1);
    if (act) atomicOr(&s_act, 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        P.cnt->s[(r + 2) % 3u] = 0;
        P.cnt->b[(r + 2) % 3u] = 0;
        P.cnt->blocks_done = 0;
        P.pass->any_adv = s_adv;
        if (!s_act) P.pass->all_done = 1;
        const uint32_t nr = next_round(r);
        P.pass->round = nr;
        st_agent(&P.pass->word, pass_word(nr, s_adv, !s_act, did));
        __threadfence();
    }
}

// ---------------------------------------------------------------- persistent

// Sense-counting grid barrier for a cooperative launch.  The arrival's
// acquire-release atomic publishes the workgroup's writes; the wait polls with
// relaxed loads and acquires once when it ends (an acquiring load in the loop
// would invalidate the L2 on every poll, slowing every other workgroup in
// proportion to the number waiting).  Gives up after a bounded spin (then
// every workgroup leaves the kernel).
DEVI bool grid_barrier(Counters *cn, uint32_t nblocks, PassCtl *pass, int *s_abort) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t g = __hip_atomic_load(&cn->bar_gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t arrived =
            __hip_atomic_fetch_add(&cn->bar_count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        int ab = 0;
        if (arrived == nblocks - 1) {
            __hip_atomic_store(&cn->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&cn->bar_gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            uint32_t spins = 0;
            while (__hip_atomic_load(&cn->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
                __builtin_amdgcn_s_sleep(2);
                if (++spins > (1u << 25) ||
                    __hip_atomic_load(&cn->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    atomicOr(&pass->err, ERR_BARRIER_TIMEOUT);
                    atomicExch(&cn->abort, 1u);
                    ab = 1;
                    break;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *s_abort = ab;
    }
    __syncthreads();
    return *s_abort == 0;
}

template <bool NARROW>
__global__ void __launch_bounds__(256) k_persistent(VorParams P, uint32_t max_rounds) {
    extern __shared__ __align__(16) unsigned char dyn_smem[];
    WaveScratch *s_wave = (WaveScratch *)dyn_smem;
    __shared__ uint64_t s_thr[PERSIST_SLOTS], s_thr_prev[PERSIST_SLOTS];
    __shared__ uint32_t s_carry[PERSIST_SLOTS], s_active[PERSIST_SLOTS], s_adv[PERSIST_SLOTS];
    __shared__ uint32_t s_done[PERSIST_SLOTS], s_advances[PERSIST_SLOTS];
    __shared__ int s_abort, s_any_adv, s_any_act;
    const uint32_t ns = P.nslots;
    for (uint32_t q = threadIdx.x; q < ns; q += blockDim.x) {
        s_thr[q] = P.slot.thr[q];
        s_thr_prev[q] = P.slot.thr_prev[q];
        s_carry[q] = P.slot.carry[q];
        s_active[q] = P.slot.active[q];
        s_adv[q] = 0;
        s_done[q] = P.slot.done[q];
        s_advances[q] = P.slot.advances[q];
    }
    __syncthreads();
    if (P.pass->all_done) return;
    uint32_t r = P.pass->round;
    const uint32_t wpb = blockDim.x / 64, w = threadIdx.x / 64;
    const uint32_t wave_gid = blockIdx.x * wpb + w, nwaves = gridDim.x * wpb;
    bool finished = false, ok = true;
    for (uint32_t it = 0; it < max_rounds; it++) {
        const RoundIdx R = round_idx(r);
        const uint32_t cs = min(ld_agent(&P.cnt->s[r % 3u]), P.cap_s);
        const uint32_t cb = min(ld_agent(&P.cnt->b[r % 3u]), P.cap_b);
        relax_round_body<NARROW>(P, R, s_thr, cs, cb, &s_wave[w], wave_gid, nwaves);
        if (blockIdx.x == 0) {
            const uint32_t nb = (r + 1) % 3u;
            for (uint32_t q = threadIdx.x; q < ns; q += blockDim.x) {
                P.near_mark[(size_t)nb * ns + q] = 0;
                P.settle_mark[(size_t)nb * ns + q] = 0;
                P.far_min[(size_t)nb * ns + q] = DIST_INF;
            }
            if (threadIdx.x == 0) {
                P.cnt->s[(r + 2) % 3u] = 0;
                P.cnt->b[(r + 2) % 3u] = 0;
            }
        }
        if (!(ok = grid_barrier(P.cnt, gridDim.x, P.pass, &s_abort))) break;
        if (threadIdx.x == 0) { s_any_adv = 0; s_any_act = 0; }
        __syncthreads();
        bool aa = false, act = false;
        for (uint32_t q = threadIdx.x; q < ns; q += blockDim.x)
            decide_slot(P, r, q, s_thr, s_thr_prev, s_carry, s_active, s_adv, s_done, s_advances, aa, act);
        if (aa) atomicOr(&s_any_adv, 1);
        if (act) atomicOr(&s_any_act, 1);
        __syncthreads();
        const bool any_adv = s_any_adv != 0, any_act = s_any_act != 0;
        if (any_adv) {
            advance_body(P, s_thr, s_thr_prev, s_adv, r + 1, (r + 1) & 1u, (r + 1) % 3u, (r + 1) % 3u, -1, wave_gid,
                         nwaves, &s_wave[w]);
            if (!(ok = grid_barrier(P.cnt, gridDim.x, P.pass, &s_abort))) break;
        }
        r = next_round(r);
        if (!any_act) {
            finished = true;
            break;
        }
    }
    if (blockIdx.x == 0) {
        for (uint32_t q = threadIdx.x; q < ns; q += blockDim.x) {
            P.slot.thr[q] = s_thr[q];
            P.slot.thr_prev[q] = s_thr_prev[q];
            P.slot.carry[q] = s_carry[q];
            P.slot.active[q] = s_active[q];
            P.slot.adv[q] = 0;
            P.slot.done[q] = s_done[q];
            P.slot.advances[q] = s_advances[q];
        }
        if (threadIdx.x == 0) {
            P.pass->round = r;
            if (finished) P.pass->all_done = 1;
            P.pass->any_adv = 0;
            P.pass->word = pass_word(r, 0, P.pass->all_done, NO_LAUNCH);
            (void)ok;
        }
    }
}

// ------------------------------------------------------------------ set-up

template <typename T>
__global__ void k_fill(T *p, uint64_t count, T value) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

__global__ void k_pass_reset(VorParams P) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) {
        P.pass->round = 0;
        P.pass->all_done = 1;  // no active query yet
        P.pass->any_adv = 0;
        P.pass->err = 0;
        P.pass->word = pass_word(0, 0, 1, NO_LAUNCH);
        for (int i = 0; i < 3; i++) { P.cnt->s[i] = 0; P.cnt->b[i] = 0; }
        P.cnt->bar_count = 0;
        P.cnt->bar_gen = 0;
        P.cnt->abort = 0;
        P.cnt->blocks_done = 0;
        for (int i = 0; i < EV_N; i++) P.cnt->ev[i] = 0;
        for (int i = 0; i < 4; i++) P.cnt->scan_ev[i] = 0;
    }
    for (uint32_t i = t; i < ROUND_GROUPS * 32; i += gridDim.x * blockDim.x) P.cnt->grp_done[i] = 0;
    for (uint32_t q = t; q < P.nslots; q += gridDim.x * blockDim.x) {
        for (int b = 0; b < 3; b++) {
            P.far_min[(size_t)b * P.nslots + q] = DIST_INF;
            P.near_mark[(size_t)b * P.nslots + q] = 0;
            P.settle_mark[(size_t)b * P.nslots + q] = 0;
        }
        P.slot.active[q] = 0;
        P.slot.done[q] = 0;
        P.slot.adv[q] = 0;
        P.slot.advances[q] = 0;
        P.slot.carry[q] = DIST_INF;
        P.slot.thr[q] = 0;
        P.slot.thr_prev[q] = 0;
    }
}

// Per-vertex state of one query: keys unreached, stamps and marks clear.
__global__ void k_slot_clear(uint64_t *key, uint32_t *aux, uint8_t *dirty, uint8_t *settled, uint32_t n,
                             uint32_t *heavy_pe, uint32_t nheavy) {
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        key[v] = KEY_INF;
        aux[v] = 0;
        dirty[v] = 0;
        settled[v] = 0;
    }
    for (uint32_t h = blockIdx.x * blockDim.x + threadIdx.x; h < nheavy; h += gridDim.x * blockDim.x)
        heavy_pe[h] = NONE;
}

// Seeds of one query (distinct; seed index = position) become the
// cells' roots (Alg. 3 initialisation) and the frontier of the current round.
__global__ void k_slot_seed(VorParams P, uint32_t slot, const uint32_t *seeds, uint32_t k) {
    const uint32_t r = P.pass->round;
    const RoundIdx R = round_idx(r);
    const uint32_t n = P.g.n;
    // wave-uniform loop: the list appends are aggregated per wave (one counter atomic per wave and list)
    for (uint32_t base = blockIdx.x * blockDim.x; base < k; base += gridDim.x * blockDim.x) {
        const uint32_t i = base + threadIdx.x;
        const bool on = i < k;
        uint32_t v = 0, deg = 0;
        if (on) {
            v = seeds[i];
            P.key[(size_t)slot * n + v] = (uint64_t)i;  // dist 0, seed index i
            P.aux[(size_t)slot * n + v] = r;
            deg = P.g.rp[v + 1] - P.g.rp[v];
        }
        append_s(P, R.cur, r % 3u, on && deg <= P.small_max, s_item(slot, v));
        append_b(P, R.cur, r % 3u, on && deg > P.small_max, slot, v, deg);
    }
    if (blockIdx.x != 0) return;
    if (threadIdx.x == 0) {
        P.slot.thr[slot] = P.delta == 0xFFFFFFFFu ? ~0ull : (uint64_t)P.delta;
        P.slot.thr_prev[slot] = 0;
        P.slot.carry[slot] = DIST_INF;
        P.slot.active[slot] = 1;
        P.slot.adv[slot] = 0;
        P.slot.done[slot] = 0;
        P.slot.advances[slot] = 0;
        for (int b = 0; b < 3; b++) {
            P.far_min[(size_t)b * P.nslots + slot] = DIST_INF;
            P.near_mark[(size_t)b * P.nslots + slot] = 0;
            P.settle_mark[(size_t)b * P.nslots + slot] = 0;
        }
        P.pass->all_done = 0;
        P.pass->word &= ~(1ull << 63);
    }
}

// ------------------------------------------------- pred + boundary scan

struct ScanWave {
    uint32_t incl[64];
    uint32_t beg[64];
    uint32_t row[64];
    uint32_t found[64];  // 1: the row needs no pred search (seed, unreached, or pred not wanted)
    uint32_t best[64];   // smallest caller id of a qualifying neighbour so far
    uint32_t rank[64];   // pair-table rank of the row's cell
    uint64_t key[64];
};

DEVI uint64_t pair_index(uint32_t i, uint32_t j) {  // i < j
    return (uint64_t)j * (j - 1) / 2 + i;
}

// Edge id of entry e: the caller's CSR offset of the edge's entry leaving
// its smaller caller id.  Each edge is scanned once, from its entry leaving
// the smaller (internal) id.
DEVI uint32_t edge_id(const DevGraph &g, uint32_t e) { return g.eo ? g.eo[e] : e; }

// Caller id of internal vertex v.
DEVI uint32_t caller_id(const DevGraph &g, uint32_t v) { return g.perm ? g.perm[v] : v; }
// Internal vertex of caller id c.
DEVI uint32_t internal_id(const DevGraph &g, uint32_t c) { return g.inv ? g.inv[c] : c; }

DEVI void set_err(uint32_t *err, uint32_t bit) {
    if (!(*err & bit)) atomicOr(err, bit);
}

// Cross-cell candidate of the edge of entry e, row -> u (row < u); ra is
// the pair-table rank of the row's cell.  The edge id is loaded only if the
// sum does not already lose to the pair's current entry.
// Returns 0 (no candidate), 1 (a candidate that lost to the entry) or 2 (an atomicMin issued).
DEVI int boundary_candidate(const DevGraph &g, uint64_t *pt, const uint32_t *tr, uint32_t *err, uint64_t krow,
                            uint32_t ra, uint64_t ku, uint32_t w, uint32_t e) {
    const uint32_t i1 = (uint32_t)krow, i2 = (uint32_t)ku;
    if (i1 == i2) return 0;
    const uint64_t bsum = (krow >> 32) + (uint64_t)w + (ku >> 32);
    if (bsum >= (1ull << 32)) {
        set_err(err, ERR_SUM_OVERFLOW);
        return 0;
    }
    const uint64_t rb = tr ? tr[i2] : i2, lo = min((uint64_t)ra, rb), hi = max((uint64_t)ra, rb);
    uint64_t *p = pt + hi * (hi - 1) / 2 + lo;
    const uint64_t cur = *p;
    if (bsum > (cur >> 32)) return 1;
    const uint64_t val = (bsum << 32) | edge_id(g, e);
    if (val >= cur) return 1;
    atomicMin((unsigned long long *)p, (unsigned long long)val);
    return 2;
}

// One wave scans the rows of group grp (64 consecutive vertices of at most
// scan_heavy entries each), 64 entries per step.  Every edge {a, b}, a < b,
// is a boundary candidate from row a.  With pred, every entry of a reached
// row gathers its neighbour's key and pred is the qualifying neighbour of
// smallest caller id; without, only entries a -> b with a < b do, unreached
// rows included, which still sees every edge once for the overflow test.
constexpr int SCAN_UNROLL = 4;

// Adds the wave's per-lane event counts to the scan counters (counting mode).
DEVI void scan_count(unsigned long long *ev, uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
    const uint32_t v[SCAN_EV_N] = {a, b, c, d};
#pragma unroll
    for (int i = 0; i < SCAN_EV_N; i++) {
        uint32_t x = v[i];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x += (uint32_t)__shfl_xor((int)x, o, 64);
        if (lane() == 0 && x) atomicAdd(ev + i, (unsigned long long)x);
    }
}

// REV: the lazy scan of a renumbered graph, each edge read from its larger id (the gathered keys are hub
// keys); COUNT: event counters.
template <bool REV, bool COUNT>
DEVI void scan_light_group(const ScanParams &S, const uint64_t *key, uint32_t *pred, uint64_t *pt, const uint32_t *tr,
                           uint32_t *err, uint32_t *heavy_pe, uint32_t grp, ScanWave *L) {
    const uint32_t n = S.g.n, ln = lane();
    const bool wp = !REV && S.with_pred != 0;
    constexpr bool rev = REV;
    const uint32_t row = grp * 64 + ln;
    uint64_t kv = KEY_INF;
    uint32_t beg = 0, deg = 0, found = 1;
    if (row < n) {
        kv = key[row];
        const uint32_t b0 = S.g.rp[row], d0 = S.g.rp[row + 1] - b0;
        if (d0 <= S.g.scan_heavy) {
            if (kv == KEY_INF) {
                if (wp) {
                    pred[row] = NONE;
                } else {
                    beg = b0;
                    deg = d0;
                }
            } else {
                beg = b0;
                deg = d0;
                if (wp) {
                    if ((kv >> 32) == 0) pred[row] = row;  // a seed is its own predecessor
                    else found = 0;
                }
            }
        }
    }
    const uint32_t incl = wave_incl_scan(deg);
    const uint32_t total = __shfl(incl, 63, 64);
    L->incl[ln] = incl;
    L->beg[ln] = beg;
    L->row[ln] = row;
    L->found[ln] = found;
    L->best[ln] = NONE;
    L->rank[ln] = (tr && kv != KEY_INF) ? tr[(uint32_t)kv] : (uint32_t)kv;
    L->key[ln] = kv;
    wave_sync();
    uint32_t n_ent = 0, n_gat = 0, n_cand = 0, n_atom = 0;  // event counts (counting mode)
    // SCAN_UNROLL independent 64-entry steps per iteration, each level's loads issued for all of them
    // before any is used (idle lanes read entry / vertex / slot 0), so one latency chain covers them all.
    for (uint32_t base = 0; base < total; base += 64 * SCAN_UNROLL) {
        bool valid[SCAN_UNROLL], side[SCAN_UNROLL], need[SCAN_UNROLL];
        uint32_t jj[SCAN_UNROLL], e[SCAN_UNROLL], u[SCAN_UNROLL], w[SCAN_UNROLL];
        uint64_t ku[SCAN_UNROLL];
#pragma unroll
        for (int s = 0; s < SCAN_UNROLL; s++) {
            const uint32_t t = base + 64 * s + ln;
            valid[s] = t < total;
            uint32_t j = 0;
            if (valid[s]) {
                uint32_t lo = 0, hi = 63;
                while (lo < hi) {
                    uint32_t mid = (lo + hi) >> 1;
                    if (L->incl[mid] > t) hi = mid; else lo = mid + 1;
                }
                j = lo;
            }
            const uint32_t ex = j ? L->incl[j - 1] : 0;
            jj[s] = j;
            e[s] = valid[s] ? L->beg[j] + (t - ex) : 0u;
        }
#pragma unroll
        for (int s = 0; s < SCAN_UNROLL; s++) {
            const uint2 a = S.g.adj[e[s]];
            u[s] = a.x;
            w[s] = a.y;
        }
#pragma unroll
        for (int s = 0; s < SCAN_UNROLL; s++) {
            side[s] = valid[s] && (rev ? u[s] < L->row[jj[s]] : L->row[jj[s]] < u[s]);
            need[s] = valid[s] && (wp || side[s]);
            ku[s] = key[need[s] ? u[s] : 0u];
        }
#pragma unroll
        for (int s = 0; s < SCAN_UNROLL; s++) {
            const uint64_t kr = L->key[jj[s]];
            if (!need[s]) ku[s] = KEY_INF;
            else if ((ku[s] == KEY_INF) != (kr == KEY_INF)) set_err(err, ERR_DIST_OVERFLOW);
            if (wp && valid[s] && !L->found[jj[s]] && ku[s] != KEY_INF && (uint32_t)ku[s] == (uint32_t)kr &&
                (ku[s] >> 32) + w[s] == (kr >> 32))
                atomicMin(&L->best[jj[s]], caller_id(S.g, u[s]));
            // reversed: this row may be the pred of a heavy neighbour (heavy rows are the ids below nheavy)
            if (rev && u[s] < S.g.nheavy && ku[s] != KEY_INF && kr != KEY_INF && (uint32_t)ku[s] == (uint32_t)kr &&
                (kr >> 32) + w[s] == (ku[s] >> 32))
                atomicMin(heavy_pe + u[s], caller_id(S.g, L->row[jj[s]]));
        }
        // boundary candidates: the pair slots, then the current values, then the winners' atomics
        uint64_t *slot[SCAN_UNROLL], bsum[SCAN_UNROLL], cur[SCAN_UNROLL];
        bool cand[SCAN_UNROLL];
#pragma unroll
        for (int s = 0; s < SCAN_UNROLL; s++) {
            const uint64_t kr = L->key[jj[s]];
            const uint32_t i1 = (uint32_t)kr, i2 = (uint32_t)ku[s];
            cand[s] = side[s] && ku[s] != KEY_INF && kr != KEY_INF && i1 != i2;
            bsum[s] = (kr >> 32) + (uint64_t)w[s] + (ku[s] >> 32);
            if (cand[s] && bsum[s] >= (1ull << 32)) {
                set_err(err, ERR_SUM_OVERFLOW);
                cand[s] = false;
            }
            const uint64_t ra = L->rank[jj[s]], rb = tr ? tr[cand[s] ? i2 : 0u] : i2;
            const uint64_t lo = min(ra, rb), hi = max(ra, rb);
            slot[s] = pt + (cand[s] ? hi * (hi - 1) / 2 + lo : 0u);
        }
#pragma unroll
        for (int s = 0; s < SCAN_UNROLL; s++) cur[s] = *slot[s];
#pragma unroll
        for (int s = 0; s < SCAN_UNROLL; s++) {
            if (COUNT) {
                n_ent += valid[s];
                n_gat += need[s];
                n_cand += cand[s];
            }
            if (!cand[s] || bsum[s] > (cur[s] >> 32)) continue;
            const uint64_t val = (bsum[s] << 32) | edge_id(S.g, e[s]);
            if (val < cur[s]) {
                atomicMin((unsigned long long *)slot[s], (unsigned long long)val);
                if (COUNT) n_atom++;
            }
        }
    }
    wave_sync();
    if (wp && !found) pred[row] = L->best[ln] == NONE ? NONE : internal_id(S.g, L->best[ln]);
    if (COUNT) scan_count(S.ev, n_ent, n_gat, n_cand, n_atom);
}

// One wave scans one chunk of a row above scan_heavy: boundary candidates and
// the smallest caller id of a qualifying neighbour (atomicMin into heavy_pe).
// An unreached row only checks its edges a -> b, a < b, for the overflow test
// (without pred; with pred every reached row checks all of its own entries).
template <bool REV, bool COUNT>
DEVI void scan_heavy_chunk(const ScanParams &S, const uint64_t *key, uint64_t *pt, const uint32_t *tr, uint32_t *err,
                           uint32_t *heavy_pe, uint32_t lc) {
    // heavy row h owning chunk lc: largest h with heavy_chunk_off[h] <= lc
    uint32_t lo = 0, hi = S.g.nheavy;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (S.g.heavy_chunk_off[mid] <= lc) lo = mid; else hi = mid;
    }
    const uint32_t h = lo, row = S.g.heavy_rows[h];
    const uint32_t c = lc - S.g.heavy_chunk_off[h];
    const uint64_t kv = key[row];
    if (kv == KEY_INF && S.with_pred) return;
    const uint32_t beg = S.g.rp[row] + c * S.g.scan_chunk;
    const uint32_t lim = S.g.rp[row + 1];
    const uint32_t end = (lim - beg > S.g.scan_chunk) ? beg + S.g.scan_chunk : lim;
    uint32_t n_ent = 0, n_gat = 0, n_cand = 0, n_atom = 0;  // event counts (counting mode)
    if (REV) {
        // Each edge is read from its larger id, so this row takes only its entries to smaller ids (other heavy
        // rows; a sorted prefix of the row): candidates, the overflow test, and the pred minima of both ends
        // (every entry to a larger id is seen from that neighbour's row).
        const bool is_seed = kv != KEY_INF && (kv >> 32) == 0;
        const uint32_t ra = (tr && kv != KEY_INF) ? tr[(uint32_t)kv] : (uint32_t)kv;
        uint32_t best = NONE;
        for (uint32_t e0 = beg; e0 < end; e0 += 64) {
            const uint32_t e = e0 + lane();
            const uint2 a = S.g.adj[e < end ? e : beg];
            const bool on = e < end && a.x < row;
            if (__ballot(on) == 0) break;  // sorted row: the rest is above row
            if (!on) continue;
            n_ent++;
            n_gat++;
            const uint64_t ku = key[a.x];
            if ((ku == KEY_INF) != (kv == KEY_INF)) {
                set_err(err, ERR_DIST_OVERFLOW);
                continue;
            }
            if (kv == KEY_INF) continue;
            if ((uint32_t)ku == (uint32_t)kv) {
                if (!is_seed && (ku >> 32) + a.y == (kv >> 32)) best = min(best, caller_id(S.g, a.x));
                if ((kv >> 32) + a.y == (ku >> 32)) atomicMin(heavy_pe + a.x, caller_id(S.g, row));
            } else {
                const int c = boundary_candidate(S.g, pt, tr, err, kv, ra, ku, a.y, e);
                n_cand += c != 0;
                n_atom += c == 2;
            }
        }
        best = wave_min(best);
        if (lane() == 0 && best != NONE) atomicMin(heavy_pe + h, best);
        if (COUNT) scan_count(S.ev, n_ent, n_gat, n_cand, n_atom);
        return;
    }
    if (kv == KEY_INF) {
        for (uint32_t e0 = beg; e0 < end; e0 += 64) {
            const uint32_t e = e0 + lane();
            if (e < end) {
                const uint32_t u = S.g.adj[e].x;
                n_ent++;
                if (row < u) {
                    n_gat++;
                    if (key[u] != KEY_INF) set_err(err, ERR_DIST_OVERFLOW);
                }
            }
        }
        if (COUNT) scan_count(S.ev, n_ent, n_gat, 0, 0);
        return;
    }
    const bool is_seed = (kv >> 32) == 0;
    const uint32_t ra = tr ? tr[(uint32_t)kv] : (uint32_t)kv;
    uint32_t best = NONE;
    for (uint32_t e0 = beg; e0 < end; e0 += 64) {
        const uint32_t e = e0 + lane();
        if (e < end) {
            const uint2 a = S.g.adj[e];
            const uint64_t ku = key[a.x];
            n_ent++;
            n_gat++;
            if (ku == KEY_INF) {
                set_err(err, ERR_DIST_OVERFLOW);
            } else {
                if (!is_seed && (uint32_t)ku == (uint32_t)kv && (ku >> 32) + a.y == (kv >> 32))
                    best = min(best, caller_id(S.g, a.x));
                if (row < a.x) {
                    const int c = boundary_candidate(S.g, pt, tr, err, kv, ra, ku, a.y, e);
                    n_cand += c != 0;
                    n_atom += c == 2;
                }
            }
        }
    }
    best = wave_min(best);
    if (lane() == 0 && best != NONE) atomicMin(heavy_pe + h, best);
    if (COUNT) scan_count(S.ev, n_ent, n_gat, n_cand, n_atom);
}

template <bool REV, bool COUNT>
__global__ void __launch_bounds__(256) k_scan(ScanParams S) {
    __shared__ ScanWave s_wave[4];
    const uint32_t n = S.g.n;
    const uint32_t wpb = blockDim.x / 64, w = threadIdx.x / 64;
    const uint64_t nwaves = (uint64_t)gridDim.x * wpb;
    const uint32_t ngroups = (n + 63) / 64;
    const uint64_t per_slot = (uint64_t)ngroups + S.g.nheavy_chunks;
    const uint64_t units = per_slot * S.nscan;
    for (uint64_t u = (uint64_t)blockIdx.x * wpb + w; u < units; u += nwaves) {
        const uint32_t si = (uint32_t)(u / per_slot);
        const uint32_t lu = (uint32_t)(u % per_slot);
        const uint32_t slot = S.slot_ids[si];
        const uint64_t *key = S.key + (size_t)slot * n;
        uint64_t *pt = S.pt[slot];
        const uint32_t *tr = S.tr ? S.tr[slot] : nullptr;
        uint32_t *err = S.slot_err + slot;
        if (lu < ngroups)
            scan_light_group<REV, COUNT>(S, key, S.aux + (size_t)slot * n, pt, tr, err,
                                         S.heavy_pe + (size_t)slot * S.g.nheavy, lu, &s_wave[w]);
        else
            scan_heavy_chunk<REV, COUNT>(S, key, pt, tr, err, S.heavy_pe + (size_t)slot * S.g.nheavy, lu - ngroups);
    }
}

// pred of heavy rows from the smallest caller id of a qualifying neighbour.
__global__ void k_scan_heavy_pred(ScanParams S) {
    const uint32_t n = S.g.n, nh = S.g.nheavy;
    const uint64_t total = (uint64_t)nh * S.nscan;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t slot = S.slot_ids[t / nh], h = (uint32_t)(t % nh);
        const uint32_t row = S.g.heavy_rows[h];
        const uint64_t kv = S.key[(size_t)slot * n + row];
        uint32_t p;
        if (kv == KEY_INF) p = NONE;
        else if ((kv >> 32) == 0) p = row;
        else {
            const uint32_t c = S.heavy_pe[(size_t)slot * nh + h];
            p = c == NONE ? NONE : internal_id(S.g, c);
        }
        S.aux[(size_t)slot * n + row] = p;
    }
}

// --------------------------------------------------------- G'1 compaction

DEVI void pair_of(uint32_t p, uint32_t *i, uint32_t *j);

// G'1 extraction: the finite entries of each query's pair table, as (pair
// index in seed-index order, value).  A workgroup takes tiles of 1024 entries
// (each lane four, coalesced) and reserves its output slots with one atomic
// per tile.
__global__ void __launch_bounds__(256) k_compact(CompactParams C) {
    __shared__ uint32_t s_wave_sum[4];
    __shared__ uint32_t s_base;
    const uint32_t wv = threadIdx.x / 64;
    for (uint32_t si = 0; si < C.nscan; si++) {
        const uint32_t slot = C.slot_ids[si];
        const uint64_t *pt = C.pt[slot];
        const uint32_t *ts = C.ts ? C.ts[slot] : nullptr;
        uint64_t *ov = C.out_val[slot];
        const uint64_t len = C.pt_len[slot];
        const uint64_t tiles = (len + 1023) / 1024;
        for (uint64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {  // uniform per workgroup
            uint64_t val[4];
            uint32_t cnt = 0;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const uint64_t i = tile * 1024 + (uint64_t)j * 256 + threadIdx.x;
                val[j] = i < len ? pt[i] : KEY_INF;
                cnt += val[j] != KEY_INF;
            }
            const uint32_t incl = wave_incl_scan(cnt);
            if (lane() == 63) s_wave_sum[wv] = incl;
            __syncthreads();
            uint32_t before = 0, total = 0;
            for (uint32_t i = 0; i < blockDim.x / 64; i++) {
                if (i < wv) before += s_wave_sum[i];
                total += s_wave_sum[i];
            }
            if (threadIdx.x == 0 && total) s_base = atomicAdd(&C.out_cnt[slot], total);
            __syncthreads();
            if (cnt) {
                uint32_t pos = s_base + before + incl - cnt;
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    if (val[j] == KEY_INF) continue;
                    if (pos < C.out_cap[slot]) {
                        uint32_t q = (uint32_t)(tile * 1024 + (uint64_t)j * 256 + threadIdx.x);
                        if (ts) {  // table slot -> pair index of the two seed indices
                            uint32_t a, b;
                            pair_of(q, &a, &b);
                            const uint32_t x = ts[a], y = ts[b];
                            q = (uint32_t)pair_index(min(x, y), max(x, y));
                        }
                        C.out_idx[slot][pos] = q;
                        if (ov) ov[pos] = val[j];
                    } else {
                        atomicOr(&C.pass->err, ERR_LIST_OVERFLOW);
                    }
                    pos++;
                }
            }
            __syncthreads();
        }
    }
}

// --------------------------------------------------------------- expansion

// Alg. 2 Steps 5-6 on the pred forest: the tree is every chosen cross-cell
// edge plus, from both of its endpoints, every edge (x, pred(x)) up to the
// cell's seed.  Walks claim the vertices they pass and find their preds; one
// pass over the marks then writes each claimed vertex's edge once, which is
// the set semantics of E_S, and clears the marks.

DEVI void emit_edges(const ExpandParams &E, bool on, uint32_t x, uint32_t y, uint32_t w) {
    const uint64_t m = __ballot(on);
    if (!m) return;
    const uint32_t leader = (uint32_t)__ffsll((unsigned long long)m) - 1;
    uint32_t pos = 0;
    if (lane() == leader) pos = atomicAdd(E.ocnt, (uint32_t)__popcll(m));
    pos = __shfl(pos, leader, 64) + lanes_below(m);
    if (on && pos < E.g.n) {
        x = caller_id(E.g, x);
        y = caller_id(E.g, y);
        E.oa[pos] = min(x, y);
        E.ob[pos] = max(x, y);
        E.ow[pos] = w;
    }
}

// Row of CSR offset e: the largest r with rp[r] <= e, by a 64-way search
// (each step probes 64 offsets, one per lane).  Wave-uniform result.
DEVI uint32_t wave_row_of(const DevGraph &g, uint32_t e) {
    uint32_t lo = 0, hi = g.n;  // rp[lo] <= e < rp[hi]
    while (hi - lo > 1) {
        const uint32_t span = hi - lo;
        const uint32_t probe = lo + (uint32_t)(((uint64_t)span * lane()) >> 6);
        const bool ok = lane() == 0 || g.rp[probe] <= e;
        const uint64_t m = __ballot(ok);
        const uint32_t jm = 63u - (uint32_t)__clzll((long long)m);
        const uint32_t nlo = __shfl(probe, (int)jm, 64);
        const uint32_t nhi = jm == 63 ? hi : __shfl(probe, (int)jm + 1, 64);
        lo = nlo;
        hi = nhi;
    }
    return lo;
}

// pred of reached non-seed vertex x (key kx): rows above scan_heavy have it
// from the scan; smaller rows are scanned here, 64 entries per step, for the
// neighbour of smallest caller id in the same cell on a shortest path (in the
// caller's order, rows sorted by column, the first qualifying entry).
// Wave-uniform result, NONE if there is none.
DEVI uint32_t wave_pred_of(const ExpandParams &E, uint32_t x, uint64_t kx) {
    const uint32_t beg = E.g.rp[x], deg = E.g.rp[x + 1] - beg;
    if (deg > E.g.scan_heavy) return E.pred[x];
    if (E.g.perm) {
        uint32_t best = NONE;
        for (uint32_t c = 0; c < deg; c += 64) {
            const uint32_t i = c + lane();
            if (i < deg) {
                const uint2 a = E.g.adj[beg + i];
                const uint64_t ku = E.key[a.x];
                if (ku != KEY_INF && (uint32_t)ku == (uint32_t)kx && (ku >> 32) + a.y == (kx >> 32))
                    best = min(best, E.g.perm[a.x]);
            }
        }
        best = wave_min(best);
        return best == NONE ? NONE : E.g.inv[best];
    }
    for (uint32_t c = 0; c < deg; c += 64) {
        const uint32_t i = c + lane();
        bool q = false;
        uint32_t u = 0;
        if (i < deg) {
            const uint2 a = E.g.adj[beg + i];
            u = a.x;
            const uint64_t ku = E.key[u];
            q = ku != KEY_INF && (uint32_t)ku == (uint32_t)kx && (ku >> 32) + a.y == (kx >> 32);
        }
        const uint64_t m = __ballot(q);
        if (m) return __shfl(u, __ffsll((unsigned long long)m) - 1, 64);
    }
    return NONE;
}

// One wave per walk: walk 2q starts at the row end of chosen edge q (and
// writes that edge), walk 2q+1 at its column end.  A walk claims each vertex
// it reaches (a byte of mark); the first walk to claim a vertex finds its
// pred and goes on, a later one stops there, since the rest of the path is
// the same.  Claimed vertices get their pred in E.pred.
__global__ void __launch_bounds__(256) k_expand_walk(ExpandParams E) {
    const uint32_t wid = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    const uint32_t q = wid >> 1, end = wid & 1u, n = E.g.n;
    const bool live = q < *E.nsel;
    uint32_t x = 0, v = 0, w = 0;
    if (live) {
        const uint32_t e = E.g.onew ? E.g.onew[E.sel_e[q]] : E.sel_e[q];
        const uint2 a = E.g.adj[e];
        v = a.x;
        w = a.y;
        x = end == 0 ? wave_row_of(E.g, e) : a.x;
    }
    emit_edges(E, live && end == 0 && lane() == 0, x, v, w);
    if (!live) return;
    for (uint32_t steps = 0; steps < n; steps++) {
        const uint64_t kx = E.key[x];
        if ((kx >> 32) == 0 || kx == KEY_INF) break;  // the seed (an unreached vertex cannot occur)
        const uint32_t bit = 1u << (8 * (x & 3u));
        uint32_t old = 0;
        if (lane() == 0) old = atomicOr(E.mark + (x >> 2), bit);
        old = __shfl(old, 0, 64);
        if (old & bit) break;  // another walk goes on from here
        const uint32_t p = wave_pred_of(E, x, kx);
        if (lane() == 0) E.pred[x] = p;
        if (p >= n) break;  // cannot happen for a converged pass; the emit pass skips x
        x = p;
    }
}

// With every pred known: two threads per chosen edge, thread 2q starting at
// the row end (and writing the edge), 2q+1 at the column end; a walk only
// sets the marks of the vertices it passes (one dependent load per step).
__global__ void __launch_bounds__(256) k_expand_walk_ready(ExpandParams E) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t q = t >> 1, end = t & 1u, n = E.g.n;
    const bool live = q < *E.nsel;
    uint32_t x = 0, v = 0, w = 0;
    if (live) {
        const uint32_t e = E.g.onew ? E.g.onew[E.sel_e[q]] : E.sel_e[q];
        const uint2 a = E.g.adj[e];
        v = a.x;
        w = a.y;
        x = a.x;
        if (end == 0) {
            uint32_t lo = 0, hi = n;  // rp[lo] <= e < rp[hi]
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (E.g.rp[mid] <= e) lo = mid; else hi = mid;
            }
            x = lo;
        }
    }
    emit_edges(E, live && end == 0, x, v, w);
    if (!live) return;
    for (uint32_t steps = 0; steps < n; steps++) {
        const uint32_t p = E.pred[x];
        if (p == x || p >= n) break;  // the seed (or, never for a converged pass, an unreached vertex)
        ((uint8_t *)E.mark)[x] = 1;
        x = p;
    }
}

// Writes the edge (x, pred x) of every marked vertex and clears the marks.
// Each thread covers one 4-vertex mark word; a workgroup reserves the output
// slots of its whole tile with one atomic.
__global__ void __launch_bounds__(256) k_expand_emit(ExpandParams E) {
    __shared__ uint32_t s_wave_sum[4];
    __shared__ uint32_t s_base;
    const uint32_t n = E.g.n, words = (n + 3) / 4;
    const uint32_t stride = gridDim.x * blockDim.x;
    const uint32_t wv = threadIdx.x / 64;
    for (uint32_t base = blockIdx.x * blockDim.x; base < words; base += stride) {  // uniform trip count
        const uint32_t t = base + threadIdx.x;
        const uint32_t word = t < words ? E.mark[t] : 0u;
        uint32_t px[4], wx[4], cnt = 0;
        if (word) {
            E.mark[t] = 0u;
#pragma unroll
            for (uint32_t b = 0; b < 4; b++) {
                px[b] = NONE;
                if ((word >> (8 * b)) & 0xFFu) {
                    const uint32_t x = 4 * t + b;
                    const uint32_t p = E.pred[x];
                    if (p < n) {
                        px[b] = p;
                        wx[b] = (uint32_t)((E.key[x] >> 32) - (E.key[p] >> 32));
                        cnt++;
                    }
                }
            }
        }
        const uint32_t incl = wave_incl_scan(cnt);
        if (lane() == 63) s_wave_sum[wv] = incl;
        __syncthreads();
        uint32_t before = 0, total = 0;
        for (uint32_t i = 0; i < blockDim.x / 64; i++) {
            if (i < wv) before += s_wave_sum[i];
            total += s_wave_sum[i];
        }
        if (threadIdx.x == 0 && total) s_base = atomicAdd(E.ocnt, total);
        __syncthreads();
        if (cnt) {
            uint32_t pos = s_base + before + incl - cnt;
#pragma unroll
            for (uint32_t b = 0; b < 4; b++) {
                if (!((word >> (8 * b)) & 0xFFu) || px[b] >= n) continue;
                const uint32_t x = 4 * t + b;
                if (pos < n) {
                    const uint32_t cx = caller_id(E.g, x), cp = caller_id(E.g, px[b]);
                    E.oa[pos] = min(cx, cp);
                    E.ob[pos] = max(cx, cp);
                    E.ow[pos] = wx[b];
                }
                pos++;
            }
        }
        __syncthreads();  // s_wave_sum and s_base are reused by the next tile
    }
}

// ------------------------------------------------------------ MST of G'1

DEVI void pair_of(uint32_t p, uint32_t *i, uint32_t *j) {  // inverse of j(j-1)/2 + i, i < j
    uint32_t jj = (uint32_t)((1.0 + sqrt(1.0 + 8.0 * (double)p)) * 0.5);
    while ((uint64_t)jj * (jj - 1) / 2 > p) jj--;
    while ((uint64_t)(jj + 1) * jj / 2 <= p) jj++;
    *j = jj;
    *i = p - (uint32_t)((uint64_t)jj * (jj - 1) / 2);
}

// Row-major rank of pair (i, j), i < j < k, among all such pairs, and its inverse.
DEVI uint64_t row_start(uint64_t i, uint64_t k) { return i * (2 * k - i - 1) / 2; }
DEVI uint32_t rank_of(uint32_t i, uint32_t j, uint32_t k) { return (uint32_t)(row_start(i, k) + (j - i - 1)); }
DEVI void rank_pair(uint32_t r, uint32_t k, uint32_t *i, uint32_t *j) {
    const double a = 2.0 * k - 1.0;
    double f = (a - sqrt(a * a - 8.0 * (double)r)) * 0.5;
    int64_t ii = f < 0.0 ? 0 : (int64_t)f;
    if (ii > (int64_t)k - 2) ii = (int64_t)k - 2;
    while (ii > 0 && row_start((uint64_t)ii, k) > r) ii--;
    while (ii + 1 <= (int64_t)k - 2 && row_start((uint64_t)ii + 1, k) <= r) ii++;
    *i = (uint32_t)ii;
    *j = (uint32_t)(r - row_start((uint64_t)ii, k) + (uint64_t)ii + 1);
}

// atomicMin(best + root, key) for every lane with `on`.  Late rounds send many
// edges to few roots, so the lanes sharing the roots of the first two pending
// lanes are combined in the wave first (one atomic per such root).
DEVI void wave_min_to_root(unsigned long long *best, uint32_t root, unsigned long long key, bool on) {
    uint64_t pending = __ballot(on);
    for (int it = 0; it < 2 && pending; it++) {
        const uint32_t leader = (uint32_t)__ffsll((unsigned long long)pending) - 1;
        const uint32_t r = __shfl(root, (int)leader, 64);
        const bool mine = on && root == r;
        const uint64_t peers = __ballot(mine);
        unsigned long long v = mine ? key : ~0ull;
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) {
            const unsigned long long o = __shfl_xor(v, d, 64);
            v = o < v ? o : v;
        }
        if (lane() == leader && v < best[r]) atomicMin(best + r, v);
        if (mine) on = false;
        pending &= ~peers;
    }
    if (on && key < best[root]) atomicMin(best + root, key);
}

__global__ void k_mst_init(MstParams M, const uint32_t *g1_idx, uint32_t m) {
    const uint32_t t0 = blockIdx.x * blockDim.x + threadIdx.x, st = gridDim.x * blockDim.x;
    for (uint32_t c = t0; c < M.k; c += st) {
        M.par[c] = c;
        M.best[c] = ~0ull;
    }
    for (uint32_t t = t0; t < m; t += st) M.edges[0][t] = g1_idx[t];
    if (t0 == 0) {
        M.hdr[0] = m;
        M.hdr[1] = 0;
        M.hdr[2] = 0;
        M.hdr[3] = 0;
    }
}

// Every edge still joining two components offers its key to both roots and
// moves to the other list; edges inside a component are dropped.
__global__ void __launch_bounds__(256) k_mst_edges(MstParams M, uint32_t in) {
    const uint32_t out = in ^ 1u;
    const uint32_t m = M.hdr[in];
    const uint32_t st = gridDim.x * blockDim.x;
    for (uint32_t base = blockIdx.x * blockDim.x; base < m; base += st) {
        const uint32_t t = base + threadIdx.x;
        bool live = false;
        uint32_t p = 0, ci = 0, cj = 0;
        unsigned long long key = 0;
        if (t < m) {
            p = M.edges[in][t];
            uint32_t i, j;
            pair_of(p, &i, &j);
            ci = M.par[i];
            cj = M.par[j];
            if (ci != cj) {
                live = true;
                key = ((M.pt[pair_slot(M.tr, i, j)] >> 32) << 32) | rank_of(i, j, M.k);
            }
        }
        wave_min_to_root(M.best, ci, key, live);
        wave_min_to_root(M.best, cj, key, live);
        const uint64_t mk = __ballot(live);
        if (mk) {
            const uint32_t leader = (uint32_t)__ffsll((unsigned long long)mk) - 1;
            uint32_t pos = 0;
            if (lane() == leader) pos = atomicAdd(M.hdr + out, (uint32_t)__popcll(mk));
            pos = __shfl(pos, leader, 64);
            if (live) M.edges[out][pos + lanes_below(mk)] = p;
        }
    }
}

// One workgroup: each root hooks under the root at the other end of its
// lightest edge and records that edge; when two roots chose the same edge
// only the smaller records it and only the larger hooks.  With distinct keys
// those 2-cycles are the only cycles, so pointer jumping flattens the hooks
// into trees, every seed then takes its new root, and the minima are reset.
DEVI void mst_merge_body(const MstParams &M, int *s_changed) {
    const uint32_t k = M.k;
    for (uint32_t c = threadIdx.x; c < k; c += blockDim.x) {
        uint32_t h = c;
        const unsigned long long b = M.best[c];
        if (M.par[c] == c && b != ~0ull) {
            uint32_t i, j;
            rank_pair((uint32_t)b, k, &i, &j);
            const uint32_t ci = M.par[i], cj = M.par[j];
            const uint32_t other = ci == c ? cj : ci;
            const bool mutual = M.best[other] == b;
            if (!mutual || c < other) {
                const uint32_t pos = atomicAdd(M.hdr + 2, 1u);
                if (pos < k) M.sel[pos] = (uint32_t)M.pt[pair_slot(M.tr, i, j)];
            }
            if (!mutual || c > other) h = other;
        }
        M.hook[c] = h;
    }
    __syncthreads();
    for (;;) {
        if (threadIdx.x == 0) *s_changed = 0;
        __syncthreads();
        for (uint32_t c = threadIdx.x; c < k; c += blockDim.x) {
            const uint32_t h = M.hook[c], hh = M.hook[h];
            if (hh != h) {
                M.hook[c] = hh;
                *s_changed = 1;
            }
        }
        __syncthreads();
        const int changed = *s_changed;
        __syncthreads();
        if (!changed) break;
    }
    for (uint32_t c = threadIdx.x; c < k; c += blockDim.x) M.par[c] = M.hook[M.par[c]];
    for (uint32_t c = threadIdx.x; c < k; c += blockDim.x) M.best[c] = ~0ull;
    __syncthreads();
}

__global__ void __launch_bounds__(1024) k_mst_merge(MstParams M, uint32_t in) {
    __shared__ int s_changed;
    mst_merge_body(M, &s_changed);
    if (threadIdx.x == 0) M.hdr[in] = 0;
}

// The whole Borůvka in one workgroup, for a small G'1: the same steps as
// k_mst_edges + k_mst_merge per round, with the list counts in LDS.
__global__ void __launch_bounds__(1024) k_mst_small(MstParams M, const uint32_t *g1_idx, uint32_t m, uint32_t rounds) {
    __shared__ uint32_t s_cnt[2];
    __shared__ int s_changed;
    for (uint32_t c = threadIdx.x; c < M.k; c += blockDim.x) {
        M.par[c] = c;
        M.best[c] = ~0ull;
    }
    if (threadIdx.x == 0) {
        s_cnt[0] = m;
        s_cnt[1] = 0;
        M.hdr[0] = M.hdr[1] = M.hdr[2] = M.hdr[3] = 0;
    }
    __syncthreads();
    uint32_t in = 0;
    for (uint32_t r = 0; r <= rounds; r++) {
        const uint32_t cnt = s_cnt[in], out = in ^ 1u;
        if (cnt == 0) break;  // uniform: read after a barrier
        const uint32_t *src = r == 0 ? g1_idx : M.edges[in];
        for (uint32_t base = 0; base < cnt; base += blockDim.x) {
            const uint32_t t = base + threadIdx.x;
            bool live = false;
            uint32_t p = 0, ci = 0, cj = 0;
            unsigned long long key = 0;
            if (t < cnt) {
                p = src[t];
                uint32_t i, j;
                pair_of(p, &i, &j);
                ci = M.par[i];
                cj = M.par[j];
                if (ci != cj) {
                    live = true;
                    key = ((M.pt[pair_slot(M.tr, i, j)] >> 32) << 32) | rank_of(i, j, M.k);
                }
            }
            wave_min_to_root(M.best, ci, key, live);
            wave_min_to_root(M.best, cj, key, live);
            const uint64_t mk = __ballot(live);
            if (mk) {
                const uint32_t leader = (uint32_t)__ffsll((unsigned long long)mk) - 1;
                uint32_t pos = 0;
                if (lane() == leader) pos = atomicAdd(&s_cnt[out], (uint32_t)__popcll(mk));
                pos = __shfl(pos, leader, 64);
                if (live) M.edges[out][pos + lanes_below(mk)] = p;
            }
        }
        __syncthreads();
        mst_merge_body(M, &s_changed);
        if (threadIdx.x == 0) s_cnt[in] = 0;
        __syncthreads();
        in = out;
    }
}

// ------------------------------------------- cluster-local relaxation
// One query (driver 3).  A vertex is active in an activation of its cluster
// when its key is below the key its edges were last relaxed with
// (expanded).  The workgroup copies the cluster's keys into LDS, relaxes the
// internal edges of active members sweep by sweep (LDS 64-bit atomicMin; a
// member improved in a sweep is active in the next) until a sweep improves
// nothing, writes the keys back with atomicMin, relaxes the external edges of
// every member it touched with its final key (global atomicMin; a target
// that improves gets its cluster listed once for the next round) and records
// the keys as expanded.  The fixed point is the same unique one: a key that
// drops, from inside or outside, always gets all of its edges relaxed again.

__global__ void k_cluster_start(ClusterParams C, const uint32_t *seeds, uint32_t k) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
        const uint32_t c = C.cl_of[seeds[i]];
        if (atomicExch(C.stamp + c, 1u) != 1u) {
            const uint32_t pos = atomicAdd(&C.ctl->cnt[0], 1u);
            if (pos < C.nclusters) C.list[0][pos] = c;
            else atomicOr(&C.ctl->err, 1u);
        }
    }
}

__global__ void __launch_bounds__(256) k_cluster_round(ClusterParams C) {
    __shared__ uint64_t lkey[CLUSTER_MAX];
    __shared__ uint2 ladj[CLUSTER_EDGES];          // the cluster's internal edges (local target, w)
    __shared__ uint16_t lrp[CLUSTER_MAX + 1];      // member i's internal edges: ladj[lrp[i], lrp[i+1])
    __shared__ uint8_t act[2][CLUSTER_MAX];
    __shared__ uint8_t touched[CLUSTER_MAX];
    __shared__ int s_changed[2];
    __shared__ int s_last;
    if (ld_agent(&C.ctl->done)) return;
    const uint32_t r = ld_agent(&C.ctl->round);
    const uint32_t cur = r & 1u, nxt = cur ^ 1u;
    const uint32_t ncur = min(ld_agent(&C.ctl->cnt[r % 3u]), C.nclusters);
    uint32_t *cnt_next = &C.ctl->cnt[(r + 1) % 3u];
    const uint32_t tag = r + 2;  // stamp of a listing for round r + 1
    for (uint32_t it = blockIdx.x; it < ncur; it += gridDim.x) {
        const uint32_t c = C.list[cur][it];
        const uint32_t b = C.cstart[c], m = min(C.cstart[c + 1] - b, CLUSTER_MAX);
        const uint32_t e0 = C.irp[b], ne = min(C.irp[b + m] - e0, CLUSTER_EDGES);
        for (uint32_t j = threadIdx.x; j < ne; j += blockDim.x) ladj[j] = C.ie[e0 + j];
        for (uint32_t i = threadIdx.x; i <= m; i += blockDim.x) lrp[i] = (uint16_t)min(C.irp[b + i] - e0, ne);
        for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) {
            const uint32_t v = C.members[b + i];
            const uint64_t kv = ld_agent(C.key + v);
            lkey[i] = kv;
            const uint8_t a0 = kv < C.expanded[v] ? 1 : 0;
            act[0][i] = a0;
            act[1][i] = 0;
            touched[i] = a0;
        }
        if (threadIdx.x == 0) s_changed[0] = s_changed[1] = 0;
        __syncthreads();
        uint32_t a = 0;
        for (uint32_t sweep = 0; sweep <= m; sweep++) {  // Bellman-Ford on m vertices settles within m sweeps
            for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) {
                if (!act[a][i]) continue;
                act[a][i] = 0;
                const uint64_t kv = lkey[i];
                const uint64_t dv = kv >> 32;
                for (uint32_t e = lrp[i]; e < lrp[i + 1]; e++) {
                    const uint2 ed = ladj[e];
                    const uint64_t d = dv + ed.y;
                    if (d >= DIST_INF) continue;
                    const uint64_t cand = (d << 32) | (kv & 0xFFFFFFFFull);
                    if (cand < lkey[ed.x]) {
                        const uint64_t old = atomicMin((unsigned long long *)&lkey[ed.x], (unsigned long long)cand);
                        if (cand < old) {
                            act[a ^ 1u][ed.x] = 1;
                            touched[ed.x] = 1;
                            s_changed[a] = 1;
                        }
                    }
                }
            }
            __syncthreads();
            const int changed = s_changed[a];
            __syncthreads();
            if (threadIdx.x == 0) s_changed[a] = 0;  // reused two sweeps later, after further barriers
            if (!changed) break;
            a ^= 1u;
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) {
            if (!touched[i]) continue;
            const uint32_t v = C.members[b + i];
            const uint64_t kv = lkey[i];
            if (kv < ld_agent(C.key + v)) (void)atomicMin((unsigned long long *)(C.key + v), (unsigned long long)kv);
            const uint64_t dv = kv >> 32;
            const uint32_t p = b + i;
            for (uint32_t e = C.erp[p]; e < C.erp[p + 1]; e++) {
                const uint2 ed = C.ee[e];
                const uint64_t d = dv + ed.y;
                if (d >= DIST_INF) continue;
                const uint64_t cand = (d << 32) | (kv & 0xFFFFFFFFull);
                if (cand < C.key[ed.x]) {
                    const uint64_t old = atomicMin((unsigned long long *)(C.key + ed.x), (unsigned long long)cand);
                    if (cand < old) {
                        const uint32_t cu = C.cl_of[ed.x];
                        if (atomicExch(C.stamp + cu, tag) != tag) {
                            const uint32_t pos = atomicAdd(cnt_next, 1u);
                            if (pos < C.nclusters) C.list[nxt][pos] = cu;
                            else atomicOr(&C.ctl->err, 1u);
                        }
                    }
                }
            }
            C.expanded[v] = kv;
        }
        __syncthreads();  // LDS is reused by the next cluster
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        s_last = atomicAdd(&C.ctl->blocks_done, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!s_last || threadIdx.x != 0) return;
    __threadfence();
    C.ctl->cnt[(r + 2) % 3u] = 0;
    C.ctl->blocks_done = 0;
    if (ld_agent(cnt_next) == 0) C.ctl->done = 1;
    C.ctl->round = r + 1;
    __threadfence();
}

// ------------------------------------------------------------ launchers

static uint32_t fill_grid(uint64_t count) {
    uint64_t g = (count + 255) / 256;
    return (uint32_t)(g < 4096 ? (g ? g : 1) : 4096);
}

hipError_t launch_fill_u64(uint64_t *p, uint64_t count, uint64_t value, hipStream_t s) {
    if (!count) return hipSuccess;
    hipLaunchKernelGGL(k_fill<uint64_t>, dim3(fill_grid(count)), dim3(256), 0, s, p, count, value);
    return hipGetLastError();
}
hipError_t launch_fill_u32(uint32_t *p, uint64_t count, uint32_t value, hipStream_t s) {
    if (!count) return hipSuccess;
    hipLaunchKernelGGL(k_fill<uint32_t>, dim3(fill_grid(count)), dim3(256), 0, s, p, count, value);
    return hipGetLastError();
}
hipError_t launch_fill_u8(uint8_t *p, uint64_t count, uint8_t value, hipStream_t s) {
    if (!count) return hipSuccess;
    hipLaunchKernelGGL(k_fill<uint8_t>, dim3(fill_grid(count)), dim3(256), 0, s, p, count, value);
    return hipGetLastError();
}

hipError_t launch_pass_reset(const VorParams &P, hipStream_t s) {
    hipLaunchKernelGGL(k_pass_reset, dim3((P.nslots + 255) / 256), dim3(256), 0, s, P);
    return hipGetLastError();
}

hipError_t launch_slot_start(const VorParams &P, uint32_t slot, const uint32_t *d_seeds, uint32_t k,
                             uint32_t *heavy_pe_slot, uint32_t nheavy, hipStream_t s) {
    const uint32_t n = P.g.n;
    hipLaunchKernelGGL(k_slot_clear, dim3(fill_grid(n)), dim3(256), 0, s, P.key + (size_t)slot * n,
                       P.aux + (size_t)slot * n, P.dirty + (size_t)slot * n, P.settled + (size_t)slot * n, n,
                       heavy_pe_slot, nheavy);
    if (P.xkey)
        hipLaunchKernelGGL(k_fill<uint64_t>, dim3(fill_grid(P.xchunks)), dim3(256), 0, s,
                           P.xkey + (size_t)slot * P.xchunks, (uint64_t)P.xchunks, KEY_INF);
    hipLaunchKernelGGL(k_slot_seed, dim3(std::max(1u, std::min((k + 255) / 256, 256u))), dim3(256), 0, s, P, slot,
                       d_seeds, k);
    return hipGetLastError();
}

static size_t wave_smem(uint32_t block) { return (size_t)(block / 64) * sizeof(WaveScratch); }

hipError_t launch_round(const VorParams &P, uint32_t grid, uint32_t block, hipStream_t s) {
    // fixed-stride rows, all of them within the local queue's size limit (no chunked rows)
    if (P.g.ell && P.g.max_deg <= min(ELL_W, P.small_max))
        hipLaunchKernelGGL(k_round<true>, dim3(grid), dim3(block), wave_smem(block), s, P);
    else
        hipLaunchKernelGGL(k_round<false>, dim3(grid), dim3(block), wave_smem(block), s, P);
    return hipGetLastError();
}

hipError_t build_round_graph(const VorParams &P, uint32_t grid, uint32_t block, uint32_t rounds, hipGraphExec_t *exec) {
    *exec = nullptr;
    hipGraph_t gr = nullptr;
    hipError_t e = hipGraphCreate(&gr, 0);
    if (e != hipSuccess) return e;
    const bool narrow = P.g.ell && P.g.max_deg <= min(ELL_W, P.small_max);
    VorParams arg = P;
    void *args[] = {(void *)&arg};
    hipKernelNodeParams kp{};
    kp.func = narrow ? (void *)k_round<true> : (void *)k_round<false>;
    kp.gridDim = dim3(grid);
    kp.blockDim = dim3(block);
    kp.sharedMemBytes = (unsigned)wave_smem(block);
    kp.kernelParams = args;
    kp.extra = nullptr;
    hipGraphNode_t prev = nullptr;
    for (uint32_t i = 0; i < rounds && e == hipSuccess; i++) {  // a chain: round i + 1 after round i
        hipGraphNode_t node = nullptr;
        e = hipGraphAddKernelNode(&node, gr, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
        prev = node;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(exec, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (e != hipSuccess) *exec = nullptr;
    return e;
}

hipError_t launch_cluster_start(const ClusterParams &C, const uint32_t *seeds, uint32_t k, hipStream_t s) {
    hipLaunchKernelGGL(k_cluster_start, dim3((k + 255) / 256 + 1), dim3(256), 0, s, C, seeds, k);
    return hipGetLastError();
}

hipError_t launch_cluster_round(const ClusterParams &C, uint32_t grid, hipStream_t s) {
    hipLaunchKernelGGL(k_cluster_round, dim3(grid), dim3(256), 0, s, C);
    return hipGetLastError();
}

int cluster_max_grid() {
    int dev = 0, per_cu = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_cluster_round, 256, 0) != hipSuccess) return 0;
    return per_cu * prop.multiProcessorCount;
}

int round_max_grid(uint32_t block) {
    int dev = 0, per_cu = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_round<false>, (int)block, wave_smem(block)) != hipSuccess)
        return 0;
    return per_cu * prop.multiProcessorCount;
}

int persistent_max_grid(uint32_t block) {
    int dev = 0, per_cu = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persistent<false>, (int)block, wave_smem(block)) !=
        hipSuccess)
        return 0;
    return per_cu * prop.multiProcessorCount;
}

hipError_t launch_persistent(const VorParams &P, uint32_t grid, uint32_t block, uint32_t max_rounds,
                             hipStream_t s) {
    if (P.nslots > PERSIST_SLOTS) return hipErrorInvalidValue;
    VorParams p = P;
    void *args[] = {&p, &max_rounds};
    // fixed-stride rows, all within the local queue's size limit: the same instance choice as launch_round
    const bool narrow = P.g.ell && P.g.max_deg <= min(ELL_W, P.small_max);
    return hipLaunchCooperativeKernel(narrow ? (const void *)k_persistent<true> : (const void *)k_persistent<false>,
                                      dim3(grid), dim3(block), args, wave_smem(block), s);
}

hipError_t launch_scan(const ScanParams &S, uint32_t grid, uint32_t block, hipStream_t s) {
    const bool rev = !S.with_pred && S.g.reverse_scan, cnt = S.ev != nullptr;
    if (rev && cnt) hipLaunchKernelGGL((k_scan<true, true>), dim3(grid), dim3(block), 0, s, S);
    else if (rev) hipLaunchKernelGGL((k_scan<true, false>), dim3(grid), dim3(block), 0, s, S);
    else if (cnt) hipLaunchKernelGGL((k_scan<false, true>), dim3(grid), dim3(block), 0, s, S);
    else hipLaunchKernelGGL((k_scan<false, false>), dim3(grid), dim3(block), 0, s, S);
    if (S.g.nheavy) {
        const uint64_t t = (uint64_t)S.g.nheavy * S.nscan;
        hipLaunchKernelGGL(k_scan_heavy_pred, dim3(fill_grid(t)), dim3(256), 0, s, S);
    }
    return hipGetLastError();
}

hipError_t launch_compact(const CompactParams &C, uint32_t grid, uint32_t block, hipStream_t s) {
    hipLaunchKernelGGL(k_compact, dim3(grid), dim3(block), 0, s, C);
    return hipGetLastError();
}

hipError_t launch_expand(const ExpandParams &E, uint32_t emit_grid, hipStream_t s) {
    if (E.nsel_max && E.pred_ready) {
        const uint64_t threads = 2ull * E.nsel_max;  // one thread per walk
        hipLaunchKernelGGL(k_expand_walk_ready, dim3((uint32_t)((threads + 255) / 256)), dim3(256), 0, s, E);
    } else if (E.nsel_max) {
        const uint64_t waves = 2ull * E.nsel_max;  // one wave per walk, four per workgroup
        hipLaunchKernelGGL(k_expand_walk, dim3((uint32_t)((waves + 3) / 4)), dim3(256), 0, s, E);
    }
    hipLaunchKernelGGL(k_expand_emit, dim3(emit_grid), dim3(256), 0, s, E);
    return hipGetLastError();
}

hipError_t launch_mst(const MstParams &M, const uint32_t *g1_idx, uint32_t m, hipStream_t s) {
    // every round at least halves the number of components that still have an outgoing edge
    uint32_t rounds = 1;
    while ((1ull << rounds) < M.k) rounds++;
    const uint32_t one = M.block ? M.block : 1024;  // workgroup size of the single-workgroup kernels
    if (m <= (1u << 16)) {
        hipLaunchKernelGGL(k_mst_small, dim3(1), dim3(one), 0, s, M, g1_idx, m, rounds);
        return hipGetLastError();
    }
    const uint32_t grid = (uint32_t)std::min<uint64_t>(2048, ((uint64_t)std::max(m, M.k) + 255) / 256);
    hipLaunchKernelGGL(k_mst_init, dim3(grid), dim3(256), 0, s, M, g1_idx, m);
    const uint32_t egrid = (uint32_t)std::min<uint64_t>(2048, ((uint64_t)m + 255) / 256 + 1);
    for (uint32_t r = 0; r <= rounds; r++) {
        hipLaunchKernelGGL(k_mst_edges, dim3(egrid), dim3(256), 0, s, M, r & 1u);
        hipLaunchKernelGGL(k_mst_merge, dim3(1), dim3(one), 0, s, M, r & 1u);
    }
    return hipGetLastError();
}

}  // namespace stn
