// steiner_solve_noalloc: steiner_solve for callers that cannot allocate
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid allocation).  Same kernels, same results; every device buffer of the
// solve is carved from one file-scope device array per GPU, and host staging
// uses static buffers, so the call makes no device or pinned-host allocation
// and creates no stream or event.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <mutex>

#include "engine.h"

using namespace stn;

namespace {

// The device memory of every allocation-free solve on a GPU.  Each GPU that
// runs the library holds its own copy until the process ends.  In host code
// this name is only a stand-in: kernels get the per-device address that
// hipGetSymbolAddress returns (scratch_ptr below), never the name itself.
__device__ __align__(256) uint8_t scratch[STEINER_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
// Seeds a call may pass (duplicates included): the dense pair table of more
// distinct seeds could not fit the scratch anyway (8 bytes per seed pair).
constexpr uint32_t MAX_K = 8192;
constexpr size_t HOST_CTL_BYTES = 64 << 10;

std::mutex g_mu;  // one scratch per GPU and one host staging area: calls run one at a time
void *scratch_ptr[MAX_DEVICES];
alignas(256) uint8_t h_ctl[HOST_CTL_BYTES];  // pass control image and read-backs
uint32_t h_raw[MAX_K];                        // the caller's seeds, sorted and deduplicated in place
uint32_t h_seeds[3 * MAX_K];                  // internal seed ids, table ranks, inverse ranks

// Device address of `scratch` on the current device (the device whose id is
// given), looked up once per device.  Caller holds g_mu.
int scratch_for(int device, void **out) {
    if (device < 0 || device >= MAX_DEVICES) return fail(STEINER_EINVAL, "device %d out of range", device);
    if (!scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(STEINER_EDEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", device,
                        hipGetErrorString(e));
        }
        scratch_ptr[device] = p;
    }
    *out = scratch_ptr[device];
    return STEINER_OK;
}

// Bump carving of the scratch (256-byte aligned pieces).
struct Carve {
    uint8_t *base;
    uint64_t used = 0;
    uint8_t *take(uint64_t bytes) {
        uint8_t *p = base + used;
        used += (bytes + 255) & ~255ull;
        return p;
    }
};

// In-place heapsort of tree edges by (a, b); w rides along.  (A tree has one
// edge per vertex pair, so (a, b) is the whole order (a, b, w).)
void sort_edges(uint32_t *a, uint32_t *b, uint32_t *w, uint64_t m) {
    auto key = [&](uint64_t i) { return ((uint64_t)a[i] << 32) | b[i]; };
    auto swap3 = [&](uint64_t i, uint64_t j) {
        std::swap(a[i], a[j]);
        std::swap(b[i], b[j]);
        std::swap(w[i], w[j]);
    };
    auto sift = [&](uint64_t i, uint64_t len) {
        for (;;) {
            uint64_t c = 2 * i + 1;
            if (c >= len) return;
            if (c + 1 < len && key(c + 1) > key(c)) c++;
            if (key(i) >= key(c)) return;
            swap3(i, c);
            i = c;
        }
    };
    for (uint64_t i = m / 2; i-- > 0;) sift(i, m);
    for (uint64_t end = m; end > 1; end--) {
        swap3(0, end - 1);
        sift(0, end - 1);
    }
}

}  // namespace

// Looks up the allocation-free scratch of `device` (the current device) once;
// called when a graph is created on a device.  A failure is reported again by
// the first steiner_solve_noalloc on that device.
void stn::noalloc_setup(int device) {
    std::lock_guard<std::mutex> lk(g_mu);
    void *p = nullptr;
    if (scratch_for(device, &p)) (void)hipGetLastError();
}

extern "C" int steiner_solve_noalloc(steiner_graph *g, const uint32_t *seeds, uint32_t k, const steiner_options *opt,
                                     uint64_t cap, uint64_t *m_out, uint32_t *a, uint32_t *b, uint32_t *w,
                                     uint64_t *total) {
    const auto t_start = std::chrono::steady_clock::now();
    if (!g || !m_out || !total || (cap && (!a || !b || !w))) return fail(STEINER_EINVAL, "NULL argument");
    if (k == 0) return fail(STEINER_EINVAL, "k must be > 0");
    if (!seeds) return fail(STEINER_EINVAL, "seeds is NULL");
    if (k > MAX_K)
        return fail(STEINER_ENOMEM, "steiner_solve_noalloc takes at most %u seeds (duplicates included), got %u", MAX_K,
                    k);
    std::lock_guard<std::mutex> lk_all(g_mu);
    std::lock_guard<std::mutex> lk(g->mu);
    int rc = hip_check(hipSetDevice(g->device), "hipSetDevice");
    if (rc) return rc;
    void *sp = nullptr;
    if ((rc = scratch_for(g->device, &sp))) return rc;
    const uint32_t n = g->n;
    hipStream_t st = g->stream;

    // Seeds: sorted, deduplicated caller ids (seed index = rank), then internal ids and table ranks.
    for (uint32_t i = 0; i < k; i++) {
        if (seeds[i] >= n) return fail(STEINER_EINVAL, "seed %u >= n", seeds[i]);
        h_raw[i] = seeds[i];
    }
    std::sort(h_raw, h_raw + k);
    const uint32_t kk = (uint32_t)(std::unique(h_raw, h_raw + k) - h_raw);
    if (kk < 2) {  // k == 1: empty tree, D = 0
        *m_out = 0;
        *total = 0;
        return STEINER_OK;
    }
    uint32_t *S = h_seeds, *tr = h_seeds + kk, *ts = h_seeds + 2 * kk;
    const bool ranked = g->reordered;
    for (uint32_t i = 0; i < kk; i++) S[i] = ranked ? g->h_inv[h_raw[i]] : h_raw[i];
    if (ranked) {
        for (uint32_t i = 0; i < kk; i++) ts[i] = i;
        std::sort(ts, ts + kk, [&](uint32_t x, uint32_t y) { return S[x] < S[y]; });
        for (uint32_t r = 0; r < kk; r++) tr[ts[r]] = r;
    }

    Options o = resolve_options(g, opt);
    o.timing = false;  // no events
    // the relaxation is host-stepped (the cluster-local driver builds clusters with allocations)

    // Every device buffer, carved from the scratch.
    const uint64_t P_ = (uint64_t)kk * (kk - 1) / 2, oc = std::min<uint64_t>(P_, g->nnz / 2 + 1);
    const uint64_t chunks = big_row_chunks(g, o.small_max, o.chunk, false);
    const uint64_t cap_s = 2ull * n + 64, cap_b = 2ull * chunks + 64;
    if (cap_s >= (1ull << 32) || cap_b >= (1ull << 32)) return fail(STEINER_ENOMEM, "graph too large");
    const Layout L(1);
    Carve cv{(uint8_t *)sp};
    uint8_t *ctl = cv.take(L.total);
    uint64_t *key = (uint64_t *)cv.take(8ull * n);
    uint32_t *aux = (uint32_t *)cv.take(4ull * n);
    uint8_t *dirty = cv.take(n), *settled = cv.take(n);
    uint64_t *ls[2], *lb[2];
    for (int i = 0; i < 2; i++) ls[i] = (uint64_t *)cv.take(8 * cap_s);
    for (int i = 0; i < 2; i++) lb[i] = (uint64_t *)cv.take(8 * cap_b);
    uint32_t *heavy_pe = (uint32_t *)cv.take(4ull * g->nheavy + 4);
    uint32_t *d_seeds = (uint32_t *)cv.take(12ull * kk);
    uint64_t *pt = (uint64_t *)cv.take(8 * P_);
    uint32_t *cidx = (uint32_t *)cv.take(4 * oc);
    uint8_t *mst = cv.take(mst_scratch_bytes(kk, oc));
    const uint64_t mark_bytes = ((uint64_t)n + 3) / 4 * 4;
    uint32_t *mark = (uint32_t *)cv.take(mark_bytes);
    uint32_t *out = (uint32_t *)cv.take(12ull * n + 16);
    if (cv.used > STEINER_NOALLOC_SCRATCH_BYTES)
        return fail(STEINER_ENOMEM, "this solve needs %llu bytes of device scratch; the allocation-free scratch holds %llu",
                    (unsigned long long)cv.used, (unsigned long long)STEINER_NOALLOC_SCRATCH_BYTES);
    if (L.total + 4096 > HOST_CTL_BYTES) return fail(STEINER_EDEVICE, "control image too large");

    // Pass parameters and the slot's tables (host image, one copy).
    VorParams P{};
    bind_pass(P, g->dg, ctl, L, 1);
    P.key = key;
    P.aux = aux;
    P.dirty = dirty;
    P.settled = settled;
    P.items_s[0] = ls[0];
    P.items_s[1] = ls[1];
    P.items_b[0] = lb[0];
    P.items_b[1] = lb[1];
    bind_state(P, o, cap_s, cap_b);
    memset(h_ctl, 0, L.total);
    *(uint64_t *)(h_ctl + L.pt_ptr) = (uint64_t)(uintptr_t)pt;
    *(uint64_t *)(h_ctl + L.pt_len) = P_;
    *(uint64_t *)(h_ctl + L.oidx_ptr) = (uint64_t)(uintptr_t)cidx;
    *(uint64_t *)(h_ctl + L.oval_ptr) = 0;  // the G'1 values are read from the pair table
    *(uint64_t *)(h_ctl + L.ocap) = oc;
    *(uint64_t *)(h_ctl + L.tr_ptr) = ranked ? (uint64_t)(uintptr_t)(d_seeds + kk) : 0;
    *(uint64_t *)(h_ctl + L.ts_ptr) = ranked ? (uint64_t)(uintptr_t)(d_seeds + 2 * kk) : 0;
    rc = hip_check(hipMemcpyAsync(ctl + L.pt_ptr, h_ctl + L.pt_ptr, L.far_min - L.pt_ptr, hipMemcpyHostToDevice, st),
                   "H2D tables");
    if (!rc)
        rc = hip_check(hipMemcpyAsync(ctl + L.slot_err, h_ctl + L.slot_err, L.total - L.slot_err, hipMemcpyHostToDevice,
                                      st), "H2D tables");
    if (!rc)
        rc = hip_check(hipMemcpyAsync(d_seeds, h_seeds, (ranked ? 12ull : 4ull) * kk, hipMemcpyHostToDevice, st),
                       "H2D seeds");
    if (!rc) rc = hip_check(hipStreamSynchronize(st), "H2D");  // the staging buffers are reused below
    if (rc) return rc;

    // Step 1 set-up: pass control, pair table, the seeds, and the tail's marks (a previous call may have left
    // the scratch in any state)
    rc = hip_check(launch_pass_reset(P, st), "pass reset");
    if (!rc) rc = hip_check(launch_fill_u64(pt, P_, KEY_INF, st), "pair table init");
    if (!rc) rc = hip_check(launch_fill_u32(mark, mark_bytes / 4, 0u, st), "mark clear");
    if (!rc) rc = hip_check(launch_slot_start(P, 0, d_seeds, kk, heavy_pe, g->nheavy, st), "slot start");
    if (rc) return rc;

    // Step 1: host-stepped relaxation rounds until the pass converges
    PassCtl *hpass = (PassCtl *)(h_ctl + L.pass);
    uint32_t chunk_rounds = std::min<uint32_t>(std::max<uint32_t>(g->last_rounds + 2, 4), 256), launched = 0;
    uint32_t next_chunk = 4;
    for (;;) {
        for (uint32_t i = 0; i < chunk_rounds && !rc; i++) rc = hip_check(launch_round(P, o.grid_tuned, o.block, st), "round");
        if (!rc) rc = hip_check(hipMemcpyAsync(hpass, P.pass, sizeof(PassCtl), hipMemcpyDeviceToHost, st), "D2H pass");
        if (!rc) rc = hip_check(hipStreamSynchronize(st), "round sync");
        if (rc) return rc;
        launched += chunk_rounds;
        if (hpass->err & ERR_LIST_OVERFLOW) return fail(STEINER_EDEVICE, "frontier overflow");
        if (hpass->all_done) break;
        const double wall = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
        if (launched >= (1u << 26) || wall > 120.0)
            return fail(STEINER_EDEVICE, "relaxation did not converge (%u rounds)", hpass->round);
        chunk_rounds = next_chunk;
        next_chunk = std::min<uint32_t>(next_chunk * 2, 64);
    }
    g->last_rounds = hpass->round;

    // canonical pred + Step 2 boundary scan, then the G'1 compaction
    ScanParams SP{};
    SP.g = g->dg;
    SP.key = key;
    SP.aux = aux;
    SP.heavy_pe = heavy_pe;
    SP.pt = (uint64_t *const *)(ctl + L.pt_ptr);
    SP.tr = ranked ? (const uint32_t *const *)(ctl + L.tr_ptr) : nullptr;
    SP.slot_ids = (const uint32_t *)(ctl + L.slot_ids);
    SP.nscan = 1;
    SP.slot_err = (uint32_t *)(ctl + L.slot_err);
    SP.with_pred = o.lazy_pred ? 0 : 1;
    CompactParams CP{};
    CP.pt = SP.pt;
    CP.ts = ranked ? (const uint32_t *const *)(ctl + L.ts_ptr) : nullptr;
    CP.pt_len = (const uint64_t *)(ctl + L.pt_len);
    CP.out_idx = (uint32_t *const *)(ctl + L.oidx_ptr);
    CP.out_val = (uint64_t *const *)(ctl + L.oval_ptr);
    CP.out_cap = (const uint64_t *)(ctl + L.ocap);
    CP.out_cnt = (uint32_t *)(ctl + L.out_cnt);
    CP.slot_ids = SP.slot_ids;
    CP.nscan = 1;
    CP.pass = P.pass;
    const uint32_t sgrid = (uint32_t)std::max(1, g->cu_count) * 8;
    rc = hip_check(launch_scan(SP, sgrid, 256, st), "scan");
    if (!rc) rc = hip_check(launch_compact(CP, sgrid, 256, st), "compact");
    uint32_t *h_err = (uint32_t *)(h_ctl + L.slot_err), *h_cnt = (uint32_t *)(h_ctl + L.out_cnt);
    if (!rc) rc = hip_check(hipMemcpyAsync(h_err, SP.slot_err, 4, hipMemcpyDeviceToHost, st), "D2H status");
    if (!rc) rc = hip_check(hipMemcpyAsync(h_cnt, CP.out_cnt, 4, hipMemcpyDeviceToHost, st), "D2H count");
    if (!rc) rc = hip_check(hipMemcpyAsync(hpass, P.pass, sizeof(PassCtl), hipMemcpyDeviceToHost, st), "D2H pass");
    if (!rc) rc = hip_check(hipStreamSynchronize(st), "compact sync");
    if (rc) return rc;
    if (hpass->err & ERR_LIST_OVERFLOW) return fail(STEINER_EDEVICE, "compaction overflow");
    if (*h_err & (ERR_DIST_OVERFLOW | ERR_SUM_OVERFLOW))
        return fail(STEINER_EOVERFLOW, "distance or cross-cell sum does not fit in 32 bits");
    const uint32_t m1 = *h_cnt;
    if (m1 > oc) return fail(STEINER_EDEVICE, "G'1 overflow (%u entries)", m1);

    // Steps 3-6 on the device, then the edges straight into the caller's arrays
    const TreeBufs tb{mst, mark, out};
    rc = launch_tree(g, st, key, aux, kk, pt, ranked ? d_seeds + kk : nullptr, cidx, m1, SP.with_pred != 0, tb, nullptr);
    uint32_t *hdr = (uint32_t *)(h_ctl + L.total);
    if (!rc) rc = hip_check(hipMemcpyAsync(hdr, mst, 16, hipMemcpyDeviceToHost, st), "D2H counts");
    if (!rc) rc = hip_check(hipStreamSynchronize(st), "tail sync");
    if (rc) return rc;
    const uint32_t nsel = hdr[2], mt = hdr[3];
    if (nsel < kk - 1) return fail(STEINER_EDISCONNECTED, "seeds are not connected");
    if (nsel > kk - 1 || mt > n)
        return fail(STEINER_EDEVICE, "tree expansion overflow (%u MST edges, %u tree edges)", nsel, mt);
    if (mt > cap) {
        *m_out = mt;
        return fail(STEINER_ENOMEM, "the tree has %u edges, capacity %llu", mt, (unsigned long long)cap);
    }
    if (mt) {
        rc = hip_check(hipMemcpyAsync(a, out, 4ull * mt, hipMemcpyDeviceToHost, st), "D2H edges");
        if (!rc) rc = hip_check(hipMemcpyAsync(b, out + n, 4ull * mt, hipMemcpyDeviceToHost, st), "D2H edges");
        if (!rc) rc = hip_check(hipMemcpyAsync(w, out + 2 * (size_t)n, 4ull * mt, hipMemcpyDeviceToHost, st), "D2H edges");
        if (!rc) rc = hip_check(hipStreamSynchronize(st), "D2H edges");
        if (rc) return rc;
    }
    // Step 7: canonical order and D
    sort_edges(a, b, w, mt);
    uint64_t D = 0;
    for (uint64_t t = 0; t < mt; t++) D += w[t];
    *m_out = mt;
    *total = D;
    return STEINER_OK;
}
