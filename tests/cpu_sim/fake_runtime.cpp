// Host implementations of the HIP stand-in and of the kernel launchers, with
// simulated pass semantics: every query converges a few rounds after it
// starts, its G'1 is a star around seed 0 and its tree has k-1 edges.  Enough
// to drive the engine's and the server's host logic (admission, slots,
// memory pool, worker threads, error paths) without a GPU.
#include <hip/hip_runtime.h>

#include <cmath>
#include <thread>
#include <unordered_map>
#include <vector>

#include "kernels.h"

thread_local dim3 blockIdx, threadIdx, blockDim, gridDim;
namespace hipsim {
std::mutex launch_mu;
}

static std::atomic<long> g_live_allocs{0};
static std::mutex g_alloc_mu;
static std::unordered_map<void *, size_t> g_dev_sizes;  // live device allocations (not pinned host ones)
static long g_live_dev_bytes = 0;
static std::atomic<bool> g_stall{false};
static std::atomic<bool> g_freeze{false};

hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetDevice(int *d) { *d = 0; return hipSuccess; }
hipError_t hipGetDeviceProperties(hipDeviceProp_t *p, int) { p->multiProcessorCount = 4; return hipSuccess; }
hipError_t hipMalloc(void **p, size_t n) {
    *p = calloc(1, n ? n : 1);
    if (!*p) return hipErrorOutOfMemory;
    g_live_allocs++;
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_dev_sizes[*p] = n;
    g_live_dev_bytes += (long)n;
    return hipSuccess;
}
hipError_t hipFree(void *p) {
    if (p) {
        {
            std::lock_guard<std::mutex> lk(g_alloc_mu);
            auto it = g_dev_sizes.find(p);
            if (it != g_dev_sizes.end()) {
                g_live_dev_bytes -= (long)it->second;
                g_dev_sizes.erase(it);
            }
        }
        free(p);
        g_live_allocs--;
    }
    return hipSuccess;
}
hipError_t hipHostMalloc(void **p, size_t n, unsigned) {
    *p = calloc(1, n ? n : 1);
    if (!*p) return hipErrorOutOfMemory;
    g_live_allocs++;
    return hipSuccess;
}
hipError_t hipHostFree(void *p) {
    if (p) { free(p); g_live_allocs--; }
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind, hipStream_t) {
    std::lock_guard<std::mutex> lk(hipsim::launch_mu);
    memmove(d, s, n);
    return hipSuccess;
}
hipError_t hipMemsetAsync(void *d, int v, size_t n, hipStream_t) {
    std::lock_guard<std::mutex> lk(hipsim::launch_mu);
    memset(d, v, n);
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) { *s = (hipStream_t) new char[1]; return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t s) { delete[] (char *)s; return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t *e) { *e = (hipEvent_t) new char[1]; return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float *m, hipEvent_t, hipEvent_t) { *m = 0.f; return hipSuccess; }
hipError_t hipEventDestroy(hipEvent_t e) { delete[] (char *)e; return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }
hipError_t hipGetSymbolAddress(void **p, const void *sym) {
    *p = const_cast<void *>(sym);
    return hipSuccess;
}
const char *hipGetErrorString(hipError_t) { return "simulated"; }
long hipsim_live_allocs() { return g_live_allocs.load(); }
namespace stn {
struct SimGraph;
hipError_t sim_graph_launch(SimGraph *g, hipStream_t s);
void sim_graph_free(SimGraph *g);
}  // namespace stn
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s) { return stn::sim_graph_launch((stn::SimGraph *)e, s); }
hipError_t hipGraphExecDestroy(hipGraphExec_t e) {
    stn::sim_graph_free((stn::SimGraph *)e);
    return hipSuccess;
}
long hipsim_live_device_bytes() {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    return g_live_dev_bytes;
}
// While set, relaxation rounds advance the round counter but no query converges.
void hipsim_stall(bool on) { g_stall.store(on); }
// While set, relaxation launches change nothing at all, not even the round counter (a broken pass).
void hipsim_freeze(bool on) { g_freeze.store(on); }

namespace stn {

static std::mutex sim_mu;  // the simulated device executes one launcher at a time
static uint32_t g_left[MAX_SLOTS];

hipError_t launch_fill_u64(uint64_t *p, uint64_t c, uint64_t v, hipStream_t) {
    std::lock_guard<std::mutex> lk(sim_mu);
    for (uint64_t i = 0; i < c; i++) p[i] = v;
    return hipSuccess;
}
hipError_t launch_fill_u32(uint32_t *p, uint64_t c, uint32_t v, hipStream_t) {
    std::lock_guard<std::mutex> lk(sim_mu);
    for (uint64_t i = 0; i < c; i++) p[i] = v;
    return hipSuccess;
}
hipError_t launch_fill_u8(uint8_t *p, uint64_t c, uint8_t v, hipStream_t) {
    std::lock_guard<std::mutex> lk(sim_mu);
    memset(p, v, c);
    return hipSuccess;
}

hipError_t launch_pass_reset(const VorParams &P, hipStream_t) {
    std::lock_guard<std::mutex> lk(sim_mu);
    memset(P.pass, 0, sizeof(PassCtl));
    P.pass->all_done = 1;
    memset(P.cnt, 0, sizeof(Counters));
    for (uint32_t q = 0; q < P.nslots; q++) {
        for (int b = 0; b < 3; b++) {
            P.far_min[(size_t)b * P.nslots + q] = DIST_INF;
            P.near_mark[(size_t)b * P.nslots + q] = 0;
        }
        P.slot.active[q] = P.slot.done[q] = P.slot.adv[q] = P.slot.advances[q] = 0;
        P.slot.carry[q] = DIST_INF;
        P.slot.thr[q] = P.slot.thr_prev[q] = 0;
    }
    return hipSuccess;
}

hipError_t launch_slot_start(const VorParams &P, uint32_t slot, const uint32_t *seeds, uint32_t k, uint32_t *hp,
                             uint32_t nheavy, hipStream_t) {
    std::lock_guard<std::mutex> lk(sim_mu);
    if (slot >= P.nslots) return hipErrorInvalidValue;
    const uint32_t n = P.g.n;
    for (uint32_t v = 0; v < n; v++) {
        P.key[(size_t)slot * n + v] = KEY_INF;
        P.aux[(size_t)slot * n + v] = 0;
        P.dirty[(size_t)slot * n + v] = 0;
    }
    for (uint32_t h = 0; h < nheavy; h++) hp[h] = NONE;
    for (uint32_t i = 0; i < k; i++) {
        if (seeds[i] >= n) return hipErrorInvalidValue;
        P.key[(size_t)slot * n + seeds[i]] = i;
    }
    P.slot.active[slot] = 1;
    P.slot.done[slot] = 0;
    P.pass->all_done = 0;
    g_left[slot] = 1 + k % 5;
    return hipSuccess;
}

hipError_t launch_round(const VorParams &P, uint32_t, uint32_t, hipStream_t) {
    std::lock_guard<std::mutex> lk(sim_mu);
    if (P.pass->all_done || g_freeze.load()) return hipSuccess;
    if (g_stall.load()) {
        P.pass->round++;
        return hipSuccess;
    }
    bool any = false;
    for (uint32_t q = 0; q < P.nslots; q++) {
        if (!P.slot.active[q]) continue;
        if (--g_left[q] == 0) {
            P.slot.active[q] = 0;
            P.slot.done[q] = 1;
        } else {
            any = true;
        }
    }
    P.pass->round++;
    if (!any) P.pass->all_done = 1;
    return hipSuccess;
}

struct SimGraph {
    VorParams P;
    uint32_t grid, block, rounds;
};

hipError_t build_round_graph(const VorParams &P, uint32_t grid, uint32_t block, uint32_t rounds, hipGraphExec_t *exec) {
    *exec = (hipGraphExec_t) new SimGraph{P, grid, block, rounds};
    return hipSuccess;
}

hipError_t sim_graph_launch(SimGraph *g, hipStream_t s) {
    for (uint32_t i = 0; i < g->rounds; i++) {
        const hipError_t e = launch_round(g->P, g->grid, g->block, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
void sim_graph_free(SimGraph *g) { delete g; }

int persistent_max_grid(uint32_t) { return 0; }
int round_max_grid(uint32_t) { return 0; }
int cluster_max_grid() { return 0; }
hipError_t launch_cluster_start(const ClusterParams &, const uint32_t *, uint32_t, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_cluster_round(const ClusterParams &, uint32_t, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_persistent(const VorParams &, uint32_t, uint32_t, uint32_t, hipStream_t) { return hipErrorInvalidValue; }

hipError_t launch_scan(const ScanParams &S, uint32_t, uint32_t, hipStream_t) {
    std::lock_guard<std::mutex> lk(sim_mu);
    for (uint32_t i = 0; i < S.nscan; i++) {
        const uint32_t slot = S.slot_ids[i];
        for (uint32_t v = 0; v < S.g.n; v++) S.aux[(size_t)slot * S.g.n + v] = v;
    }
    return hipSuccess;
}

hipError_t launch_compact(const CompactParams &C, uint32_t, uint32_t, hipStream_t) {
    std::lock_guard<std::mutex> lk(sim_mu);
    for (uint32_t i = 0; i < C.nscan; i++) {
        const uint32_t slot = C.slot_ids[i];
        const uint64_t len = C.pt_len[slot];
        const uint32_t k = (uint32_t)((1.0 + std::sqrt(1.0 + 8.0 * (double)len)) / 2.0 + 0.5);
        uint32_t m = 0;
        for (uint32_t j = 1; j < k && m < C.out_cap[slot]; j++, m++) {
            C.out_idx[slot][m] = (uint32_t)((uint64_t)j * (j - 1) / 2);  // pair (0, j)
            if (C.out_val[slot]) C.out_val[slot][m] = ((uint64_t)j << 32) | 0u;
        }
        C.out_cnt[slot] = m;
    }
    return hipSuccess;
}

hipError_t launch_mst(const MstParams &M, const uint32_t *g1_idx, uint32_t m, hipStream_t) {
    std::lock_guard<std::mutex> lk(sim_mu);
    // union-find over the listed pairs in list order (the simulated G'1 is a star)
    std::vector<uint32_t> root(M.k);
    for (uint32_t c = 0; c < M.k; c++) root[c] = c;
    auto find = [&](uint32_t x) {
        while (root[x] != x) x = root[x] = root[root[x]];
        return x;
    };
    uint32_t nsel = 0;
    for (uint32_t t = 0; t < m; t++) {
        const uint32_t p = g1_idx[t];
        const uint32_t j = (uint32_t)((1.0 + std::sqrt(1.0 + 8.0 * (double)p)) / 2.0);
        const uint32_t i = p - j * (j - 1) / 2;
        if (i >= j || j >= M.k) return hipErrorInvalidValue;
        const uint32_t a = find(i), b = find(j);
        if (a == b) continue;
        root[a] = b;
        M.sel[nsel++] = (uint32_t)M.pt[p];
    }
    M.hdr[0] = M.hdr[1] = 0;
    M.hdr[2] = nsel;
    M.hdr[3] = 0;
    return hipSuccess;
}

hipError_t launch_expand(const ExpandParams &E, uint32_t, hipStream_t) {
    std::lock_guard<std::mutex> lk(sim_mu);
    const uint32_t nsel = *E.nsel;
    if (nsel > E.nsel_max) return hipErrorInvalidValue;
    for (uint32_t t = 0; t < nsel && t + 1 < E.g.n; t++) {
        E.oa[t] = t;
        E.ob[t] = t + 1;
        E.ow[t] = 1;
    }
    for (uint32_t x = 0; x < (E.g.n + 3) / 4; x++)
        if (E.mark[x]) return hipErrorInvalidValue;  // marks are zero between calls
    *E.ocnt = nsel;
    return hipSuccess;
}

}  // namespace stn
