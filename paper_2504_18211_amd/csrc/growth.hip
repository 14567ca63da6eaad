/*
 * growth.hip -- the growth line (C ABI in include/hbheap_growth.h).
 *
 * Many agents grow int32 lists by doubling reallocation inside persistent
 * kernels: allocation and free from running kernels is the paper's use case
 * (Introduction; Methods: many threads allocate at once).  Every step is one
 * grid-stride launch over all agents; the steps of one run are chained as
 * kernel nodes of one HIP graph and replayed with a single launch.  An
 * autotuner times the graph for each (chunk size, queue variant,
 * aggregation width) candidate.
 *
 * Per agent and step s >= 1 (agent active when doublings[a] >= s):
 *   q = allocate 2 * bytes; copy the old list; append the new words; free
 *   the old block once the wave's reads of it have returned (no cache
 *   write-back is needed for a block only read); the table then points at
 *   q.
 * Copies of lists of 512 B and more are done by all active lanes of the
 * wave, one list at a time, 16 B per lane per instruction (coalesced);
 * smaller ones per lane.
 */
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "hbheap_device.h"
#include "hbheap_growth.h"
#include "pattern.h"

using namespace hbheap::detail;

struct hbheap_growth {
    heap_t heap = nullptr;
    hbheap_dev_t dev;
    uint32_t agents = 0, steps = 0, seed = 0, blocks = 0;
    void* mem = nullptr;          /* one allocation for every table below */
    uint64_t* lists = nullptr;    /* agents: list address or 0            */
    uint32_t* elems = nullptr;    /* agents: elements in the list         */
    int32_t* doublings = nullptr; /* agents: clamped to [0, steps - 1]    */
    unsigned long long* fails = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

constexpr uint32_t kGrowBlock = 256;
constexpr uint64_t kCoopList = 512;

struct GrowArgs {
    uint64_t* lists;
    uint32_t* elems;
    const int32_t* doublings;
    unsigned long long* fails;
    uint32_t agents;
    uint32_t seed;
};

/* 16-byte units [u0, u1) of agent pattern `sr` into dst (per lane). */
__device__ __forceinline__ void put_words(uint4* dst, uint32_t sr, uint32_t u0, uint32_t u1, uint32_t first,
                                          uint32_t stride)
{
    for (uint32_t u = u0 + first; u < u1; u += stride) {
        const uint32_t j = u * 4;
        dst[u] = make_uint4(pat_word(sr, j), pat_word(sr, j + 1), pat_word(sr, j + 2), pat_word(sr, j + 3));
    }
}

__global__ void __launch_bounds__(kGrowBlock) k_growth_step(hbheap_dev_t h, GrowArgs g, uint32_t step)
{
    const uint64_t stride = (uint64_t)gridDim.x * kGrowBlock;
    for (uint64_t a = (uint64_t)blockIdx.x * kGrowBlock + threadIdx.x; a < g.agents; a += stride) {
        const uint32_t sr = g.seed ^ fmix32((uint32_t)a);
        /* home shard: the agent's linear wave index */
        const uint32_t home = (uint32_t)((a >> 6) % h.n_shards);
        const bool dry = home_pool_dry(h, home);
        if (step == 0) {
            void* p = malloc_wave(h, 16, home, dry);
            if (p) *(uint4*)p = make_uint4(pat_word(sr, 0), pat_word(sr, 1), pat_word(sr, 2), pat_word(sr, 3));
            else atomicAdd(g.fails, 1ull);
            g.lists[a] = (uint64_t)p;
            g.elems[a] = p ? 4u : 0u;
            continue;
        }
        const uint64_t old = g.lists[a];
        const uint32_t e = g.elems[a];
        const bool active = old != 0 && g.doublings[a] >= (int32_t)step;
        void* q = nullptr;
        if (active) q = malloc_wave(h, (size_t)e * 8u, home, dry);
        const bool ok = active && q != nullptr;
        if (active && !ok) atomicAdd(g.fails, 1ull);
        const uint32_t nu = e / 4u; /* 16-byte units of the old list */
        if (ok && (uint64_t)e * 4u < kCoopList) {
            const uint4* src = (const uint4*)old;
            uint4* dst = (uint4*)q;
            for (uint32_t u = 0; u < nu; ++u) dst[u] = src[u];
            put_words(dst, sr, nu, 2u * nu, 0, 1);
        }
        uint64_t big = __ballot(ok && (uint64_t)e * 4u >= kCoopList);
        /* the lanes of this iteration share the units (the last wave of the
         * grid may be partial) */
        const uint64_t act = exec_mask();
        const uint32_t nact = (uint32_t)__popcll(act), r = rank_in(act);
        while (big) {
            const uint32_t l = ctz64(big);
            big &= big - 1ull;
            const uint4* src = (const uint4*)bcast64(old, l);
            uint4* dst = (uint4*)bcast64((uint64_t)q, l);
            const uint32_t n = bcast(nu, l);
            const uint32_t bsr = bcast(sr, l);
            for (uint32_t u = r; u < n; u += nact) dst[u] = src[u];
            put_words(dst, bsr, n, 2u * n, r, nact);
        }
        /* the wave only read the old block: once those reads have returned
         * it can be handed out again (the new block's writes are ordered for
         * the next step by the kernel boundary) */
        wait_own_accesses();
        if (ok) {
            (void)free_wave(h, (void*)old, 0, false);
            g.lists[a] = (uint64_t)q;
            g.elems[a] = 2u * e;
        }
    }
}

__global__ void __launch_bounds__(kGrowBlock) k_growth_release(hbheap_dev_t h, GrowArgs g)
{
    const uint64_t stride = (uint64_t)gridDim.x * kGrowBlock;
    for (uint64_t a = (uint64_t)blockIdx.x * kGrowBlock + threadIdx.x; a < g.agents; a += stride) {
        const uint64_t p = g.lists[a];
        if (p) (void)free_wave(h, (void*)p, 0, false);
        g.lists[a] = 0;
        g.elems[a] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *g.fails = 0;
}

__global__ void __launch_bounds__(kGrowBlock) k_growth_export(GrowArgs g, uint64_t* ptrs, uint64_t* bytes,
                                                              uint64_t* failures)
{
    const uint64_t stride = (uint64_t)gridDim.x * kGrowBlock;
    for (uint64_t a = (uint64_t)blockIdx.x * kGrowBlock + threadIdx.x; a < g.agents; a += stride) {
        if (ptrs) ptrs[a] = g.lists[a];
        if (bytes) bytes[a] = (uint64_t)g.elems[a] * 4u;
    }
    if (failures && blockIdx.x == 0 && threadIdx.x == 0) *failures = *g.fails;
}

__global__ void k_growth_init(GrowArgs g, const int32_t* src, int32_t* dst, uint32_t max_d)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < g.agents) {
        const int32_t d = src[i];
        dst[i] = d < 0 ? 0 : (d > (int32_t)max_d ? (int32_t)max_d : d);
        g.lists[i] = 0;
        g.elems[i] = 0;
    }
    if (i == 0) *g.fails = 0;
}

GrowArgs args_of(const hbheap_growth* g)
{
    return GrowArgs{g->lists, g->elems, g->doublings, g->fails, g->agents, g->seed};
}

uint64_t al256(uint64_t x) { return (x + 255) & ~255ull; }

}  // namespace

extern "C" {

int growth_create(heap_t h, uint32_t agents, const int32_t* doublings, uint32_t steps, uint32_t seed, growth_t* out)
{
    if (!h || !out || !doublings || agents == 0 || agents > (1u << 24) || steps == 0 || steps > 16)
        return HBHEAP_E_INVAL;
    heap_info_t info;
    if (heap_info(h, &info) != HBHEAP_OK) return HBHEAP_E_INVAL;
    if ((16ull << (steps - 1)) > info.chunk_bytes) return HBHEAP_E_INVAL;
    hbheap_growth* g = new (std::nothrow) hbheap_growth();
    if (!g) return HBHEAP_E_NOMEM;
    g->heap = h;
    if (heap_device_handle(h, &g->dev) != HBHEAP_OK) { delete g; return HBHEAP_E_INVAL; }
    g->agents = agents;
    g->steps = steps;
    g->seed = seed;
    const uint64_t o_el = al256(8ull * agents), o_d = o_el + al256(4ull * agents), o_f = o_d + al256(4ull * agents);
    if (hipMalloc(&g->mem, o_f + 256) != hipSuccess) { delete g; return HBHEAP_E_NOMEM; }
    uint8_t* m = (uint8_t*)g->mem;
    g->lists = (uint64_t*)m;
    g->elems = (uint32_t*)(m + o_el);
    g->doublings = (int32_t*)(m + o_d);
    g->fails = (unsigned long long*)(m + o_f);
    /* persistent grid: what the device keeps resident, capped by the work */
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_growth_step, kGrowBlock, 0) !=
            hipSuccess) {
        (void)hipFree(g->mem);
        delete g;
        return HBHEAP_E_HIP;
    }
    const uint64_t need = (agents + kGrowBlock - 1) / kGrowBlock;
    g->blocks = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(need, (uint64_t)std::max(1, cus * per_cu)));
    const GrowArgs ga = args_of(g);
    hipLaunchKernelGGL(k_growth_init, dim3((agents + 255) / 256), dim3(256), 0, 0, ga, doublings, g->doublings,
                       steps - 1);
    if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        (void)hipFree(g->mem);
        delete g;
        return HBHEAP_E_HIP;
    }
    *out = g;
    return HBHEAP_OK;
}

int growth_destroy(growth_t g)
{
    if (!g) return HBHEAP_OK;
    int rc = HBHEAP_OK;
    if (g->exec && hipGraphExecDestroy(g->exec) != hipSuccess) rc = HBHEAP_E_HIP;
    if (g->graph && hipGraphDestroy(g->graph) != hipSuccess) rc = HBHEAP_E_HIP;
    if (g->mem && hipFree(g->mem) != hipSuccess) rc = HBHEAP_E_HIP;
    delete g;
    return rc;
}

int growth_step(growth_t g, uint32_t step, hipStream_t stream)
{
    if (!g || step >= g->steps) return HBHEAP_E_INVAL;
    hipLaunchKernelGGL(k_growth_step, dim3(g->blocks), dim3(kGrowBlock), 0, stream, g->dev, args_of(g), step);
    return hipGetLastError() == hipSuccess ? HBHEAP_OK : HBHEAP_E_HIP;
}

int growth_graph_launch(growth_t g, hipStream_t stream)
{
    if (!g) return HBHEAP_E_INVAL;
    if (!g->exec) {
        hipGraph_t graph = nullptr;
        if (hipGraphCreate(&graph, 0) != hipSuccess) return HBHEAP_E_HIP;
        hipGraphNode_t prev = nullptr;
        GrowArgs ga = args_of(g);
        hbheap_dev_t dv = g->dev;
        for (uint32_t s = 0; s < g->steps; ++s) {
            uint32_t step = s;
            void* kargs[] = {&dv, &ga, &step};
            hipKernelNodeParams p;
            memset(&p, 0, sizeof(p));
            p.func = (void*)k_growth_step;
            p.gridDim = dim3(g->blocks);
            p.blockDim = dim3(kGrowBlock);
            p.sharedMemBytes = 0;
            p.kernelParams = kargs;
            p.extra = nullptr;
            hipGraphNode_t node = nullptr;
            if (hipGraphAddKernelNode(&node, graph, prev ? &prev : nullptr, prev ? 1 : 0, &p) != hipSuccess) {
                (void)hipGraphDestroy(graph);
                return HBHEAP_E_HIP;
            }
            prev = node;
        }
        hipGraphExec_t exec = nullptr;
        if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return HBHEAP_E_HIP;
        }
        g->graph = graph;
        g->exec = exec;
    }
    return hipGraphLaunch(g->exec, stream) == hipSuccess ? HBHEAP_OK : HBHEAP_E_HIP;
}

int growth_release(growth_t g, hipStream_t stream)
{
    if (!g) return HBHEAP_E_INVAL;
    hipLaunchKernelGGL(k_growth_release, dim3(g->blocks), dim3(kGrowBlock), 0, stream, g->dev, args_of(g));
    return hipGetLastError() == hipSuccess ? HBHEAP_OK : HBHEAP_E_HIP;
}

int growth_export(growth_t g, uint64_t* ptrs, uint64_t* bytes, uint64_t* failures, hipStream_t stream)
{
    if (!g) return HBHEAP_E_INVAL;
    if (!ptrs && !bytes && !failures) return HBHEAP_OK;
    hipLaunchKernelGGL(k_growth_export, dim3(g->blocks), dim3(kGrowBlock), 0, stream, args_of(g), ptrs, bytes,
                       failures);
    return hipGetLastError() == hipSuccess ? HBHEAP_OK : HBHEAP_E_HIP;
}

int growth_launch_shape(growth_t g, uint32_t* blocks, uint32_t* threads)
{
    if (!g) return HBHEAP_E_INVAL;
    if (blocks) *blocks = g->blocks;
    if (threads) *threads = kGrowBlock;
    return HBHEAP_OK;
}

int growth_autotune(size_t heap_bytes, uint32_t agents, const int32_t* doublings, uint32_t steps, uint32_t seed,
                    const growth_candidate_t* cand, uint32_t n_cand, uint32_t reps, float* ms, int32_t* best)
{
    if (!doublings || !cand || !n_cand || !ms || !best || !reps || reps > 1000) return HBHEAP_E_INVAL;
    *best = -1;
    hipStream_t st = nullptr;
    if (hipStreamCreate(&st) != hipSuccess) return HBHEAP_E_HIP;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    unsigned long long* dfail = nullptr;
    int rc = HBHEAP_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess ||
        hipMalloc(&dfail, sizeof(unsigned long long)) != hipSuccess) {
        rc = HBHEAP_E_HIP;
    }
    float best_ms = 0.f;
    for (uint32_t i = 0; i < n_cand && rc == HBHEAP_OK; ++i) {
        ms[i] = -1.f;
        heap_config_t cfg;
        memset(&cfg, 0, sizeof(cfg));
        cfg.variant = cand[i].variant;
        cfg.width = cand[i].width;
        cfg.flags = cand[i].flags & HBHEAP_FLAG_EAGER;
        heap_t h = nullptr;
        if (heap_create_ex(heap_bytes, cand[i].chunk_bytes, &cfg, &h) != HBHEAP_OK) continue;
        growth_t g = nullptr;
        if (growth_create(h, agents, doublings, steps, seed, &g) != HBHEAP_OK) {
            (void)heap_destroy(h);
            continue;
        }
        std::vector<float> t;
        unsigned long long fails = 0;
        bool good = growth_graph_launch(g, st) == HBHEAP_OK && growth_release(g, st) == HBHEAP_OK;
        for (uint32_t r = 0; r < reps && good; ++r) {
            good = hipEventRecord(e0, st) == hipSuccess && growth_graph_launch(g, st) == HBHEAP_OK &&
                   hipEventRecord(e1, st) == hipSuccess &&
                   growth_export(g, nullptr, nullptr, (uint64_t*)dfail, st) == HBHEAP_OK &&
                   growth_release(g, st) == HBHEAP_OK && hipStreamSynchronize(st) == hipSuccess;
            float x = 0.f;
            if (good) good = hipEventElapsedTime(&x, e0, e1) == hipSuccess;
            unsigned long long f = 0;
            if (good) good = hipMemcpy(&f, dfail, sizeof(f), hipMemcpyDeviceToHost) == hipSuccess;
            fails += f;
            t.push_back(x);
        }
        uint32_t err = 0;
        if (good && heap_get_error(h, &err) == HBHEAP_OK && err == 0 && fails == 0) {
            std::sort(t.begin(), t.end());
            ms[i] = t[t.size() / 2];
            if (*best < 0 || ms[i] < best_ms) {
                *best = (int32_t)i;
                best_ms = ms[i];
            }
        }
        if (hipStreamSynchronize(st) != hipSuccess) rc = HBHEAP_E_HIP;
        (void)growth_destroy(g);
        (void)heap_destroy(h);
    }
    if (dfail) (void)hipFree(dfail);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(st);
    return rc;
}

}  // extern "C"
