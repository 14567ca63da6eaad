/*
 * serve.hip -- the serving line (C ABI in include/hbheap_serve.h).
 *
 * A host loop over arriving batches of allocation and free requests, K
 * batches in flight on their own streams, admission against the chunks in
 * use, and one kernel per batch in which every lane serves one request with
 * dev_malloc / dev_free on the resident heap (Introduction: allocation from
 * running kernels on a heap the host preallocated).
 *
 * Host side, per batch: stage the requests in the slot's pinned buffers,
 * copy them in, launch, copy the packed results out, record an event; the
 * loop polls the events, so several batches overlap on the device while
 * the host admits the next ones.
 */
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "hbheap_device.h"
#include "hbheap_serve.h"
#include "pattern.h"

using namespace hbheap::detail;

namespace {

constexpr uint32_t kServeBlock = 256;
constexpr uint64_t kServeCoop = 1024;
constexpr uint32_t kMaxSlots = 16;
constexpr uint32_t kMaxBatch = 65536;
constexpr uint32_t kMaxClasses = 16;
/* chunk-usage words (usage_read): chunks in use, then one per class */
constexpr uint64_t kUsageWords = 1 + kMaxClasses;
constexpr uint64_t kUsageBytes = 8 * kUsageWords;

struct Slot {
    hipStream_t st = nullptr;
    hipEvent_t done = nullptr;
    int64_t* ops_d = nullptr;
    uint64_t* aux_d = nullptr;
    uint64_t* res_d = nullptr;  /* results, then the chunk-usage words */
    uint32_t* done_d = nullptr; /* workgroups of the running batch finished */
    int64_t* ops_h = nullptr;   /* pinned */
    uint64_t* aux_h = nullptr;  /* pinned */
    uint64_t* res_h = nullptr;  /* pinned */
    int64_t batch = -1;
};

}  // namespace

struct hbheap_server {
    heap_t heap = nullptr;
    hbheap_dev_t dev;
    heap_info_t info;
    serve_config_t cfg;
    uint64_t* handles = nullptr; /* device, max_requests */
    std::vector<Slot> slots;
    hipStream_t mon = nullptr;
    hipEvent_t mon_done = nullptr;
    uint64_t* usage_d = nullptr;  /* 1 + kMaxClasses u64 */
    uint64_t* usage_h = nullptr;  /* pinned, same size */
    std::vector<uint64_t> class_cap; /* page variant: chunks class k may own */
};

namespace {

/* ---------------- device ---------------- */

/* One wave: out[0] = chunks taken from the pools (per shard, its chunks
 * minus the pool's remaining ones: size - min(bump, size), or with eager
 * retirement the chunks its pool ring holds); out[1 + k], page variant:
 * chunks owned by class k over all shards (0 otherwise).  Agent-scope loads
 * of counters that only grow until a trim (with eager retirement, the pool
 * rings also shrink the count as chunks retire). */
__device__ __forceinline__ void usage_read(const hbheap_dev_t& h, uint64_t* out)
{
    const uint32_t j = lane();
    uint64_t used = 0;
    for (uint32_t s = j; s < h.n_shards; s += 64) {
        const uint64_t* pb = h.pool + 16ull * s;
        const uint64_t bump = __hip_atomic_load(pb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t size = ((const uint32_t*)pb)[2];
        const uint64_t lo = (uint64_t)s << h.log2_span;
        const uint64_t hi = std::min<uint64_t>((uint64_t)h.n_chunks, ((uint64_t)s + 1) << h.log2_span);
        /* eager retirement: the pool ring's published chunks */
        const uint64_t left = eager(h) ? (uint64_t)std::max<int32_t>(state_count(bump), 0)
                                       : size - std::min<uint64_t>(bump, size);
        used += (hi - lo) - left;
    }
    for (uint32_t o = 32; o; o >>= 1) used += __shfl_xor(used, o);
    if (j == 0) out[0] = used;
    for (uint32_t k = j; k < h.n_classes; k += 64) {
        uint64_t own = 0;
        if (h.variant == HBHEAP_VARIANT_PAGE)
            for (uint32_t s = 0; s < h.n_shards; ++s) own += a_load64(owned_of(h, s, k));
        out[1 + k] = own;
    }
}

__global__ void k_usage(hbheap_dev_t h, uint64_t* out) { usage_read(h, out); }

/* 32-bit sum of the words of [0, size) read back, per lane (units u of 16 B
 * with u = first, first + step, ...), tail bytes by the lane with first 0.
 * Eight units per lane are loaded before any is added, so a lane waits once
 * per eight loads rather than once per load.  The tail (size not a multiple
 * of 16) is read as its whole 16-byte unit, which lies inside the block's
 * page (a multiple of 16 bytes), and each word is masked to the bytes below
 * size: the same sum as adding the bytes one by one, each at its place in
 * its word. */
__device__ __forceinline__ uint32_t sum_range(const uint8_t* p, uint64_t size, uint64_t first, uint64_t step)
{
    const uint64_t nq = size >> 4;
    const uint4* q = (const uint4*)p;
    uint32_t s = 0;
    for (uint64_t u = first; u < nq; u += 8u * step) {
        uint4 v[8];
#pragma unroll
        for (uint32_t b = 0; b < 8u; ++b) {
            const uint64_t x = u + b * step;
            v[b] = x < nq ? q[x] : make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (uint32_t b = 0; b < 8u; ++b) s += v[b].x + v[b].y + v[b].z + v[b].w;
    }
    const uint32_t nb = (uint32_t)(size & 15u);
    if (first == 0 && nb) {
        const uint4 v = q[nq];
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (uint32_t k = 0; k < 4u; ++k) {
            const uint32_t m = nb >= 4u * k + 4u ? ~0u : nb <= 4u * k ? 0u : (1u << (8u * (nb - 4u * k))) - 1u;
            s += w[k] & m;
        }
    }
    return s;
}

/* One lane per request.  ops[i] >= 0: allocate, write the words, read them
 * back; ops[i] < 0: read the target block back, then free it.  Blocks of
 * kServeCoop bytes and more are written and read by all active lanes of the
 * wave, each lane on the same 16-byte units in both passes (so every lane
 * reads back what it wrote itself). */
__device__ __forceinline__ void serve_one(const hbheap_dev_t& h, const int64_t* ops, const uint64_t* aux, uint64_t i,
                                          uint64_t first_req, uint64_t* handles, uint64_t* res, uint32_t seed)
{
    const uint32_t me = lane();
    /* home shard: the wave's index in the launch, offset per batch (the
     * value must be the same on every lane of the wave); its pool hint is
     * loaded together with the request */
    const uint32_t home = (uint32_t)(((first_req >> 6) + (i >> 6)) % h.n_shards);
    const bool dry = home_pool_dry(h, home);
    __asm__ volatile("" ::: "memory");
    const int64_t op = ops[i];
    const uint64_t req = first_req + i;
    const bool is_alloc = op >= 0;
    uint8_t* p = nullptr;
    uint64_t size = 0;
    uint32_t sr = 0;
    if (is_alloc) {
        size = (uint64_t)op;
        sr = seed ^ fmix32((uint32_t)req);
        p = (uint8_t*)malloc_wave(h, size, home, dry);
        handles[req] = (uint64_t)p;
        if (!p) size = 0;
    } else {
        const uint64_t t = (uint64_t)(-(op + 1));
        p = (uint8_t*)handles[t];
        size = p ? aux[i] : 0;
        sr = seed ^ fmix32((uint32_t)t);
    }
    int32_t cls = -1;
    if (p) cls = h.chunk_class[(uint64_t)(p - h.data) >> h.log2_chunk];
    const bool coop = size >= kServeCoop;
    const uint64_t act = exec_mask();
    const uint32_t nact = (uint32_t)__popcll(act), r = rank_in(act);
    /* write (allocations) */
    if (is_alloc && size && !coop) pat_write_range(p, size, sr, 0, 1);
    uint64_t big = __ballot(is_alloc && coop);
    while (big) {
        const uint32_t l = ctz64(big);
        big &= big - 1ull;
        pat_write_range((uint8_t*)bcast64((uint64_t)p, l), bcast64(size, l), bcast(sr, l), r, nact);
    }
    /* read back (both kinds) */
    uint32_t sum = 0;
    if (size && !coop) sum = sum_range(p, size, 0, 1);
    big = __ballot(coop);
    if (big) {
        /* each lane adds its part of every large block to the block owner's
         * LDS word; one wait for all of them at the end */
        uint32_t* acc = (uint32_t*)stage_for_wave();
        acc[me] = 0;
        wave_sync_lds();
        while (big) {
            const uint32_t l = ctz64(big);
            big &= big - 1ull;
            const uint32_t part = sum_range((const uint8_t*)bcast64((uint64_t)p, l), bcast64(size, l), r, nact);
            __hip_atomic_fetch_add(acc + l, part, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        wave_sync_lds();
        if (coop) sum = acc[me];
        wave_sync_lds();
    }
    uint32_t status = is_alloc ? (p ? SERVE_OK : SERVE_ALLOC_NULL) : SERVE_FREE_NULL;
    if (!is_alloc) {
        /* the reads above complete before the block can be handed out again
         * (its writes were ordered by the end of the allocating kernel) */
        wait_own_accesses();
        const uint32_t st = free_wave(h, p, 0, false);
        status = st == kFreeOk ? SERVE_OK : st == kFreeDouble ? SERVE_FREE_DOUBLE
                                          : st == kFreeInvalid ? SERVE_FREE_INVAL : SERVE_FREE_NULL;
    }
    res[i] = (uint64_t)sum | ((uint64_t)status << 32) | ((uint64_t)(uint8_t)(int8_t)cls << 40);
}

/* One batch: lane i serves request i (serve_one).  The batch's last
 * workgroup to finish then reads the chunk usage into res[n ..): every
 * workgroup waits for its own memory operations (the pool and owned
 * counters its refills moved included) before it counts itself done, so the
 * words are exact for this batch and hold whatever other batches in flight
 * had done by then.  The usage travels back with the results, in the same
 * copy; done is left at zero for the slot's next batch. */
__global__ void __launch_bounds__(kServeBlock) k_serve_batch(hbheap_dev_t h, const int64_t* ops, const uint64_t* aux,
                                                             uint32_t n, uint64_t first_req, uint64_t* handles,
                                                             uint64_t* res, uint32_t seed, uint32_t* done)
{
    __shared__ uint32_t last;
    const uint64_t i = (uint64_t)blockIdx.x * kServeBlock + threadIdx.x;
    if (i < n) serve_one(h, ops, aux, i, first_req, handles, res, seed);
    wait_own_accesses();
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t before = __hip_atomic_fetch_add(done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        last = before + 1u == gridDim.x;
    }
    __syncthreads();
    if (last && threadIdx.x < 64) {
        usage_read(h, res + n);
        if (threadIdx.x == 0) __hip_atomic_store(done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ void k_serve_export(const uint64_t* handles, uint64_t first, uint64_t n, uint64_t* dst)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = handles[first + i];
}

/* ---------------- host ---------------- */

using Clock = std::chrono::steady_clock;

uint64_t ns_since(Clock::time_point t0)
{
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now() - t0).count();
}

int host_class(uint64_t n, uint64_t chunk)
{
    if (n == 0 || n > chunk) return -1;
    if (n <= 16) return 0;
    uint32_t r = 0;
    while ((1ull << r) < n) ++r;
    return (int)r - 4;
}

void free_slot(Slot& s)
{
    if (s.done) (void)hipEventDestroy(s.done);
    if (s.st) (void)hipStreamDestroy(s.st);
    if (s.ops_d) (void)hipFree(s.ops_d);
    if (s.aux_d) (void)hipFree(s.aux_d);
    if (s.res_d) (void)hipFree(s.res_d);
    if (s.done_d) (void)hipFree(s.done_d);
    if (s.ops_h) (void)hipHostFree(s.ops_h);
    if (s.aux_h) (void)hipHostFree(s.aux_h);
    if (s.res_h) (void)hipHostFree(s.res_h);
    s = Slot();
}

void release(hbheap_server* s)
{
    for (Slot& sl : s->slots) free_slot(sl);
    if (s->mon_done) (void)hipEventDestroy(s->mon_done);
    if (s->mon) (void)hipStreamDestroy(s->mon);
    if (s->usage_d) (void)hipFree(s->usage_d);
    if (s->usage_h) (void)hipHostFree(s->usage_h);
    if (s->handles) (void)hipFree(s->handles);
    delete s;
}

int usage_issue(hbheap_server* s)
{
    hipLaunchKernelGGL(k_usage, dim3(1), dim3(64), 0, s->mon, s->dev, s->usage_d);
    if (hipGetLastError() != hipSuccess) return HBHEAP_E_HIP;
    return hipMemcpyAsync(s->usage_h, s->usage_d, kUsageBytes, hipMemcpyDeviceToHost, s->mon) == hipSuccess
               ? HBHEAP_OK : HBHEAP_E_HIP;
}

int usage_sync(hbheap_server* s)
{
    if (usage_issue(s) != HBHEAP_OK) return HBHEAP_E_HIP;
    return hipStreamSynchronize(s->mon) == hipSuccess ? HBHEAP_OK : HBHEAP_E_HIP;
}

}  // namespace

/* ---------------- chunks in use without allocating ----------------
 *
 * Staging of heap_chunks_in_use_noalloc: what k_usage writes -- the chunks
 * in use, then the chunks each class owns -- in a fixed array instead of
 * memory allocated per call.  Each GPU the library runs on holds its own
 * copy until the process ends; every call on a GPU uses that GPU's copy, so
 * calls that overlap on one GPU race on it.  Host code never passes the
 * array's name to a kernel (in host code it is not a device address): it
 * uses the address hipGetSymbolAddress gave for the current device. */
constexpr uint32_t kNoAllocWords = kUsageWords;
static __device__ __align__(256) uint64_t scratch[kNoAllocWords];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint64_t* g_scratch[kMaxDevices] = {};

/* Device address of `scratch` on the current device: looked up on the first
 * call on that device (with it current) and kept. */
int scratch_on_current_device(uint64_t** out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return HBHEAP_E_HIP;
    if (dev < 0 || dev >= kMaxDevices) return HBHEAP_E_UNSUP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return HBHEAP_E_HIP;
        g_scratch[dev] = (uint64_t*)p;
    }
    *out = g_scratch[dev];
    return HBHEAP_OK;
}
}  // namespace

extern "C" {

int heap_chunks_in_use_noalloc(heap_t h, uint64_t* out, hipStream_t stream)
{
    if (!h || !out) return HBHEAP_E_INVAL;
    hbheap_dev_t d;
    if (heap_device_handle(h, &d) != HBHEAP_OK) return HBHEAP_E_INVAL;
    if (1u + d.n_classes > kNoAllocWords) return HBHEAP_E_RANGE;
    uint64_t* sp = nullptr;
    const int rc = scratch_on_current_device(&sp);
    if (rc != HBHEAP_OK) return rc;
    /* k_usage writes every word it reports (the count and one per class of
     * this heap): nothing needs clearing first */
    hipLaunchKernelGGL(k_usage, dim3(1), dim3(64), 0, stream, d, sp);
    if (hipGetLastError() != hipSuccess) return HBHEAP_E_HIP;
    return hipMemcpyAsync(out, sp, 8, hipMemcpyDeviceToDevice, stream) == hipSuccess ? HBHEAP_OK : HBHEAP_E_HIP;
}

int heap_chunks_in_use(heap_t h, uint64_t* out, hipStream_t stream)
{
    if (!h || !out) return HBHEAP_E_INVAL;
    hbheap_dev_t d;
    if (heap_device_handle(h, &d) != HBHEAP_OK) return HBHEAP_E_INVAL;
    uint64_t* dv = nullptr;
    if (hipMalloc(&dv, kUsageBytes) != hipSuccess) return HBHEAP_E_NOMEM;
    hipLaunchKernelGGL(k_usage, dim3(1), dim3(64), 0, stream, d, dv);
    int rc = HBHEAP_OK;
    if (hipGetLastError() != hipSuccess || hipMemcpyAsync(out, dv, 8, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        rc = HBHEAP_E_HIP;
    (void)hipFree(dv);
    return rc;
}

int serve_create(heap_t h, const serve_config_t* cfg, server_t* out)
{
    if (!h || !cfg || !out) return HBHEAP_E_INVAL;
    const serve_config_t c = *cfg;
    if (c.slots == 0 || c.slots > kMaxSlots || c.max_batch == 0 || c.max_batch > kMaxBatch || c.max_requests == 0 ||
        c.max_requests > (1ull << 32) || !(c.admit > 0.0 && c.admit <= 1.0) || c.free_lag == 0)
        return HBHEAP_E_INVAL;
    hbheap_server* s = new (std::nothrow) hbheap_server();
    if (!s) return HBHEAP_E_NOMEM;
    s->heap = h;
    s->cfg = c;
    /* the virtualised page variants are refused: the classes of a shard
     * share one page budget there, and a request can fail with chunks left
     * in one shard and budget left in another, which no bound on chunks in
     * use (nor on the pages committed in total) rules out */
    if (heap_device_handle(h, &s->dev) != HBHEAP_OK || heap_info(h, &s->info) != HBHEAP_OK ||
        HBHEAP_VARIANT_SHARED_PAGES(s->info.variant)) {
        delete s;
        return HBHEAP_E_INVAL;
    }
    if (hipMalloc(&s->handles, 8ull * c.max_requests) != hipSuccess) { s->handles = nullptr; release(s); return HBHEAP_E_NOMEM; }
    if (hipStreamCreate(&s->mon) != hipSuccess || hipEventCreateWithFlags(&s->mon_done, hipEventDisableTiming) != hipSuccess ||
        hipMalloc(&s->usage_d, kUsageBytes) != hipSuccess ||
        hipHostMalloc(&s->usage_h, kUsageBytes, hipHostMallocDefault) != hipSuccess) {
        release(s);
        return HBHEAP_E_HIP;
    }
    /* page variant: class k owns at most min(shard chunks, queue entries /
     * pages per chunk) chunks of each shard (a request is served from any
     * shard, so this sum is the class's capacity) */
    s->class_cap.assign(s->info.n_classes, UINT64_MAX);
    if (s->info.variant == HBHEAP_VARIANT_PAGE) {
        const uint64_t N = s->info.n_chunks, span = 1ull << s->dev.log2_span;
        for (uint32_t k = 0; k < s->info.n_classes; ++k) {
            const uint64_t per = s->info.ring_entries / (s->info.chunk_bytes >> (4 + k));
            uint64_t cap = 0;
            for (uint64_t lo = 0; lo < N; lo += span) cap += std::min(std::min(N, lo + span) - lo, per);
            s->class_cap[k] = cap;
        }
    }
    s->slots.resize(c.slots);
    const uint64_t mb = c.max_batch;
    for (Slot& sl : s->slots) {
        if (hipStreamCreate(&sl.st) != hipSuccess || hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
            hipMalloc(&sl.ops_d, 8 * mb) != hipSuccess || hipMalloc(&sl.aux_d, 8 * mb) != hipSuccess ||
            hipMalloc(&sl.res_d, 8 * (mb + kUsageWords)) != hipSuccess ||
            hipMalloc(&sl.done_d, sizeof(uint32_t)) != hipSuccess ||
            hipHostMalloc(&sl.ops_h, 8 * mb, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc(&sl.aux_h, 8 * mb, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc(&sl.res_h, 8 * (mb + kUsageWords), hipHostMallocDefault) != hipSuccess) {
            release(s);
            return HBHEAP_E_NOMEM;
        }
        if (hipMemset(sl.done_d, 0, sizeof(uint32_t)) != hipSuccess) {
            release(s);
            return HBHEAP_E_HIP;
        }
    }
    *out = s;
    return HBHEAP_OK;
}

int serve_destroy(server_t s)
{
    if (!s) return HBHEAP_OK;
    int rc = HBHEAP_OK;
    for (Slot& sl : s->slots)
        if (sl.st && hipStreamSynchronize(sl.st) != hipSuccess) rc = HBHEAP_E_HIP;
    if (s->mon && hipStreamSynchronize(s->mon) != hipSuccess) rc = HBHEAP_E_HIP;
    release(s);
    return rc;
}

int serve_export(server_t s, uint64_t first, uint64_t n, uint64_t* dst, hipStream_t stream)
{
    if (!s || (n && !dst) || first > s->cfg.max_requests || n > s->cfg.max_requests - first) return HBHEAP_E_INVAL;
    if (!n) return HBHEAP_OK;
    hipLaunchKernelGGL(k_serve_export, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, stream, s->handles, first, n,
                       dst);
    return hipGetLastError() == hipSuccess ? HBHEAP_OK : HBHEAP_E_HIP;
}

int serve_run(server_t s, uint32_t nb, const uint64_t* first, const int64_t* ops, const uint64_t* arrival_ns,
              int alone, uint8_t* status, int8_t* cls, uint32_t* sum, uint64_t* latency_ns, uint64_t* wait_ns,
              serve_stats_t* stats)
{
    if (!s || !first || (nb && !ops) || (!alone && nb && !arrival_ns)) return HBHEAP_E_INVAL;
    const serve_config_t& c = s->cfg;
    const uint64_t C = s->info.chunk_bytes;
    const uint64_t R = nb ? first[nb] : 0;
    if (first[0] != 0 || R > c.max_requests) return HBHEAP_E_INVAL;
    const uint32_t K = s->info.n_classes;
    const bool per_class = s->info.variant == HBHEAP_VARIANT_PAGE;

    /* ---- validate the request list, size the frees, price the batches ---- */
    std::vector<uint64_t> aux(R, 0);
    std::vector<uint32_t> worst_k((size_t)nb * K, 0); /* fresh chunks a batch may take, per class */
    std::vector<uint64_t> worst(nb, 0);
    std::vector<uint32_t> batch_of(R);
    std::vector<uint8_t> freed(R, 0);
    const uint32_t width = s->dev.width ? s->dev.width : 64;
    for (uint32_t b = 0; b < nb; ++b) {
        if (first[b + 1] < first[b] || first[b + 1] - first[b] > c.max_batch) return HBHEAP_E_INVAL;
        if (!alone && b && arrival_ns[b] < arrival_ns[b - 1]) return HBHEAP_E_INVAL;
        for (uint64_t g0 = first[b]; g0 < first[b + 1]; g0 += width) {
            /* one aggregation group per (segment of `width` lanes, class):
             * a group never takes more than ceil(g / pages per chunk) chunks */
            uint32_t cnt[kMaxClasses] = {0};
            const uint64_t g1 = std::min<uint64_t>(first[b + 1], g0 + width);
            for (uint64_t i = g0; i < g1; ++i) {
                batch_of[i] = b;
                const int64_t op = ops[i];
                if (op >= 0) {
                    const int k = host_class((uint64_t)op, C);
                    if (k >= 0) ++cnt[k];
                    continue;
                }
                const uint64_t t = (uint64_t)(-(op + 1));
                if (t >= first[b] || ops[t] < 0 || freed[t] || batch_of[t] + c.free_lag > b) return HBHEAP_E_INVAL;
                freed[t] = 1;
                aux[i] = (uint64_t)ops[t];
            }
            for (uint32_t k = 0; k < K; ++k) {
                const uint64_t ppc = C >> (4 + k);
                const uint32_t w = (uint32_t)((cnt[k] + ppc - 1) / ppc);
                worst_k[(size_t)b * K + k] += w;
                worst[b] += w;
            }
        }
    }

    /* ---- the chunk budget ----
     * bound(now) = base + L, L = worst cases of every batch launched in this
     * run; a usage read resets base so that the bound is the read value plus
     * the worst cases of the batches not seen complete when it was issued.
     * The same per class (page variant), against the class capacities. */
    const uint64_t cap = (uint64_t)((double)s->info.n_chunks * c.admit);
    int64_t base = 0;
    uint64_t L = 0;
    std::vector<int64_t> base_k(K, 0);
    std::vector<uint64_t> L_k(K, 0);
    auto set_exact = [&]() {
        base = (int64_t)s->usage_h[0] - (int64_t)L;
        for (uint32_t k = 0; k < K; ++k) base_k[k] = (int64_t)s->usage_h[1 + k] - (int64_t)L_k[k];
    };
    auto admissible = [&](uint32_t b) {
        if (base + (int64_t)(L + worst[b]) > (int64_t)cap) return false;
        if (per_class)
            for (uint32_t k = 0; k < K; ++k) {
                const uint32_t w = worst_k[(size_t)b * K + k];
                if (w && base_k[k] + (int64_t)(L_k[k] + w) > (int64_t)s->class_cap[k]) return false;
            }
        return true;
    };

    serve_stats_t st;
    memset(&st, 0, sizeof(st));
    st.batches = nb;
    st.requests = R;
    for (uint64_t i = 0; i < R; ++i) (ops[i] >= 0 ? st.allocs : st.frees) += 1;

    for (Slot& sl : s->slots)
        if (hipStreamSynchronize(sl.st) != hipSuccess) return HBHEAP_E_HIP;
    if (usage_sync(s) != HBHEAP_OK) return HBHEAP_E_HIP;
    set_exact();

    /* per batch, fixed at its launch: L with it included, and the worst
     * cases of the other batches then in flight (not seen complete when its
     * usage words were read, at its end) */
    std::vector<uint64_t> at_L(nb, 0), at_out(nb, 0);
    std::vector<uint64_t> at_L_k((size_t)nb * K, 0), at_out_k((size_t)nb * K, 0);
    std::vector<uint8_t> done(nb, 0);
    uint32_t prefix = 0; /* batches [0, prefix) are complete */
    uint32_t next = 0, inflight = 0;
    std::vector<uint64_t> launch_ns(nb, 0);
    bool stalled = false;

    auto finish = [&](Slot& sl, uint64_t now) {
        const uint32_t b = (uint32_t)sl.batch;
        const uint64_t f = first[b], n = first[b + 1] - f;
        for (uint64_t i = 0; i < n; ++i) {
            const uint64_t r = sl.res_h[i];
            if (sum) sum[f + i] = (uint32_t)r;
            if (status) status[f + i] = (uint8_t)(r >> 32);
            if (cls) cls[f + i] = (int8_t)(uint8_t)(r >> 40);
        }
        if (n) {
            /* the usage words read at the batch's end: a bound from them
             * (the batches in flight at its launch keep their worst case,
             * as do those launched since); keep the tighter one */
            const uint64_t* u = sl.res_h + n;
            base = std::min(base, (int64_t)u[0] + (int64_t)at_out[b] - (int64_t)at_L[b]);
            for (uint32_t k = 0; k < K; ++k)
                base_k[k] = std::min(base_k[k], (int64_t)u[1 + k] + (int64_t)at_out_k[(size_t)b * K + k] -
                                                    (int64_t)at_L_k[(size_t)b * K + k]);
            ++st.monitor_reads;
        }
        if (latency_ns) latency_ns[b] = now - (alone ? launch_ns[b] : arrival_ns[b]);
        done[b] = 1;
        while (prefix < nb && done[prefix]) ++prefix;
        sl.batch = -1;
        --inflight;
    };
    auto launch = [&](Slot& sl, uint32_t b, uint64_t now) -> int {
        const uint64_t f = first[b], n = first[b + 1] - f;
        sl.batch = b;
        launch_ns[b] = now;
        if (wait_ns) wait_ns[b] = alone ? 0 : now - arrival_ns[b];
        uint64_t out = 0;
        for (const Slot& o : s->slots)
            if (o.batch >= 0 && &o != &sl) {
                out += worst[o.batch];
                for (uint32_t k = 0; k < K; ++k) at_out_k[(size_t)b * K + k] += worst_k[(size_t)o.batch * K + k];
            }
        at_out[b] = out;
        L += worst[b];
        for (uint32_t k = 0; k < K; ++k) L_k[k] += worst_k[(size_t)b * K + k];
        at_L[b] = L;
        for (uint32_t k = 0; k < K; ++k) at_L_k[(size_t)b * K + k] = L_k[k];
        st.peak_bound = std::max<uint64_t>(st.peak_bound, (uint64_t)(base + (int64_t)L));
        ++inflight;
        if (!n) return hipEventRecord(sl.done, sl.st) == hipSuccess ? HBHEAP_OK : HBHEAP_E_HIP;
        memcpy(sl.ops_h, ops + f, 8 * n);
        memcpy(sl.aux_h, aux.data() + f, 8 * n);
        if (hipMemcpyAsync(sl.ops_d, sl.ops_h, 8 * n, hipMemcpyHostToDevice, sl.st) != hipSuccess ||
            hipMemcpyAsync(sl.aux_d, sl.aux_h, 8 * n, hipMemcpyHostToDevice, sl.st) != hipSuccess)
            return HBHEAP_E_HIP;
        hipLaunchKernelGGL(k_serve_batch, dim3((uint32_t)((n + kServeBlock - 1) / kServeBlock)), dim3(kServeBlock), 0,
                           sl.st, s->dev, sl.ops_d, sl.aux_d, (uint32_t)n, f, s->handles, sl.res_d, c.seed, sl.done_d);
        if (hipGetLastError() != hipSuccess) return HBHEAP_E_HIP;
        /* results and the usage words after them, in one copy */
        if (hipMemcpyAsync(sl.res_h, sl.res_d, 8 * (n + 1 + K), hipMemcpyDeviceToHost, sl.st) != hipSuccess)
            return HBHEAP_E_HIP;
        return hipEventRecord(sl.done, sl.st) == hipSuccess ? HBHEAP_OK : HBHEAP_E_HIP;
    };
    /* quiescent trim and exact recount; the caller made sure nothing runs */
    auto trim_recount = [&]() -> int {
        if (heap_trim(s->heap, s->mon) != HBHEAP_OK) return HBHEAP_E_HIP;
        if (usage_sync(s) != HBHEAP_OK) return HBHEAP_E_HIP;
        set_exact();
        ++st.trims;
        return HBHEAP_OK;
    };

    const Clock::time_point t0 = Clock::now();
    if (alone) {
        Slot& sl = s->slots[0];
        for (uint32_t b = 0; b < nb; ++b) {
            if (!admissible(b)) {
                ++st.admission_stalls;
                if (trim_recount() != HBHEAP_OK) return HBHEAP_E_HIP;
                if (!admissible(b)) return HBHEAP_E_NOMEM;
            }
            if (launch(sl, b, ns_since(t0)) != HBHEAP_OK) return HBHEAP_E_HIP;
            if (hipEventSynchronize(sl.done) != hipSuccess) return HBHEAP_E_HIP;
            /* nothing else in flight: the usage words the batch read at its
             * end make the count exact */
            finish(sl, ns_since(t0));
        }
    } else {
        while (next < nb || inflight) {
            const uint64_t now = ns_since(t0);
            bool progress = false;
            for (Slot& sl : s->slots) {
                if (sl.batch < 0) continue;
                const hipError_t q = hipEventQuery(sl.done);
                if (q == hipSuccess) {
                    finish(sl, ns_since(t0));
                    progress = true;
                } else if (q != hipErrorNotReady) {
                    return HBHEAP_E_HIP;
                }
            }
            if (next < nb && now >= arrival_ns[next] && prefix + c.free_lag > next) {
                const uint32_t b = next;
                Slot* free_sl = nullptr;
                for (Slot& sl : s->slots)
                    if (sl.batch < 0) { free_sl = &sl; break; }
                if (free_sl) {
                    if (admissible(b)) {
                        if (launch(*free_sl, b, ns_since(t0)) != HBHEAP_OK) return HBHEAP_E_HIP;
                        ++next;
                        stalled = false;
                        progress = true;
                    } else {
                        if (!stalled) ++st.admission_stalls;
                        stalled = true;
                        if (!inflight) {
                            /* quiescent: first an exact count, then, if that
                             * is not enough, a trim */
                            if (usage_sync(s) != HBHEAP_OK) return HBHEAP_E_HIP;
                            set_exact();
                            if (!admissible(b)) {
                                if (trim_recount() != HBHEAP_OK) return HBHEAP_E_HIP;
                                if (!admissible(b)) return HBHEAP_E_NOMEM;
                            }
                            progress = true;
                        }
                    }
                }
            }
            if (!progress) std::this_thread::yield();
        }
    }
    st.wall_s = (double)ns_since(t0) * 1e-9;
    if (usage_sync(s) != HBHEAP_OK) return HBHEAP_E_HIP;
    st.final_chunks = s->usage_h[0];
    if (stats) *stats = st;
    return HBHEAP_OK;
}

}  // extern "C"
