/*
 * hbheap.hip -- host library and kernels of the device heap allocator
 * (C ABI in include/hbheap.h, device API in include/hbheap_device.h).
 *
 * Contents:
 *   - heap creation: state-region layout (snapshot version 4) and init;
 *   - batch alloc / free kernels (one lane per request, 256-lane blocks);
 *   - single-lane replay kernel;
 *   - quiescent trim: retire fully free chunks, rebuild pool and queues in
 *     ascending order (a counting pass, a scan, a writing pass);
 *   - payload pattern write/check (the paper's driver writes data into each
 *     block and checks it on read-back, Methods);
 *   - measurement kernels: device atomic probes and an HBM copy.
 * The plain baseline (the runtime's own device malloc/free) is in
 * plain_baseline.hip.
 */
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <new>
#include <vector>

#include "hbheap.h"
#include "hbheap_device.h"
#include "pattern.h"

using namespace hbheap::detail;

namespace {

constexpr uint32_t kMagic = 0x48424850u;
constexpr uint32_t kVersion = 4;
constexpr uint32_t kBatchBlock = 256;
constexpr uint32_t kTrimBlock = 1024;
constexpr uint32_t kMaxKeys = 1024; /* trim keys: 64 shards x (13 classes + pool) + none */
constexpr uint32_t kMaxShards = 64;

struct Layout {
    uint64_t off_pool, off_cl, off_cls, off_cnt, off_bits, off_pid, off_sl, total;
    uint32_t log2q;
    uint64_t n_slots; /* u32 slots of the ring storage */
    /* virtualised array variants */
    uint64_t off_vdir = 0, off_vtaken = 0, off_vstore = 0, off_vslots = 0;
    uint32_t log2_seg = 0, log2_dir = 0, log2_store = 0, vsegs = 0;
    uint64_t vbudget = 0;
    /* eager retirement: count and token words, and pool ids padded to
     * S << log2_span (one ring of 2^log2_span slots per shard) */
    uint64_t off_ct = 0;
    uint64_t n_pid = 0;
};

uint64_t al256(uint64_t x) { return (x + 255) & ~255ull; }
uint32_t ilog2(uint64_t x) { uint32_t r = 0; while (x >>= 1) ++r; return r; }
uint32_t ceil_log2(uint64_t x) { uint32_t r = 0; while ((1ull << r) < x) ++r; return r; }

}  // namespace

struct hbheap_heap {
    hbheap_dev_t dev;
    Layout lay;
    void* data = nullptr;
    void* state = nullptr;
    void* aux = nullptr;      /* err word, stats, trim workspace */
    uint32_t* trim_counts = nullptr;
    uint32_t* trim_offsets = nullptr;
    uint32_t* trim_totals = nullptr;
    uint32_t* trim_owned = nullptr;
    uint32_t trim_blocks = 0;
    uint32_t owned_words = 0;
    uint64_t aux_bytes = 0;
    uint64_t shard_stat_bytes = 0;
    uint64_t chunk_bytes = 0;
    uint32_t rows = 1; /* requests per lane of the batch kernels (1 or 4) */
};

#define HB_TRY(expr)                                \
    do {                                            \
        if ((expr) != hipSuccess) return HBHEAP_E_HIP; \
    } while (0)

/* ======================================================================= */
/* kernels                                                                 */
/* ======================================================================= */

__global__ void k_fill_u32(uint32_t* p, uint64_t n, uint32_t v)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_u64(uint64_t* p, uint64_t n, uint64_t v)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_u8(uint8_t* p, uint64_t n, uint8_t v)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_iota_u32(uint32_t* p, uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = (uint32_t)i;
}

/* Batch kernels.  The Counted instances run when HBHEAP_FLAG_STATS is set
 * (measurement passes) and carry their own symbol, so profiles of the
 * plain instances are not mixed with counting launches. */
/* Occupancy target of the allocation kernel (waves per SIMD); 0 leaves the
 * choice to the compiler. */
#ifndef HBHEAP_ALLOC_WAVES
#define HBHEAP_ALLOC_WAVES 0
#endif
#if HBHEAP_ALLOC_WAVES > 0
#define HBHEAP_ALLOC_ATTR __attribute__((amdgpu_waves_per_eu(HBHEAP_ALLOC_WAVES, 8)))
#else
/* 4 requests per lane: 2^20 requests are 4096 waves, 4 per SIMD, so ask for
 * that occupancy (at most 128 VGPRs) and have every wave resident */
#define HBHEAP_ALLOC_ATTR __attribute__((amdgpu_waves_per_eu(R == 4 ? 4 : 1, 8)))
#endif

/* The batch kernels come in one instance per heap variant V (the host
 * launches the heap's own): with h.variant a constant, every variant test of
 * the inlined device code folds, and each instance carries only its
 * variant's code.  V = kChunkEager is the chunk variant with eager
 * retirement, an instance of its own for the same reason (and so that the
 * lazy instance keeps its register budget).  R: requests per lane.  Wave w serves requests
 * [64 R w, 64 R (w + 1)), row r of it on lanes l at 64 R w + 64 r + l, so
 * that each row's loads and stores are contiguous; every lane of a wave
 * stays active (rows past n carry no request). */
constexpr uint32_t kChunkEager = 6;
template <uint32_t V>
__device__ __forceinline__ void batch_variant(hbheap_dev_t& h)
{
    h.variant = V == kChunkEager ? (uint32_t)HBHEAP_VARIANT_CHUNK : V;
    if (V == kChunkEager) h.flags |= HBHEAP_FLAG_EAGER;
    else h.flags &= ~HBHEAP_FLAG_EAGER;
}

template <bool Counted, uint32_t V, uint32_t R>
__global__ void __launch_bounds__(kBatchBlock) HBHEAP_ALLOC_ATTR k_alloc_batch(hbheap_dev_t h, const uint64_t* __restrict__ sizes,
                                                             void** __restrict__ ptrs, uint64_t n)
{
    /* out-of-memory proofs shared by the waves of this workgroup */
    __shared__ uint32_t share[kShareSlots];
    if (threadIdx.x < kShareSlots) share[threadIdx.x] = kShareFree;
    __syncthreads();
    const uint64_t wave = ((uint64_t)blockIdx.x * kBatchBlock + threadIdx.x) >> 6;
    const uint64_t base = wave * 64u * R + lane();
    if (wave * 64u * R >= n) return;
    batch_variant<V>(h);
    if (Counted) h.flags |= HBHEAP_FLAG_STATS;
    else h.flags &= ~HBHEAP_FLAG_STATS;
    /* home shard: the linear wave index, spread evenly over the shards (a
     * wave-uniform 32-bit remainder, taken on the scalar unit); its pool hint
     * is loaded before the sizes so that the loads are in flight together
     * (the empty asm keeps the compiler from sinking it) */
    const uint32_t wv = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)wave);
    const uint32_t home = wv % h.n_shards;
    const bool dry = home_pool_dry(h, home);
    __asm__ volatile("" ::: "memory");
    /* requests past n load the wave's first size (index wave * 64 R < n, in
     * bounds) and carry no request: no branch per row */
    uint64_t sz[R];
    bool has[R];
#pragma unroll
    for (uint32_t r = 0; r < R; ++r) {
        has[r] = base + 64u * r < n;
        sz[r] = sizes[has[r] ? base + 64u * r : wave * 64u * R];
        sz[r] = has[r] ? sz[r] : 0;
    }
    Rows<R> q;
    malloc_rows<R>(h, q, sz, has, home, dry, share);
#pragma unroll
    for (uint32_t r = 0; r < R; ++r)
        if (has[r]) ptrs[base + 64u * r] = q.off[r] == kNoPage ? nullptr : (void*)(h.data + q.off[r]);
}

template <bool Counted, uint32_t V, uint32_t R>
__global__ void __launch_bounds__(kBatchBlock) k_free_batch(hbheap_dev_t h, const uint64_t* __restrict__ sizes,
                                                            void* const* __restrict__ ptrs, uint64_t n,
                                                            int32_t* __restrict__ status)
{
    const uint64_t wave = ((uint64_t)blockIdx.x * kBatchBlock + threadIdx.x) >> 6;
    const uint64_t base = wave * 64u * R + lane();
    if (wave * 64u * R >= n) return;
    batch_variant<V>(h);
    if (Counted) h.flags |= HBHEAP_FLAG_STATS;
    else h.flags &= ~HBHEAP_FLAG_STATS;
    void* p[R];
    uint64_t hint[R];
    bool has[R];
#pragma unroll
    for (uint32_t r = 0; r < R; ++r) {
        has[r] = base + 64u * r < n;
        p[r] = has[r] ? ptrs[base + 64u * r] : nullptr;
        hint[r] = has[r] && sizes ? sizes[base + 64u * r] : 0;
    }
    uint32_t st[R];
    free_rows<R>(h, p, hint, sizes != nullptr, st);
    if (status) {
#pragma unroll
        for (uint32_t r = 0; r < R; ++r)
            if (has[r]) status[base + 64u * r] = (int32_t)st[r];
    }
}

/* One lane runs the op list in order. */
__global__ void k_replay(hbheap_dev_t h, const int64_t* ops, int64_t* out, uint64_t n)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    h.flags |= HBHEAP_FLAG_HOME0;
    for (uint64_t i = 0; i < n; ++i) {
        const int64_t op = ops[i];
        if (op >= 0) {
            void* p = malloc_wave(h, (uint64_t)op, 0, home_pool_dry(h, 0));
            out[i] = p ? (int64_t)((uint8_t*)p - h.data) : -1;
        } else {
            const uint64_t j = (uint64_t)(-op - 1);
            const int64_t o = j < i ? out[j] : -1;
            void* p = o >= 0 ? (void*)(h.data + o) : nullptr;
            out[i] = (int64_t)free_wave(h, p, 0, false);
        }
    }
}

/* ---------------- trim ---------------- */

/* Keys of the trim compaction: ring (shard j, class k) = j*K + k; pool of
 * shard j = S*K + j; nothing = S*(K+1).  A chunk contributes `weight`
 * entries under its key: an unowned chunk one pool id, a chunk-variant chunk
 * with free pages its id, a page-variant chunk its free pages. */
struct TrimKey {
    uint32_t key, weight;
};

__device__ __forceinline__ uint32_t trim_nkeys(const hbheap_dev_t& h) { return h.n_shards * (h.n_classes + 1) + 1; }

__device__ __forceinline__ TrimKey trim_key(const hbheap_dev_t& h, uint64_t c)
{
    TrimKey t;
    const uint32_t j = shard_of_chunk(h, c);
    const uint32_t k = h.chunk_class[c];
    if (k == kFreeClass) {
        t.key = h.n_shards * h.n_classes + j;
        t.weight = 1;
        return t;
    }
    if (HBHEAP_VARIANT_LISTS_CHUNKS(h.variant)) {
        const bool listed = eager(h) ? ct_count(h.chunk_ct[c]) > 0 : h.chunk_cnt[c] > 0;
        t.key = listed ? j * h.n_classes + k : h.n_shards * (h.n_classes + 1);
        t.weight = listed ? 1u : 0u;
    } else {
        uint32_t f = 0;
        const uint32_t ppc = 1u << (h.log2_chunk - 4u - k);
        const uint32_t nw = ppc >= 64u ? ppc >> 6 : 1u;
        for (uint32_t w = 0; w < nw; ++w) f += (uint32_t)__popcll(h.bits[bit_index(h, c, w)]);
        t.key = j * h.n_classes + k;
        t.weight = f;
    }
    return t;
}

/* Pass 1: retire fully free chunks, count entries per key per block, and
 * count the chunks each (shard, class) keeps. */
__global__ void __launch_bounds__(kTrimBlock) k_trim_count(hbheap_dev_t h, uint32_t* counts, uint32_t nblocks,
                                                           uint32_t* owned)
{
    __shared__ uint32_t cnt[kMaxKeys], own[kMaxKeys];
    const uint32_t nkeys = trim_nkeys(h);
    for (uint32_t i = threadIdx.x; i < kMaxKeys; i += kTrimBlock) {
        cnt[i] = 0;
        own[i] = 0;
    }
    __syncthreads();
    const uint64_t c = (uint64_t)blockIdx.x * kTrimBlock + threadIdx.x;
    if (c < h.n_chunks) {
        const uint32_t k = h.chunk_class[c];
        if (k != kFreeClass) {
            const uint32_t ppc = 1u << (h.log2_chunk - 4u - k);
            const uint32_t nw = ppc >= 64u ? ppc >> 6 : 1u;
            uint32_t f = 0;
            for (uint32_t w = 0; w < nw; ++w) f += (uint32_t)__popcll(h.bits[bit_index(h, c, w)]);
            if (f == ppc) {
                for (uint32_t w = 0; w < h.words_per_chunk; ++w) h.bits[bit_index(h, c, w)] = 0;
                h.chunk_cnt[c] = 0;
                if (eager(h)) h.chunk_ct[c] = ct_word(kTokNone, 0);
                h.chunk_class[c] = (uint8_t)kFreeClass;
            } else {
                atomicAdd(&own[shard_of_chunk(h, c) * h.n_classes + k], 1u);
            }
        }
        const TrimKey t = trim_key(h, c);
        if (t.weight) atomicAdd(&cnt[t.key], t.weight);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < nkeys; i += kTrimBlock) {
        counts[(uint64_t)i * nblocks + blockIdx.x] = cnt[i];
        if (i < h.n_shards * h.n_classes && own[i]) atomicAdd(&owned[i], own[i]);
    }
}

/* Pass 2: per key, exclusive scan of the block counts. */
__global__ void k_trim_scan(const uint32_t* counts, uint32_t* offsets, uint32_t* totals, uint32_t nblocks, uint32_t nkeys)
{
    for (uint32_t key = threadIdx.x; key < nkeys; key += blockDim.x) {
        uint32_t run = 0;
        for (uint32_t b = 0; b < nblocks; ++b) {
            offsets[(uint64_t)key * nblocks + b] = run;
            run += counts[(uint64_t)key * nblocks + b];
        }
        totals[key] = run;
    }
}

/* Block-wide exclusive scan of v over the 1024 threads (all active). */
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* wsum)
{
    const uint32_t me = lane(), wave = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (me >= (uint32_t)d) x += y;
    }
    if (me == 63) wsum[wave] = x;
    __syncthreads();
    if (threadIdx.x < 64) {
        uint32_t s = threadIdx.x < kTrimBlock / 64 ? wsum[threadIdx.x] : 0;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t y = __shfl_up(s, d, 64);
            if (me >= (uint32_t)d) s += y;
        }
        if (threadIdx.x < kTrimBlock / 64) wsum[threadIdx.x] = s;
    }
    __syncthreads();
    const uint32_t before = wave ? wsum[wave - 1] : 0u;
    const uint32_t r = before + x - v;
    __syncthreads();
    return r;
}

/* Pass 3: write pool ids and ring entries in ascending chunk (page) order,
 * for the keys of the shards this block's chunks belong to. */
/* Segmented queues after a trim (totals == nullptr: at creation, all
 * empty): queue (j, k) holds its entries at positions 0 .. totals[j*K+k]-1
 * in segments numbered from the shard's first, queue after queue.  A
 * virtualised list queue always keeps one segment, even when empty. */
__device__ __forceinline__ uint32_t seg_used(const hbheap_dev_t& h, const uint32_t* totals, uint32_t j, uint32_t k)
{
    const uint32_t g = 1u << h.log2_seg;
    const uint32_t n = totals ? (totals[j * h.n_classes + k] + g - 1u) >> h.log2_seg : 0u;
    return HBHEAP_VARIANT_IS_VL(h.variant) && n == 0 ? 1u : n;
}
__device__ __forceinline__ uint32_t va_first_seg(const hbheap_dev_t& h, const uint32_t* totals, uint32_t j, uint32_t k)
{
    uint32_t base = 0;
    for (uint32_t kk = 0; kk < k; ++kk) base += seg_used(h, totals, j, kk);
    return base;
}

__global__ void __launch_bounds__(kTrimBlock) k_trim_write(hbheap_dev_t h, const uint32_t* offsets, uint32_t nblocks,
                                                           const uint32_t* totals)
{
    __shared__ uint32_t wsum[kTrimBlock / 64];
    const uint64_t c0 = (uint64_t)blockIdx.x * kTrimBlock;
    const uint64_t c = c0 + threadIdx.x;
    const uint64_t c_last = (c0 + kTrimBlock <= h.n_chunks ? c0 + kTrimBlock : h.n_chunks) - 1;
    TrimKey t;
    t.key = h.n_shards * (h.n_classes + 1);
    t.weight = 0;
    if (c < h.n_chunks) t = trim_key(h, c);
    const uint64_t Q = 1ull << h.log2q;
    const uint32_t K = h.n_classes, S = h.n_shards;
    const uint32_t j0 = shard_of_chunk(h, c0), j1 = shard_of_chunk(h, c_last);
    for (uint32_t j = j0; j <= j1; ++j) {
        for (uint32_t kk = 0; kk <= K; ++kk) {
            const uint32_t key = kk < K ? j * K + kk : S * K + j;
            const uint32_t w = t.key == key ? t.weight : 0u;
            const uint32_t pos = offsets[(uint64_t)key * nblocks + blockIdx.x] + block_excl_scan(w, wsum);
            if (!w) continue;
            if (kk == K) {
                const uint64_t idx = ((uint64_t)j << h.log2_span) + pos;
                if (idx < h.n_chunks) h.pool_ids[idx] = (uint32_t)c;
            } else if (h.variant == HBHEAP_VARIANT_CHUNK) {
                if (pos < Q) h.slots[(uint64_t)key * Q + pos] = (uint32_t)c;
                if (eager(h)) h.chunk_ct[c] = ct_word(tok_listed(kk, pos), ct_count(h.chunk_ct[c]));
            } else if (HBHEAP_VARIANT_SEGMENTED(h.variant) && HBHEAP_VARIANT_LISTS_CHUNKS(h.variant)) {
                const uint64_t seg = va_first_seg(h, totals, j, kk) + (pos >> h.log2_seg);
                if (seg < h.vsegs)
                    h.slots[(((uint64_t)j * h.vsegs + seg) << h.log2_seg) + (pos & ((1u << h.log2_seg) - 1u))] =
                        (uint32_t)c;
            } else {
                const uint32_t shift = 4u + kk;
                const uint32_t ppc = 1u << (h.log2_chunk - shift);
                const uint32_t nw = ppc >= 64u ? ppc >> 6 : 1u;
                uint32_t q = pos;
                const bool va = HBHEAP_VARIANT_SEGMENTED(h.variant);
                const uint32_t seg0 = va ? va_first_seg(h, totals, j, kk) : 0u;
                for (uint32_t wd = 0; wd < nw; ++wd) {
                    uint64_t x = h.bits[bit_index(h, c, wd)];
                    while (x) {
                        const uint32_t b = ctz64(x);
                        x &= x - 1ull;
                        const uint64_t off = (c << h.log2_chunk) + ((uint64_t)(wd * 64u + b) << shift);
                        if (va) {
                            const uint64_t seg = seg0 + (q >> h.log2_seg);
                            if (seg < h.vsegs)
                                h.slots[(((uint64_t)j * h.vsegs + seg) << h.log2_seg) + (q & ((1u << h.log2_seg) - 1u))] =
                                    (uint32_t)(off >> 4);
                        } else if (q < Q) {
                            h.slots[(uint64_t)key * Q + q] = (uint32_t)(off >> 4);
                        }
                        ++q;
                    }
                }
            }
        }
    }
    /* eager retirement: an owned chunk with no free page has no token; the
     * queues were rewritten without stale entries, so no flag stays set */
    if (eager(h) && c < h.n_chunks && (h.chunk_class[c] == kFreeClass || t.weight == 0))
        h.chunk_ct[c] = ct_word(kTokNone, 0);
}

/* Pass 4: queue control words and pool counters. */
__global__ void k_trim_ctl(hbheap_dev_t h, const uint32_t* totals, const uint32_t* owned)
{
    const uint32_t K = h.n_classes, S = h.n_shards;
    for (uint32_t i = threadIdx.x; i < S * K; i += blockDim.x) {
        uint8_t* cb = h.classes + (uint64_t)i * kClassBlock;
        *(uint64_t*)cb = (uint64_t)(totals[i] + kBias);
        *(uint32_t*)(cb + 128) = 0;
        *(uint32_t*)(cb + 256) = totals[i];
        *(uint64_t*)(cb + 384) = !HBHEAP_VARIANT_LISTS_CHUNKS(h.variant) ? (uint64_t)owned[i] : 0ull;
    }
    for (uint32_t j = threadIdx.x; j < S; j += blockDim.x) {
        uint64_t* pb = h.pool + 16ull * j;
        if (eager(h)) { /* pool ring: the free chunks at positions 0 .. n-1 */
            pb[0] = (uint64_t)totals[S * K + j] + kBias;
            ((uint32_t*)pb)[4] = 0;
            ((uint32_t*)pb)[5] = totals[S * K + j];
        } else {
            pb[0] = 0;
            ((uint32_t*)pb)[2] = totals[S * K + j];
        }
    }
}

/* Virtualised array queues, all at once (heap creation: totals == nullptr,
 * every queue empty; trim: queue (j, k) holds totals[j*K+k] entries written
 * by k_trim_write): directories name the segments in use, every segment's
 * consumed count is zero, each shard's store holds its unused segment ids
 * in ascending order, and the shard's committed pages are those its
 * classes own. */
__global__ void k_va_rebuild(hbheap_dev_t h, const uint32_t* totals, const uint32_t* owned)
{
    const uint32_t S = h.n_shards, K = h.n_classes, M = h.vsegs;
    const uint64_t D = 1ull << h.log2_dir, QS = 1ull << h.log2_store;
    const bool vl = HBHEAP_VARIANT_IS_VL(h.variant);
    const uint64_t n_dir = vl ? (uint64_t)S * M : (uint64_t)S * K * D, n_taken = (uint64_t)S * M,
                   n_store = (uint64_t)S * QS;
    const uint64_t n = n_dir > n_store ? (n_dir > n_taken ? n_dir : n_taken) : (n_store > n_taken ? n_store : n_taken);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        if (i < n_dir && !vl) {
            const uint64_t q = i >> h.log2_dir, dd = i & (D - 1);
            const uint32_t j = (uint32_t)(q / K), k = (uint32_t)(q % K);
            const uint32_t used = seg_used(h, totals, j, k);
            const uint32_t base = va_first_seg(h, totals, j, k);
            h.vdir[i] = dd < used && base + dd < M ? ((dd << 32) | (uint64_t)(base + (uint32_t)dd)) : kDirEmpty;
        }
        if (i < n_dir && vl) {
            /* segment m of shard j: tag (queue << 32 | number) and link to
             * the next segment of its queue, or no tag and no link */
            const uint32_t j = (uint32_t)(i / M), m = (uint32_t)(i % M);
            uint64_t tag = ~0ull, next = kNoLink;
            uint32_t base = 0;
            for (uint32_t k = 0; k < K; ++k) {
                const uint32_t used = seg_used(h, totals, j, k);
                if (m < base + used) {
                    tag = ((uint64_t)k << 32) | (m - base);
                    next = m + 1u < base + used ? (uint64_t)(m + 1u) : kNoLink;
                    break;
                }
                base += used;
            }
            h.vdir[i] = tag;
            h.vdir[(uint64_t)S * M + i] = next;
        }
        if (vl && i < (uint64_t)S * K) {
            /* queue front and back: its first and last segment */
            const uint32_t j = (uint32_t)(i / K), k = (uint32_t)(i % K);
            const uint32_t used = seg_used(h, totals, j, k), base = va_first_seg(h, totals, j, k);
            uint8_t* cb = h.classes + i * kClassBlock;
            *(uint64_t*)(cb + 392) = (uint64_t)base;
            *(uint64_t*)(cb + 400) = ((uint64_t)(used - 1u) << 32) | (uint64_t)(base + used - 1u);
        }
        if (i < n_taken) h.vtaken[i] = 0;
        if (i < n_store) {
            const uint32_t j = (uint32_t)(i >> h.log2_store);
            const uint32_t p = (uint32_t)(i & (QS - 1));
            const uint32_t used = va_first_seg(h, totals, j, K);
            const uint32_t free_n = used < M ? M - used : 0u;
            h.vstore_slots[i] = p < free_n ? used + p : kEmpty;
        }
        if (i < S) {
            const uint32_t j = (uint32_t)i;
            const uint32_t used0 = va_first_seg(h, totals, j, K);
            const uint32_t used = used0 < M ? used0 : M;
            uint64_t pages = 0;
            if (owned && HBHEAP_VARIANT_SHARED_PAGES(h.variant))
                for (uint32_t k = 0; k < K; ++k) pages += (uint64_t)owned[j * K + k] << (h.log2_chunk - 4u - k);
            uint8_t* sb = h.vstore + (uint64_t)j * kStoreBlock;
            *(uint64_t*)sb = (uint64_t)(M - used) + kBias;
            *(uint32_t*)(sb + 128) = 0;
            *(uint32_t*)(sb + 256) = M - used;
            *(uint64_t*)(sb + 384) = pages;
        }
    }
}

/* ---------------- payload pattern (pattern.h) ---------------- */

constexpr uint64_t kCoopBytes = 1024;

__global__ void __launch_bounds__(kBatchBlock) k_pattern(void* const* ptrs, const uint64_t* sizes, uint64_t n,
                                                         uint32_t seed, unsigned long long* mismatches, int check,
                                                         const uint8_t* lo, uint64_t span)
{
    const uint64_t i = (uint64_t)blockIdx.x * kBatchBlock + threadIdx.x;
    if (i >= n) return;
    uint8_t* p = (uint8_t*)ptrs[i];
    uint64_t size = p ? sizes[i] : 0;
    const uint32_t sr = seed ^ fmix32((uint32_t)i);
    uint32_t bad = 0;
    /* only blocks that lie inside the heap's data region are touched */
    if (size && (p < lo || (uint64_t)(p - lo) >= span || span - (uint64_t)(p - lo) < size)) {
        size = 0;
        bad = 1;
    }
    const bool coop = size >= kCoopBytes;
    if (!coop && size) {
        if (check) bad += pat_check_range(p, size, sr, 0, 1);
        else pat_write_range(p, size, sr, 0, 1);
    }
    /* large blocks: the active lanes of the wave write one block at a time,
     * 16 B per lane (the last wave of the grid may be partial) */
    uint64_t big = __ballot(coop);
    const uint32_t me = lane();
    const uint64_t act = exec_mask();
    const uint32_t nact = (uint32_t)__popcll(act), r = rank_in(act);
    while (big) {
        const uint32_t l = ctz64(big);
        big &= big - 1ull;
        uint8_t* bp = (uint8_t*)bcast64((uint64_t)p, l);
        const uint64_t bs = bcast64(size, l);
        const uint32_t bsr = bcast(sr, l);
        const uint64_t nq = bs >> 4;
        if (check) {
            const uint4* q = (const uint4*)bp;
            for (uint64_t u = r; u < nq; u += nact) {
                const uint32_t j = (uint32_t)(u * 4);
                const uint4 v = q[u];
                bad += (v.x != pat_word(bsr, j)) + (v.y != pat_word(bsr, j + 1)) + (v.z != pat_word(bsr, j + 2)) +
                       (v.w != pat_word(bsr, j + 3));
            }
        } else {
            uint4* q = (uint4*)bp;
            for (uint64_t u = r; u < nq; u += nact) {
                const uint32_t j = (uint32_t)(u * 4);
                q[u] = make_uint4(pat_word(bsr, j), pat_word(bsr, j + 1), pat_word(bsr, j + 2), pat_word(bsr, j + 3));
            }
        }
        if (me == l && (bs & 15)) {
            /* tail bytes of the owner's block */
            if (check) {
                for (uint64_t b = nq << 4; b < bs; b += 4) {
                    const uint32_t w = pat_word(bsr, (uint32_t)(b >> 2));
                    bool ok = true;
                    for (uint64_t e = b; e < bs && e < b + 4; ++e) ok &= bp[e] == (uint8_t)(w >> (8 * (e & 3)));
                    bad += ok ? 0u : 1u;
                }
            } else {
                for (uint64_t b = nq << 4; b < bs; ++b) {
                    const uint32_t w = pat_word(bsr, (uint32_t)(b >> 2));
                    bp[b] = (uint8_t)(w >> (8 * (b & 3)));
                }
            }
        }
    }
    if (check) {
        const uint64_t any = __ballot(bad != 0);
        if (any) atomicAdd(mismatches, (unsigned long long)bad);
    }
}

/* ---------------- measurement ---------------- */

__device__ __forceinline__ uint32_t hash32(uint64_t x)
{
    return fmix32((uint32_t)x ^ fmix32((uint32_t)(x >> 32) + 0x9E3779B9u));
}

__global__ void __launch_bounds__(kBatchBlock) k_atomic_probe(int pattern, uint64_t* buf, uint64_t words64, uint32_t lines,
                                                              uint32_t iters, uint64_t threads)
{
    const uint64_t tid = (uint64_t)blockIdx.x * kBatchBlock + threadIdx.x;
    if (tid >= threads) return;
    const uint64_t wave = tid >> 6;
    const uint32_t me = lane();
    uint64_t acc = 0;
    switch (pattern) {
    case 0:
        if (me == 0)
            for (uint32_t it = 0; it < iters; ++it) acc += a_add64(buf, 1);
        break;
    case 1:
        if (me == 0)
            for (uint32_t it = 0; it < iters; ++it) acc += a_add64(buf + (wave % lines) * 16, 1);
        break;
    case 2: {
        uint32_t* w32 = (uint32_t*)buf;
        const uint64_t words32 = words64 * 2;
        for (uint32_t it = 0; it < iters; ++it) acc += a_add32(w32 + hash32(tid * 131u + it) % words32, 1u);
        break;
    }
    case 3:
        if (me == 0)
            for (uint32_t it = 0; it < iters; ++it) {
                uint64_t expect = a_load64(buf);
                const bool ok = __hip_atomic_compare_exchange_strong(buf, &expect, expect + 1, __ATOMIC_RELAXED,
                                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                acc += ok ? 1 : expect;
            }
        break;
    case 4:
        for (uint32_t it = 0; it < iters; ++it) acc += a_add64(buf + 16, 1);
        break;
    case 5: {
        /* lane-contiguous 32-bit exchanges: a wave covers 256 consecutive bytes */
        uint32_t* w32 = (uint32_t*)buf;
        const uint64_t words32 = words64 * 2;
        for (uint32_t it = 0; it < iters; ++it) acc += a_xchg32(w32 + (tid + (uint64_t)it * threads) % words32, 7u);
        break;
    }
    case 6: {
        /* lane-contiguous coherent 32-bit load then store (no read-modify-write) */
        uint32_t* w32 = (uint32_t*)buf;
        const uint64_t words32 = words64 * 2;
        for (uint32_t it = 0; it < iters; ++it) {
            uint32_t* q = w32 + (tid + (uint64_t)it * threads) % words32;
            const uint32_t v = a_load32(q);
            __hip_atomic_store(q, v + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            acc += v;
        }
        break;
    }
    case 7: {
        /* lane-contiguous coherent 64-bit load then store */
        for (uint32_t it = 0; it < iters; ++it) {
            uint64_t* q = buf + (tid + (uint64_t)it * threads) % words64;
            const uint64_t v = a_load64(q);
            __hip_atomic_store(q, v + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            acc += v;
        }
        break;
    }
    case 8: {
        /* a chain of dependent round trips: each lane's next 32-bit atomic
         * add waits for the value of its previous one (its address depends
         * on it), lanes on consecutive words -- the latency floor of a kernel
         * whose waves each run `iters` such round trips one after another */
        uint32_t* w32 = (uint32_t*)buf;
        const uint64_t words32 = words64 * 2;
        uint32_t v = 0;
        for (uint32_t it = 0; it < iters; ++it) {
            v = a_add32(w32 + (tid + (uint64_t)it * threads) % words32 + zero_after(v), 1u);
            acc += v;
        }
        break;
    }
    default:
        break;
    }
    /* keep the returned values live so the atomics stay returning ones */
    if (acc == 0x5EED5EED5EED5EEDull) buf[32] = acc;
}

__global__ void k_copy(uint4* __restrict__ dst, const uint4* __restrict__ src, uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

/* ======================================================================= */
/* host side                                                               */
/* ======================================================================= */

namespace {

uint32_t grid_for(uint64_t n, uint32_t block)
{
    const uint64_t g = (n + block - 1) / block;
    return (uint32_t)(g > 0x7FFFFFFFull ? 0x7FFFFFFFull : (g ? g : 1));
}

uint32_t grid_stride(uint64_t n) { uint64_t g = (n + 255) / 256; return (uint32_t)(g > 65536 ? 65536 : (g ? g : 1)); }

int fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s)
{
    if (!n) return HBHEAP_OK;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_stride(n)), dim3(256), 0, s, p, n, v);
    return hipGetLastError() == hipSuccess ? HBHEAP_OK : HBHEAP_E_HIP;
}

int va_rebuild(const hbheap_dev_t& d, const uint32_t* totals, const uint32_t* owned, hipStream_t s)
{
    const uint64_t n = (uint64_t)d.n_shards * d.n_classes << d.log2_dir;
    hipLaunchKernelGGL(k_va_rebuild, dim3(grid_stride(n)), dim3(256), 0, s, d, totals, owned);
    return hipGetLastError() == hipSuccess ? HBHEAP_OK : HBHEAP_E_HIP;
}

int fill_u8(uint8_t* p, uint64_t n, uint8_t v, hipStream_t s)
{
    if (!n) return HBHEAP_OK;
    hipLaunchKernelGGL(k_fill_u8, dim3(grid_stride(n)), dim3(256), 0, s, p, n, v);
    return hipGetLastError() == hipSuccess ? HBHEAP_OK : HBHEAP_E_HIP;
}

/* Shards: span = smallest power of two >= ceil(N / requested); as many
 * shards as spans needed to cover N.  Auto (0): about N/256 chunks per
 * shard, between 1 and 64 shards. */
void shard_geometry(uint64_t N, uint32_t requested, uint32_t* S, uint32_t* log2_span)
{
    uint32_t want = requested;
    if (!want) {
        want = 1;
        while (want < kMaxShards && (uint64_t)want * 2 * 256 <= N) want *= 2;
    }
    if (want > N) want = (uint32_t)N;
    const uint64_t per = (N + want - 1) / want;
    *log2_span = ceil_log2(per);
    *S = (uint32_t)((N + (1ull << *log2_span) - 1) >> *log2_span);
}

Layout make_layout(uint64_t N, uint32_t log2C, uint32_t K, uint32_t variant, uint64_t bytes, uint32_t S,
                   uint32_t log2_span, bool eager_retire)
{
    Layout L;
    const uint64_t W = (1ull << log2C) / 1024;
    if (HBHEAP_VARIANT_LISTS_CHUNKS(variant)) {
        /* eager retirement: room for stale entries besides the listed chunks */
        L.log2q = log2_span + (eager_retire ? 1u : 0u);
    } else {
        const uint64_t per = bytes / 8 / K / 4 / S;
        L.log2q = per ? ilog2(per) : 0;
    }
    L.n_slots = ((uint64_t)S * K) << L.log2q;
    /* virtualised array: a shard's queues share M segments of 2^log2_seg
     * slots (Q/8, kept within 16 .. 1024).  Page queues: the page variant's
     * slot budget cut into segments; a queue spans at most the pages its
     * class owns plus partial segments at both ends and one on its way
     * back, so the classes may own (M - 3K) segments' worth of pages.  Chunk
     * queues: a chunk is listed in at most one queue, so the queues of a
     * shard hold at most span entries together: M = ceil(span / 2^g) + 3K
     * segments always suffice, and one queue spans at most
     * ceil(span / 2^g) + 2 of them. */
    uint32_t lg = L.log2q >= 3 ? L.log2q - 3 : 0;
    lg = lg < 4 ? 4 : (lg > 10 ? 10 : lg);
    if (HBHEAP_VARIANT_SHARED_PAGES(variant)) {
        L.log2_seg = lg;
        L.vsegs = (uint32_t)(((uint64_t)K << L.log2q) >> lg);
        L.log2_dir = ceil_log2((uint64_t)L.vsegs + 3);
        L.log2_store = ceil_log2(L.vsegs);
        L.vbudget = L.vsegs > 3 * K ? (uint64_t)(L.vsegs - 3 * K) << lg : 0;
    } else if (HBHEAP_VARIANT_SEGMENTED(variant)) {
        const uint64_t per_queue = ((1ull << log2_span) + (1ull << lg) - 1) >> lg;
        L.log2_seg = lg;
        L.vsegs = (uint32_t)(per_queue + 3ull * K);
        L.log2_dir = ceil_log2(per_queue + 3);
        L.log2_store = ceil_log2(L.vsegs);
        L.vbudget = 0;
    }
    /* virtualised list: no directory (its section holds the segments' tags
     * and links instead) */
    if (HBHEAP_VARIANT_IS_VL(variant)) L.log2_dir = 0;
    if (HBHEAP_VARIANT_SEGMENTED(variant)) L.n_slots = ((uint64_t)S * L.vsegs) << lg;
    L.off_pool = 256;
    L.off_cl = al256(L.off_pool + 128ull * S);
    L.off_cls = al256(L.off_cl + (uint64_t)kClassBlock * S * K);
    L.off_cnt = al256(L.off_cls + N);
    L.off_bits = al256(L.off_cnt + 4 * N);
    L.off_pid = al256(L.off_bits + 8 * N * W);
    L.n_pid = eager_retire ? (uint64_t)S << log2_span : N;
    L.off_sl = al256(L.off_pid + 4 * L.n_pid);
    L.total = al256(L.off_sl + 4ull * L.n_slots);
    if (eager_retire) {
        L.off_ct = L.total;
        L.total = al256(L.off_ct + 8 * N);
    }
    if (HBHEAP_VARIANT_SEGMENTED(variant)) {
        L.off_vdir = L.total;
        const uint64_t dir_words = HBHEAP_VARIANT_IS_VL(variant) ? 2ull * S * L.vsegs : (uint64_t)S * K << L.log2_dir;
        L.off_vtaken = al256(L.off_vdir + 8ull * dir_words);
        L.off_vstore = al256(L.off_vtaken + 4ull * S * L.vsegs);
        L.off_vslots = al256(L.off_vstore + (uint64_t)kStoreBlock * S);
        L.total = al256(L.off_vslots + 4ull * S * (1ull << L.log2_store));
    }
    return L;
}

void put32(uint8_t* b, uint64_t o, uint32_t v) { memcpy(b + o, &v, 4); }
void put64(uint8_t* b, uint64_t o, uint64_t v) { memcpy(b + o, &v, 8); }

void release(hbheap_heap* h)
{
    if (h->data) (void)hipFree(h->data);
    if (h->state) (void)hipFree(h->state);
    if (h->aux) (void)hipFree(h->aux);
    delete h;
}

}  // namespace

namespace {
/* Batch launches: requests per lane R, one 256-lane block per 4 * 64 * R
 * requests.  R = the heap's rows for every variant but the virtualised-list
 * page variant, whose takers walk its links row by row (more rows per wave
 * measured slower there); the heap's rows are 1 for widths below 16. */
static_assert(kBatchBlock / 64 <= hbheap::detail::kRowsBlockWaves, "LDS staging of the rows kernels");
template <uint32_t V>
constexpr bool rows_apply() { return V != HBHEAP_VARIANT_VL_PAGE; }
template <bool C, uint32_t V, uint32_t R>
void launch_alloc(const hbheap_heap* h, const size_t* sizes, void** ptrs, size_t n, hipStream_t stream)
{
    hipLaunchKernelGGL((k_alloc_batch<C, V, R>), dim3(grid_for((n + R - 1) / R, kBatchBlock)), dim3(kBatchBlock), 0,
                       stream, h->dev, (const uint64_t*)sizes, ptrs, (uint64_t)n);
}
template <bool C, uint32_t V>
void launch_alloc_r(const hbheap_heap* h, const size_t* sizes, void** ptrs, size_t n, hipStream_t stream)
{
    if constexpr (rows_apply<V>()) {
        if (h->rows == 4) return launch_alloc<C, V, 4>(h, sizes, ptrs, n, stream);
    }
    launch_alloc<C, V, 1>(h, sizes, ptrs, n, stream);
}
template <bool C>
void launch_alloc_v(const hbheap_heap* h, const size_t* sizes, void** ptrs, size_t n, hipStream_t stream)
{
    switch (h->dev.variant) {
    case HBHEAP_VARIANT_CHUNK:
        if (h->dev.flags & HBHEAP_FLAG_EAGER) launch_alloc_r<C, kChunkEager>(h, sizes, ptrs, n, stream);
        else launch_alloc_r<C, HBHEAP_VARIANT_CHUNK>(h, sizes, ptrs, n, stream);
        break;
    case HBHEAP_VARIANT_PAGE: launch_alloc_r<C, HBHEAP_VARIANT_PAGE>(h, sizes, ptrs, n, stream); break;
    case HBHEAP_VARIANT_VA_PAGE: launch_alloc_r<C, HBHEAP_VARIANT_VA_PAGE>(h, sizes, ptrs, n, stream); break;
    case HBHEAP_VARIANT_VA_CHUNK: launch_alloc_r<C, HBHEAP_VARIANT_VA_CHUNK>(h, sizes, ptrs, n, stream); break;
    case HBHEAP_VARIANT_VL_PAGE: launch_alloc_r<C, HBHEAP_VARIANT_VL_PAGE>(h, sizes, ptrs, n, stream); break;
    default: launch_alloc_r<C, HBHEAP_VARIANT_VL_CHUNK>(h, sizes, ptrs, n, stream); break;
    }
}
template <bool C, uint32_t V, uint32_t R>
void launch_free(const hbheap_heap* h, const size_t* sizes, void* const* ptrs, size_t n, int32_t* status,
                 hipStream_t stream)
{
    hipLaunchKernelGGL((k_free_batch<C, V, R>), dim3(grid_for((n + R - 1) / R, kBatchBlock)), dim3(kBatchBlock), 0,
                       stream, h->dev, (const uint64_t*)sizes, ptrs, (uint64_t)n, status);
}
template <bool C, uint32_t V>
void launch_free_r(const hbheap_heap* h, const size_t* sizes, void* const* ptrs, size_t n, int32_t* status,
                   hipStream_t stream)
{
    if constexpr (rows_apply<V>()) {
        if (h->rows == 4) return launch_free<C, V, 4>(h, sizes, ptrs, n, status, stream);
    }
    launch_free<C, V, 1>(h, sizes, ptrs, n, status, stream);
}
template <bool C>
void launch_free_v(const hbheap_heap* h, const size_t* sizes, void* const* ptrs, size_t n, int32_t* status,
                   hipStream_t stream)
{
    switch (h->dev.variant) {
    case HBHEAP_VARIANT_CHUNK:
        if (h->dev.flags & HBHEAP_FLAG_EAGER) launch_free_r<C, kChunkEager>(h, sizes, ptrs, n, status, stream);
        else launch_free_r<C, HBHEAP_VARIANT_CHUNK>(h, sizes, ptrs, n, status, stream);
        break;
    case HBHEAP_VARIANT_PAGE: launch_free_r<C, HBHEAP_VARIANT_PAGE>(h, sizes, ptrs, n, status, stream); break;
    case HBHEAP_VARIANT_VA_PAGE: launch_free_r<C, HBHEAP_VARIANT_VA_PAGE>(h, sizes, ptrs, n, status, stream); break;
    case HBHEAP_VARIANT_VA_CHUNK: launch_free_r<C, HBHEAP_VARIANT_VA_CHUNK>(h, sizes, ptrs, n, status, stream); break;
    case HBHEAP_VARIANT_VL_PAGE: launch_free_r<C, HBHEAP_VARIANT_VL_PAGE>(h, sizes, ptrs, n, status, stream); break;
    default: launch_free_r<C, HBHEAP_VARIANT_VL_CHUNK>(h, sizes, ptrs, n, status, stream); break;
    }
}
}  // namespace

#if HBHEAP_FUZZ
/* Sets the schedule-fuzzing parameters every fuzz point reads. */
__global__ void k_fuzz_set(uint32_t seed, uint32_t most)
{
    if (threadIdx.x == 0) {
        hbheap::detail::hbheap_fuzz_cfg[0] = seed;
        hbheap::detail::hbheap_fuzz_cfg[1] = most;
    }
}
#endif

extern "C" {

const char* hbheap_version(void) { return "hbheap 0.1 (gfx950)"; }

int heap_create_ex(size_t bytes, size_t chunk_bytes, const heap_config_t* cfg, heap_t* out)
{
    if (!out) return HBHEAP_E_INVAL;
    if (chunk_bytes < 4096 || chunk_bytes > 65536 || (chunk_bytes & (chunk_bytes - 1))) return HBHEAP_E_INVAL;
    if (bytes < chunk_bytes) return HBHEAP_E_INVAL;
    heap_config_t c = {};
    if (cfg) c = *cfg;
    if (c.variant > HBHEAP_VARIANT_VL_CHUNK) return HBHEAP_E_INVAL;
    if (!c.width) c.width = 64;
    if (c.width > 64 || (c.width & (c.width - 1))) return HBHEAP_E_INVAL;
    if (!c.spin_cap) c.spin_cap = 1u << 18;
    if (!c.backoff_max) c.backoff_max = 64;
    if (c.rows != 0 && c.rows != 1 && c.rows != 4) return HBHEAP_E_INVAL;
    const uint64_t N = bytes / chunk_bytes;
    if (N >= 0x80000000ull) return HBHEAP_E_INVAL;
    const uint32_t log2C = ilog2(chunk_bytes);
    const uint32_t K = log2C - 3;
    if (!HBHEAP_VARIANT_LISTS_CHUNKS(c.variant) && N * chunk_bytes > (64ull << 30)) return HBHEAP_E_INVAL;
    if (c.shards > kMaxShards || (c.shards & (c.shards - 1))) return HBHEAP_E_INVAL;
    uint32_t S = 1, log2_span = 0;
    shard_geometry(N, c.shards, &S, &log2_span);
    /* eager retirement: chunk variant only; queue positions must stay
     * distinct modulo 2^28 within a queue's capacity */
    const bool eager_retire = (c.flags & HBHEAP_FLAG_EAGER) != 0;
    if (eager_retire && (c.variant != HBHEAP_VARIANT_CHUNK || log2_span + 1 > 28)) return HBHEAP_E_INVAL;

    hbheap_heap* h = new (std::nothrow) hbheap_heap();
    if (!h) return HBHEAP_E_NOMEM;
    h->chunk_bytes = chunk_bytes;
    /* several requests per lane need every lane of a wave and at most 4
     * segments of lanes (so at most 52 groups of a wave) */
    h->rows = c.rows ? c.rows : 4u;
    if (c.width < 16) h->rows = 1;
    h->lay = make_layout(N, log2C, K, c.variant, bytes, S, log2_span, eager_retire);
    const Layout& L = h->lay;
    h->trim_blocks = (uint32_t)((N + kTrimBlock - 1) / kTrimBlock);
    const uint32_t nkeys = S * (K + 1) + 1;
    /* aux: err (256 B) | stats (256 B) | per-shard stats (128 B each) |
     * trim counts | offsets | totals | owned */
    const uint64_t tb = al256((uint64_t)h->trim_blocks * nkeys * 4);
    const uint64_t kb = al256((uint64_t)nkeys * 4);
    h->shard_stat_bytes = al256(8ull * kShardStatStride * S);
    h->aux_bytes = 512 + h->shard_stat_bytes + 2 * tb + 2 * kb;
    if (hipMalloc(&h->data, N * chunk_bytes) != hipSuccess) { h->data = nullptr; release(h); return HBHEAP_E_NOMEM; }
    if (hipMalloc(&h->state, L.total) != hipSuccess) { h->state = nullptr; release(h); return HBHEAP_E_NOMEM; }
    if (hipMalloc(&h->aux, h->aux_bytes) != hipSuccess) { h->aux = nullptr; release(h); return HBHEAP_E_NOMEM; }

    uint8_t* st = (uint8_t*)h->state;
    uint8_t* ax = (uint8_t*)h->aux;
    hbheap_dev_t& d = h->dev;
    d.data = (uint8_t*)h->data;
    d.state = st;
    d.pool = (uint64_t*)(st + L.off_pool);
    d.classes = st + L.off_cl;
    d.chunk_class = st + L.off_cls;
    d.chunk_cnt = (int32_t*)(st + L.off_cnt);
    d.bits = (uint64_t*)(st + L.off_bits);
    d.pool_ids = (uint32_t*)(st + L.off_pid);
    d.slots = (uint32_t*)(st + L.off_sl);
    d.chunk_ct = eager_retire ? (uint64_t*)(st + L.off_ct) : nullptr;
    d.err = (uint32_t*)ax;
    d.stats = (uint64_t*)(ax + 256);
    d.data_bytes = N * chunk_bytes;
    d.n_chunks = (uint32_t)N;
    d.log2_chunk = log2C;
    d.n_classes = K;
    d.variant = c.variant;
    d.words_per_chunk = (uint32_t)(chunk_bytes / 1024);
    d.log2q = L.log2q;
    d.width = c.width;
    d.spin_cap = c.spin_cap;
    d.backoff_max = c.backoff_max;
    d.flags = c.flags;
    d.n_shards = S;
    d.log2_span = log2_span;
    if (HBHEAP_VARIANT_SEGMENTED(c.variant)) {
        if (HBHEAP_VARIANT_SHARED_PAGES(c.variant) && L.vbudget == 0) { release(h); return HBHEAP_E_INVAL; }
        d.vdir = (uint64_t*)(st + L.off_vdir);
        d.vtaken = (uint32_t*)(st + L.off_vtaken);
        d.vstore = st + L.off_vstore;
        d.vstore_slots = (uint32_t*)(st + L.off_vslots);
        d.log2_seg = L.log2_seg;
        d.log2_dir = L.log2_dir;
        d.log2_store = L.log2_store;
        d.vsegs = L.vsegs;
        d.vbudget = L.vbudget;
    }
    uint8_t* tw = ax + 512 + h->shard_stat_bytes; /* trim workspace */
    h->trim_counts = (uint32_t*)tw;
    h->trim_offsets = (uint32_t*)(tw + tb);
    h->trim_totals = (uint32_t*)(tw + 2 * tb);
    h->trim_owned = (uint32_t*)(tw + 2 * tb + kb);
    h->owned_words = S * K;

    /* header, pool blocks and class blocks are built on the host */
    const uint64_t head_bytes = L.off_cls;
    uint8_t* hb = (uint8_t*)calloc(1, head_bytes);
    if (!hb) { release(h); return HBHEAP_E_NOMEM; }
    put32(hb, 0, kMagic);
    put32(hb, 4, kVersion);
    put64(hb, 8, d.data_bytes);
    put32(hb, 16, (uint32_t)N);
    put32(hb, 20, log2C);
    put32(hb, 24, K);
    put32(hb, 28, c.variant);
    put32(hb, 32, d.words_per_chunk);
    put32(hb, 36, L.log2q);
    put32(hb, 40, S);
    put32(hb, 44, log2_span);
    put64(hb, 48, L.off_pool);
    put64(hb, 56, L.off_cl);
    put64(hb, 64, L.off_cls);
    put64(hb, 72, L.off_cnt);
    put64(hb, 80, L.off_bits);
    put64(hb, 88, L.off_pid);
    put64(hb, 96, L.off_sl);
    put64(hb, 104, L.total);
    put32(hb, 112, L.log2_seg);
    put32(hb, 116, L.log2_dir);
    put32(hb, 120, L.log2_store);
    put32(hb, 124, L.vsegs);
    put64(hb, 128, L.vbudget);
    put64(hb, 136, L.off_vdir);
    put64(hb, 144, L.off_vtaken);
    put64(hb, 152, L.off_vstore);
    put64(hb, 160, L.off_vslots);
    put32(hb, 168, eager_retire ? 1u : 0u);
    put64(hb, 176, L.off_ct);
    for (uint32_t j = 0; j < S; ++j) {
        const uint64_t first = (uint64_t)j << log2_span;
        const uint64_t size = first + (1ull << log2_span) <= N ? (1ull << log2_span) : N - first;
        /* bump pool: u64 bump; eager retirement: u64 ring state (its
         * chunks published), u32 head at +16 and tail at +20 */
        put64(hb, L.off_pool + 128ull * j, eager_retire ? size + kBias : 0);
        put32(hb, L.off_pool + 128ull * j + 8, (uint32_t)size);
        put32(hb, L.off_pool + 128ull * j + 12, (uint32_t)first);
        if (eager_retire) put32(hb, L.off_pool + 128ull * j + 20, (uint32_t)size);
    }
    for (uint64_t i = 0; i < (uint64_t)S * K; ++i) put64(hb, L.off_cl + i * kClassBlock, kBias);

    int rc = HBHEAP_OK;
    hipStream_t s = nullptr;
    if (fill_u32((uint32_t*)st, L.total / 4, 0u, s) || fill_u8(st + L.off_cls, N, (uint8_t)kFreeClass, s) ||
        fill_u32(d.slots, L.n_slots, kEmpty, s) || fill_u32((uint32_t*)ax, h->aux_bytes / 4, 0u, s))
        rc = HBHEAP_E_HIP;
    if (rc == HBHEAP_OK) {
        hipLaunchKernelGGL(k_iota_u32, dim3(grid_stride(N)), dim3(256), 0, s, d.pool_ids, N);
        if (hipGetLastError() != hipSuccess) rc = HBHEAP_E_HIP;
    }
    if (rc == HBHEAP_OK && eager_retire) {
        /* the last shard's ring slots past its chunks, and every chunk's
         * count/token word: empty, no token */
        rc = fill_u32(d.pool_ids + N, L.n_pid - N, kEmpty, s);
        if (rc == HBHEAP_OK) {
            hipLaunchKernelGGL(k_fill_u64, dim3(grid_stride(N)), dim3(256), 0, s, d.chunk_ct, N,
                               ct_word(kTokNone, 0));
            if (hipGetLastError() != hipSuccess) rc = HBHEAP_E_HIP;
        }
    }
    if (rc == HBHEAP_OK && hipMemcpyAsync(st, hb, head_bytes, hipMemcpyHostToDevice, s) != hipSuccess) rc = HBHEAP_E_HIP;
    if (rc == HBHEAP_OK && HBHEAP_VARIANT_SEGMENTED(c.variant)) rc = va_rebuild(d, nullptr, nullptr, s);
    if (rc == HBHEAP_OK && hipStreamSynchronize(s) != hipSuccess) rc = HBHEAP_E_HIP;
    free(hb);
    if (rc != HBHEAP_OK) { release(h); return rc; }
    *out = h;
    return HBHEAP_OK;
}

int heap_create(size_t bytes, size_t chunk_bytes, heap_t* out) { return heap_create_ex(bytes, chunk_bytes, nullptr, out); }

int heap_destroy(heap_t h)
{
    if (!h) return HBHEAP_OK;
    int rc = HBHEAP_OK;
    if (h->data && hipFree(h->data) != hipSuccess) rc = HBHEAP_E_HIP;
    if (h->state && hipFree(h->state) != hipSuccess) rc = HBHEAP_E_HIP;
    if (h->aux && hipFree(h->aux) != hipSuccess) rc = HBHEAP_E_HIP;
    delete h;
    return rc;
}

int heap_alloc_batch(heap_t h, const size_t* sizes, void** ptrs, size_t n, hipStream_t stream)
{
    if (!h || (n && (!sizes || !ptrs))) return HBHEAP_E_INVAL;
    if (!n) return HBHEAP_OK;
    if (h->dev.flags & HBHEAP_FLAG_STATS) launch_alloc_v<true>(h, sizes, ptrs, n, stream);
    else launch_alloc_v<false>(h, sizes, ptrs, n, stream);
    return hipGetLastError() == hipSuccess ? HBHEAP_OK : HBHEAP_E_HIP;
}

int heap_free_batch_ex(heap_t h, const size_t* sizes, void* const* ptrs, size_t n, int32_t* status, hipStream_t stream)
{
    if (!h || (n && !ptrs)) return HBHEAP_E_INVAL;
    if (!n) return HBHEAP_OK;
    if (h->dev.flags & HBHEAP_FLAG_STATS) launch_free_v<true>(h, sizes, ptrs, n, status, stream);
    else launch_free_v<false>(h, sizes, ptrs, n, status, stream);
    return hipGetLastError() == hipSuccess ? HBHEAP_OK : HBHEAP_E_HIP;
}

int heap_free_batch(heap_t h, const size_t* sizes, void* const* ptrs, size_t n, hipStream_t stream)
{
    return heap_free_batch_ex(h, sizes, ptrs, n, nullptr, stream);
}

int heap_set_flags(heap_t h, uint32_t flags)
{
    if (!h) return HBHEAP_E_INVAL;
    /* eager retirement is fixed at creation */
    h->dev.flags = (flags & ~HBHEAP_FLAG_EAGER) | (h->dev.flags & HBHEAP_FLAG_EAGER);
    return HBHEAP_OK;
}

int heap_device_handle(heap_t h, hbheap_dev_t* out)
{
    if (!h || !out) return HBHEAP_E_INVAL;
    *out = h->dev;
    return HBHEAP_OK;
}

int heap_info(heap_t h, heap_info_t* out)
{
    if (!h || !out) return HBHEAP_E_INVAL;
    out->data = h->data;
    out->data_bytes = h->dev.data_bytes;
    out->chunk_bytes = h->chunk_bytes;
    out->n_chunks = h->dev.n_chunks;
    out->n_classes = h->dev.n_classes;
    out->variant = h->dev.variant;
    out->ring_entries = HBHEAP_VARIANT_SHARED_PAGES(h->dev.variant) ? h->lay.vbudget : 1ull << h->lay.log2q;
    out->n_shards = h->dev.n_shards;
    out->state_bytes = h->lay.total;
    out->metadata_bytes = h->lay.total + h->aux_bytes;
    return HBHEAP_OK;
}

int heap_trim(heap_t h, hipStream_t stream)
{
    if (!h) return HBHEAP_E_INVAL;
    const hbheap_dev_t& d = h->dev;
    const uint32_t nkeys = d.n_shards * (d.n_classes + 1) + 1;
    const uint32_t nb = h->trim_blocks;
    int rc = fill_u32(h->trim_owned, h->owned_words, 0u, stream);
    if (rc) return rc;
    hipLaunchKernelGGL(k_trim_count, dim3(nb), dim3(kTrimBlock), 0, stream, d, h->trim_counts, nb, h->trim_owned);
    HB_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_trim_scan, dim3(1), dim3(1024), 0, stream, h->trim_counts, h->trim_offsets, h->trim_totals, nb,
                       nkeys);
    HB_TRY(hipGetLastError());
    rc = fill_u32(d.slots, h->lay.n_slots, kEmpty, stream);
    if (!rc) rc = fill_u32(d.pool_ids, h->lay.n_pid, kEmpty, stream);
    if (rc) return rc;
    hipLaunchKernelGGL(k_trim_write, dim3(nb), dim3(kTrimBlock), 0, stream, d, h->trim_offsets, nb, h->trim_totals);
    HB_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_trim_ctl, dim3(1), dim3(1024), 0, stream, d, h->trim_totals, h->trim_owned);
    HB_TRY(hipGetLastError());
    if (HBHEAP_VARIANT_SEGMENTED(d.variant)) return va_rebuild(d, h->trim_totals, h->trim_owned, stream);
    return HBHEAP_OK;
}

int heap_snapshot(heap_t h, void* dst, size_t cap, size_t* len, hipStream_t stream)
{
    if (!h) return HBHEAP_E_INVAL;
    if (len) *len = h->lay.total;
    if (!dst) return len ? HBHEAP_OK : HBHEAP_E_INVAL;
    if (cap < h->lay.total) return HBHEAP_E_RANGE;
    HB_TRY(hipStreamSynchronize(stream));
    HB_TRY(hipMemcpy(dst, h->state, h->lay.total, hipMemcpyDeviceToHost));
    return HBHEAP_OK;
}

int heap_get_error(heap_t h, uint32_t* err)
{
    if (!h || !err) return HBHEAP_E_INVAL;
    HB_TRY(hipDeviceSynchronize());
    HB_TRY(hipMemcpy(err, h->dev.err, 4, hipMemcpyDeviceToHost));
    return HBHEAP_OK;
}

int heap_clear_error(heap_t h)
{
    if (!h) return HBHEAP_E_INVAL;
    HB_TRY(hipDeviceSynchronize());
    const uint32_t z = 0;
    HB_TRY(hipMemcpy(h->dev.err, &z, 4, hipMemcpyHostToDevice));
    return HBHEAP_OK;
}

static_assert(sizeof(heap_stats_t) == HBHEAP_STAT_COUNT * sizeof(uint64_t), "one field per counter");
static_assert(offsetof(heap_stats_t, slot_ops) == HBHEAP_STAT_SLOT_OPS * sizeof(uint64_t), "field order");
static_assert(offsetof(heap_stats_t, oom) == HBHEAP_STAT_OOM * sizeof(uint64_t), "field order");

int heap_stats(heap_t h, heap_stats_t* out)
{
    if (!h || !out) return HBHEAP_E_INVAL;
    HB_TRY(hipDeviceSynchronize());
    uint64_t all[HBHEAP_STAT_COUNT];
    HB_TRY(hipMemcpy(all, h->dev.stats, sizeof(all), hipMemcpyDeviceToHost));
    std::vector<uint64_t> per((uint64_t)kShardStatStride * h->dev.n_shards);
    HB_TRY(hipMemcpy(per.data(), h->dev.stats + kShardStatBase, per.size() * 8, hipMemcpyDeviceToHost));
    for (uint32_t j = 0; j < h->dev.n_shards; ++j) {
        all[HBHEAP_STAT_OOM] += per[(uint64_t)kShardStatStride * j];
        all[HBHEAP_STAT_OOM_WAITS] += per[(uint64_t)kShardStatStride * j + 1];
    }
    memcpy(out, all, sizeof(all));
    return HBHEAP_OK;
}

int heap_replay(heap_t h, const int64_t* ops, int64_t* out, size_t n, hipStream_t stream)
{
    if (!h || (n && (!ops || !out))) return HBHEAP_E_INVAL;
    if (!n) return HBHEAP_OK;
    hipLaunchKernelGGL(k_replay, dim3(1), dim3(64), 0, stream, h->dev, ops, out, (uint64_t)n);
    return hipGetLastError() == hipSuccess ? HBHEAP_OK : HBHEAP_E_HIP;
}

int heap_pattern_write(heap_t h, void* const* ptrs, const size_t* sizes, size_t n, uint32_t seed, hipStream_t stream)
{
    if (!h || (n && (!ptrs || !sizes))) return HBHEAP_E_INVAL;
    if (!n) return HBHEAP_OK;
    hipLaunchKernelGGL(k_pattern, dim3(grid_for(n, kBatchBlock)), dim3(kBatchBlock), 0, stream, ptrs,
                       (const uint64_t*)sizes, (uint64_t)n, seed, (unsigned long long*)nullptr, 0,
                       (const uint8_t*)h->data, h->dev.data_bytes);
    return hipGetLastError() == hipSuccess ? HBHEAP_OK : HBHEAP_E_HIP;
}

int heap_pattern_check(heap_t h, void* const* ptrs, const size_t* sizes, size_t n, uint32_t seed,
                       unsigned long long* mismatches, hipStream_t stream)
{
    if (!h || (n && (!ptrs || !sizes || !mismatches))) return HBHEAP_E_INVAL;
    if (!n) return HBHEAP_OK;
    hipLaunchKernelGGL(k_pattern, dim3(grid_for(n, kBatchBlock)), dim3(kBatchBlock), 0, stream, ptrs,
                       (const uint64_t*)sizes, (uint64_t)n, seed, mismatches, 1, (const uint8_t*)h->data,
                       h->dev.data_bytes);
    return hipGetLastError() == hipSuccess ? HBHEAP_OK : HBHEAP_E_HIP;
}

int hb_plain_pattern(void* const* ptrs, const size_t* sizes, size_t n, uint32_t seed, unsigned long long* mismatches,
                     hipStream_t stream)
{
    if (n && (!ptrs || !sizes)) return HBHEAP_E_INVAL;
    if (!n) return HBHEAP_OK;
    /* blocks of the runtime's allocator may lie anywhere: no region check */
    hipLaunchKernelGGL(k_pattern, dim3(grid_for(n, kBatchBlock)), dim3(kBatchBlock), 0, stream, ptrs,
                       (const uint64_t*)sizes, (uint64_t)n, seed, mismatches, mismatches ? 1 : 0,
                       (const uint8_t*)nullptr, ~0ull);
    return hipGetLastError() == hipSuccess ? HBHEAP_OK : HBHEAP_E_HIP;
}

int hb_atomic_probe(int pattern, void* buf, size_t buf_bytes, size_t threads, uint32_t lines, uint32_t iters,
                    hipStream_t stream)
{
    if (!buf || buf_bytes < 4096 || pattern < 0 || pattern > 8 || !threads || !iters) return HBHEAP_E_INVAL;
    if (pattern == 1 && (!lines || (uint64_t)lines * 128 > buf_bytes)) return HBHEAP_E_INVAL;
    hipLaunchKernelGGL(k_atomic_probe, dim3(grid_for(threads, kBatchBlock)), dim3(kBatchBlock), 0, stream, pattern,
                       (uint64_t*)buf, (uint64_t)(buf_bytes / 8), lines, iters, (uint64_t)threads);
    return hipGetLastError() == hipSuccess ? HBHEAP_OK : HBHEAP_E_HIP;
}

int hb_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t stream)
{
    if (!dst || !src || (bytes & 15)) return HBHEAP_E_INVAL;
    const uint64_t n = bytes / 16;
    if (!n) return HBHEAP_OK;
    const uint32_t blocks = 256 * 8;
    hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, stream, (uint4*)dst, (const uint4*)src, n);
    return hipGetLastError() == hipSuccess ? HBHEAP_OK : HBHEAP_E_HIP;
}

int hb_fuzz_set(uint32_t seed, uint32_t most_sleeps)
{
#if HBHEAP_FUZZ
    /* a test-build entry point: a failure names the HIP error on stderr */
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_fuzz_set, dim3(1), dim3(64), 0, 0, seed, most_sleeps);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        fprintf(stderr, "hb_fuzz_set: %s (%d)\n", hipGetErrorString(e), (int)e);
        return HBHEAP_E_HIP;
    }
    return HBHEAP_OK;
#else
    (void)seed;
    (void)most_sleeps;
    return HBHEAP_E_UNSUP;
#endif
}

}  // extern "C"
