/*
 * hbheap_device.h -- device-side allocation for HIP kernels on gfx950.
 *
 *   __device__ void* dev_malloc(hbheap_dev_t h, size_t n);
 *   __device__ void  dev_free(hbheap_dev_t h, void* p);
 *
 * Any kernel, any launch shape, any subset of active lanes may call them
 * (the paper's port had to flatten thread indices and work around the lack
 * of an active-lane mask, Porting section; on CDNA the EXEC mask is the
 * active mask).  `h` comes from heap_device_handle() and is passed by value.
 *
 * The method (Introduction; Results): one preallocated heap, cut into chunks
 * of a fixed size C; a chunk given to a size class is split into pages of
 * that class; each class has a lock-free queue, listing either chunks that
 * still hold free pages (chunk variant: take a chunk, then scan it for free
 * pages) or the free pages themselves (page variant).  Warp-vote aggregation
 * lets several allocations of one warp share one queue operation (Porting
 * section); here a wave64 groups its lanes by class and the group's leader
 * performs one queue operation for the whole group.
 *
 * Design for CDNA4 (not in the paper):
 *   - Class of n: max(0, ceil(log2 n) - 4) with 16 B pages; 0 or n > C is NULL.
 *   - Each class queue is a ring of u32 slots with monotone head/tail and a
 *     64-bit state word (H << 32 | count + 2^31), each on its own 128-byte
 *     line.  H counts operations in flight that may still publish entries;
 *     a shard counts as empty for a class only once its pool is exhausted
 *     and its state shows H == 0 and count <= 0 (exact out-of-memory).
 *   - Slots are taken with an atomic exchange against EMPTY and filled with
 *     compare-and-swap from EMPTY, so a slot whose producer is late is waited
 *     for instead of being read twice.
 *   - Per chunk: class byte, count of free pages (chunk variant) and a bitmask
 *     with 1 = free.  In the chunk variant only the holder of a chunk's queue
 *     entry lowers its count, so the count it read cannot go below what it
 *     takes; frees set the bit, raise the count, and a 0 -> 1 count enqueues
 *     the chunk (it is in the queue exactly while its count is positive).
 *   - Unowned chunks sit in a pool array consumed by a 64-bit bump counter,
 *     so "pool empty" is exact and never undone during a kernel; chunks come
 *     back to the pool only through heap_trim() at quiescence.  With eager
 *     retirement (HBHEAP_FLAG_EAGER, chunk variant) the pool is a ring per
 *     shard instead, and a free that makes a chunk whole puts it back at
 *     once; only frees can do that, so "pool empty" still holds for the rest
 *     of a launch that frees nothing.
 *   - The heap is split into shards, each owning a run of consecutive chunks
 *     with its own pool and its own class queues; a wave starts at its home
 *     shard (spread by wave index); when it runs dry the wave looks at every
 *     shard at once (one lane per shard) and steals from one that has
 *     something, so the queue words of one class are hit by 1/S of the
 *     waves.  A request returns NULL only when one such look finds every
 *     shard with no entry, no hold in flight and no chunk left for the
 *     class.
 *   - Every wait is bounded: past spin_cap iterations the wait gives up,
 *     sets HBHEAP_ERR_TIMEOUT and the request returns NULL.
 *   - Metadata atomics are agent-scope and relaxed.  Every metadata word
 *     that other waves read while a kernel runs is written by an atomic
 *     read-modify-write (performed where the device performs atomics, the
 *     same place for every XCD) and read by one, or by an agent-scope load;
 *     ordering comes from issuing a dependent access only after the value
 *     it depends on has returned (a refill waits for the exchanges that set
 *     its bits before it publishes pages), never from cache-wide fences.
 *
 * dev_free() starts with an agent-scope release fence so the caller's
 * writes to the block complete before the block can be handed out again.
 */
#ifndef HBHEAP_DEVICE_H
#define HBHEAP_DEVICE_H

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hbheap_types.h"

namespace hbheap {
namespace detail {

constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr uint64_t kHold = 1ull << 32;
constexpr uint32_t kBias = 0x80000000u;
constexpr uint64_t kNoPage = ~0ull;
constexpr uint32_t kFreeClass = 0xFFu;
constexpr uint32_t kClassBlock = 512;    /* state, head, tail, owned: one 128 B line each */
constexpr uint32_t kMaxWavesPerBlock = 16;

enum : uint32_t { kFreeOk = 0, kFreeDouble = 1, kFreeInvalid = 2, kFreeNull = 3 };

/* ---------------- wave primitives ---------------- */

__device__ __forceinline__ uint32_t lane() { return __lane_id(); }
__device__ __forceinline__ uint64_t exec_mask() { return __builtin_amdgcn_read_exec(); }
__device__ __forceinline__ uint32_t rank_in(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
__device__ __forceinline__ uint32_t bcast(uint32_t v, uint32_t l)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)l);
}
__device__ __forceinline__ uint64_t bcast64(uint64_t v, uint32_t l)
{
    return ((uint64_t)bcast((uint32_t)(v >> 32), l) << 32) | bcast((uint32_t)v, l);
}
__device__ __forceinline__ uint32_t ctz64(uint64_t m) { return (uint32_t)__builtin_ctzll(m); }
/* The lane of rank r among the set lanes of m (r < popcount(m)). */
__device__ __forceinline__ uint32_t lane_of_rank(uint64_t m, uint32_t r)
{
    for (uint32_t i = 0; i < r; ++i) m &= m - 1ull;
    return ctz64(m);
}

/* Exclusive prefix sum over the active lanes, in lane order, of values below
 * 2^BITS, built from one ballot per bit: inactive lanes count as zero. */
template <int BITS>
__device__ __forceinline__ uint32_t excl_scan(uint32_t x, uint32_t* total)
{
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
        const uint64_t m = __ballot((x >> b) & 1u);
        pre += rank_in(m) << b;
        tot += (uint32_t)__popcll(m) << b;
    }
    *total = tot;
    return pre;
}

/* Value of v held by lane `src` (ds_bpermute; src must be active for the
 * result to be used). */
__device__ __forceinline__ uint32_t perm32(uint32_t v, uint32_t src)
{
    return (uint32_t)__builtin_amdgcn_ds_bpermute((int)(src << 2), (int)v);
}
__device__ __forceinline__ uint64_t perm64(uint64_t v, uint32_t src)
{
    return ((uint64_t)perm32((uint32_t)(v >> 32), src) << 32) | perm32((uint32_t)v, src);
}

/* Runs of adjacent active lanes (inside aligned segments of `seg` lanes)
 * that apply bits to the same bitmask word `key` (`bit`: one set bit per
 * lane).  The run's last lane issues the run's single atomic.  incl: bits of
 * the run's lanes up to this one (the whole run at the tail); prior: bits of
 * the run's lower lanes; tail: the run's last lane.  When every run holds
 * consecutive bits in lane order (pages taken or freed in ring order: the
 * common case), each lane's bits are the range from its run's first bit to
 * its own; otherwise they are OR-ed by a segmented inclusive scan over the
 * lanes (six permute steps, whatever the number of runs). */
struct Run {
    uint64_t incl;
    uint64_t prior;
    uint32_t tail;
};
/* Bits lo..hi (lo <= hi <= 63). */
__device__ __forceinline__ uint64_t bit_range(uint32_t lo, uint32_t hi)
{
    const uint64_t upto = hi == 63u ? ~0ull : ((2ull << hi) - 1ull);
    return upto & ~((1ull << lo) - 1ull);
}
__device__ __forceinline__ Run run_combine(bool have, uint64_t key, uint64_t bit, uint32_t seg)
{
    const uint32_t me = lane();
    const uint32_t prev = me ? me - 1u : 0u;
    const uint64_t todo = __ballot(have);
    const uint32_t b = have ? (uint32_t)__builtin_ctzll(bit | (1ull << 63)) : 0u;
    const uint64_t pkey = perm64(key, prev);
    const uint32_t pb = perm32(b, prev);
    const bool same = have && (me & (seg - 1u)) != 0u && ((todo >> prev) & 1ull) && pkey == key;
    const uint64_t same_m = __ballot(same);
    const uint64_t heads = todo & ~same_m;
    const uint64_t tails = todo & ~(same_m >> 1);
    const uint64_t upto = me == 63u ? ~0ull : ((2ull << me) - 1ull);
    const uint32_t start = have ? 63u - (uint32_t)__builtin_clzll(heads & upto) : me;
    Run r;
    r.tail = have ? ctz64(tails & ~((1ull << me) - 1ull)) : me;
    if (__ballot(same && b != pb + 1u) == 0) {
        /* every run is consecutive bits: lanes start..me hold bits bs..b */
        const uint32_t bs = perm32(b, start);
        r.incl = have ? bit_range(bs, b) : 0ull;
        r.prior = same ? bit_range(bs, b - 1u) : 0ull;
        return r;
    }
    uint64_t acc = have ? bit : 0ull;
#pragma unroll
    for (uint32_t d = 1; d < 64u; d <<= 1) {
        const uint64_t v = perm64(acc, me >= d ? me - d : me);
        if (have && me >= start + d) acc |= v;
    }
    r.incl = acc;
    const uint64_t pa = perm64(acc, prev);
    r.prior = same ? pa : 0ull;
    return r;
}

/* The runs of a full wave whose lanes hold consecutive pages of one class
 * (lane l has page g0 + l, g = offset >> shift, p its page in its chunk,
 * ppc pages per chunk): a run ends at a word's last bit, at its chunk's last
 * page or at lane 63, so each lane knows its run without looking at its
 * neighbours.  Gives what run_combine gives for such a wave (segments of 64
 * lanes); false, r untouched, unless every lane has a page, the class is
 * the same on every lane and the pages are consecutive (wave-uniform). */
__device__ __forceinline__ bool run_consecutive(bool have, uint64_t o, uint32_t shift, uint32_t ppc, uint32_t p, Run& r)
{
    if (exec_mask() != ~0ull || __ballot(!have) != 0ull) return false;
    const uint32_t me = lane();
    const uint32_t s0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)shift);
    const uint64_t g = o >> shift;
    const uint64_t g0 = bcast64(g, 0);
    if (__ballot(shift != s0 || g != g0 + me) != 0ull) return false;
    const uint32_t b = p & 63u;
    const uint32_t before = me < b ? me : b;
    uint32_t after = 63u - b;
    if (63u - me < after) after = 63u - me;
    if (ppc - 1u - p < after) after = ppc - 1u - p;
    r.incl = bit_range(b - before, b);
    r.prior = before ? bit_range(b - before, b - 1u) : 0ull;
    r.tail = me + after;
    return true;
}

/* ---------------- scoped atomics ---------------- */

#define HBH_A(order) order, __HIP_MEMORY_SCOPE_AGENT
__device__ __forceinline__ uint64_t a_add64(uint64_t* p, uint64_t v) { return __hip_atomic_fetch_add(p, v, HBH_A(__ATOMIC_RELAXED)); }
__device__ __forceinline__ uint32_t a_add32(uint32_t* p, uint32_t v) { return __hip_atomic_fetch_add(p, v, HBH_A(__ATOMIC_RELAXED)); }
__device__ __forceinline__ int32_t a_addi(int32_t* p, int32_t v) { return __hip_atomic_fetch_add(p, v, HBH_A(__ATOMIC_RELAXED)); }
__device__ __forceinline__ uint64_t a_or64(uint64_t* p, uint64_t v) { return __hip_atomic_fetch_or(p, v, HBH_A(__ATOMIC_RELAXED)); }
__device__ __forceinline__ uint64_t a_and64(uint64_t* p, uint64_t v) { return __hip_atomic_fetch_and(p, v, HBH_A(__ATOMIC_RELAXED)); }
__device__ __forceinline__ uint32_t a_or32(uint32_t* p, uint32_t v) { return __hip_atomic_fetch_or(p, v, HBH_A(__ATOMIC_RELAXED)); }
__device__ __forceinline__ uint32_t a_and32(uint32_t* p, uint32_t v) { return __hip_atomic_fetch_and(p, v, HBH_A(__ATOMIC_RELAXED)); }
__device__ __forceinline__ uint32_t a_xchg32(uint32_t* p, uint32_t v) { return __hip_atomic_exchange(p, v, HBH_A(__ATOMIC_RELAXED)); }
__device__ __forceinline__ bool a_cas32(uint32_t* p, uint32_t expect, uint32_t v)
{
    return __hip_atomic_compare_exchange_strong(p, &expect, v, __ATOMIC_RELAXED, HBH_A(__ATOMIC_RELAXED));
}
/* Compare-and-swap giving the word's old value (the swap happened iff it
 * equals expect); unlike a_cas32 nothing branches on the outcome where it is
 * issued, so several of them can be in flight at once. */
__device__ __forceinline__ uint32_t a_cas32_old(uint32_t* p, uint32_t expect, uint32_t v)
{
    __hip_atomic_compare_exchange_strong(p, &expect, v, __ATOMIC_RELAXED, HBH_A(__ATOMIC_RELAXED));
    return expect;
}
__device__ __forceinline__ uint64_t a_load64(uint64_t* p) { return __hip_atomic_load(p, HBH_A(__ATOMIC_RELAXED)); }
__device__ __forceinline__ uint32_t a_load32(uint32_t* p) { return __hip_atomic_load(p, HBH_A(__ATOMIC_RELAXED)); }
__device__ __forceinline__ int32_t a_loadi(int32_t* p) { return __hip_atomic_load(p, HBH_A(__ATOMIC_RELAXED)); }
#undef HBH_A

/* Zero, computed from v by an instruction the compiler cannot see through.
 * Added to the address of a later memory operation, it makes that operation
 * wait for v: it is issued only once the earlier load or atomic has returned
 * its value, i.e. has been performed.  Between the accesses above -- atomic
 * read-modify-writes, performed at the device's one point of coherence for
 * the address, and agent-scope loads (global_load sc1), which the compiler
 * maps with no cache invalidation and which must therefore be served
 * coherently with those atomics -- this orders the two as an acquire (after
 * a load) or a release (before a store) would, without the L2 invalidation
 * or write-back those fences also issue. */
__device__ __forceinline__ uint32_t zero_after(uint32_t v)
{
    uint32_t z;
    __asm__ volatile("v_and_b32 %0, 0, %1" : "=v"(z) : "v"(v));
    return z;
}

__device__ __forceinline__ void fence_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
/* Wait until every memory operation this wave issued has completed (loads
 * have returned their data), and keep the compiler from moving memory
 * operations across: enough before freeing a block the wave has only read,
 * with no cache write-back (a release fence also writes back the L2). */
__device__ __forceinline__ void wait_own_accesses() { __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

/* Counters the out-of-memory path bumps (requests answered NULL, waits):
 * kept per home shard, one 128-byte line each after the global counters,
 * so that the waves of a launch that runs out of memory do not all add to
 * one word; heap_stats() sums them into HBHEAP_STAT_OOM and
 * HBHEAP_STAT_OOM_WAITS. */
constexpr uint32_t kShardStatBase = 32; /* u64 index from h.stats */
constexpr uint32_t kShardStatStride = 16;
__device__ __forceinline__ uint64_t* shard_stats(const hbheap_dev_t& h, uint32_t j)
{
    return h.stats + kShardStatBase + (uint64_t)kShardStatStride * j;
}

__device__ __forceinline__ void raise_err(const hbheap_dev_t& h, uint32_t bit, uint32_t stat)
{
    a_or32(h.err, bit);
    a_add64(h.stats + stat, 1);
}

/* Bounded exponential backoff on s_sleep; false once spin_cap is spent. */
struct Backoff {
    uint32_t delay = 1, spins = 0;
    __device__ __forceinline__ bool wait(const hbheap_dev_t& h)
    {
        if (++spins > h.spin_cap) return false;
        for (uint32_t i = 0; i < delay; ++i) __builtin_amdgcn_s_sleep(1);
        if (delay < h.backoff_max) delay <<= 1;
        return true;
    }
};

/* Schedule fuzzing (a build of the library with HBHEAP_FUZZ=1, for tests):
 * at each fuzz point of the protocol -- between the atomic steps of a
 * reservation, a take, a refill, a publication, a free, a scan, a segment
 * hand-off -- the wave sleeps, one point in four, for a pseudo-random
 * number of s_sleep periods drawn from (seed, point, wave, clock), which
 * widens the windows in which other waves act between the steps.  Seed 0
 * turns it off; the normal build compiles every point to nothing. */
#ifndef HBHEAP_FUZZ
#define HBHEAP_FUZZ 0
#endif
#if HBHEAP_FUZZ
/* seed, most sleep periods per point; set by a one-lane kernel of
 * hb_fuzz_set between launches. */
__device__ uint32_t hbheap_fuzz_cfg[2];
/* Chris Wellons' "lowbias32" integer hash (public domain). */
__device__ __forceinline__ uint32_t fuzz_mix(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}
#endif
__device__ __forceinline__ void fuzz_point(uint32_t site)
{
#if HBHEAP_FUZZ
    const uint32_t seed = __builtin_amdgcn_readfirstlane(*(volatile uint32_t*)&hbheap_fuzz_cfg[0]);
    if (!seed) return;
    const uint32_t most = __builtin_amdgcn_readfirstlane(*(volatile uint32_t*)&hbheap_fuzz_cfg[1]);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
    const uint32_t t = __builtin_amdgcn_readfirstlane((uint32_t)clock64());
    const uint32_t x = fuzz_mix(seed ^ fuzz_mix(site * 0x9E3779B9u ^ wave) ^ (t >> 6));
    if (x & 3u) return;
    const uint32_t n = most ? (x >> 2) % most : 0u;
    for (uint32_t i = 0; i < n; ++i) __builtin_amdgcn_s_sleep(4);
#else
    (void)site;
#endif
}

/* Atomics issued, by target, when HBHEAP_FLAG_STATS is set: class state
 * words, class head/tail words, the pool counter, per-lane atomics on
 * bitmasks, chunk counts and segment counters (spread), and per-lane
 * atomics on ring slots (slot: the lanes of a wave take or fill consecutive
 * positions, so these have their own, lane-contiguous address pattern). */
struct Tally {
    uint32_t state = 0, headtail = 0, pool = 0, spread = 0, slot = 0;
};

__device__ __forceinline__ void tally_flush(const hbheap_dev_t& h, const Tally& t)
{
    if (!(h.flags & HBHEAP_FLAG_STATS)) return;
    uint32_t s, ht, pl, sp, sl;
    (void)excl_scan<20>(t.state, &s);
    (void)excl_scan<20>(t.headtail, &ht);
    (void)excl_scan<20>(t.pool, &pl);
    (void)excl_scan<20>(t.spread, &sp);
    (void)excl_scan<20>(t.slot, &sl);
    if (lane() == ctz64(exec_mask())) {
        if (s) a_add64(h.stats + HBHEAP_STAT_STATE_OPS, s);
        if (ht) a_add64(h.stats + HBHEAP_STAT_HEADTAIL_OPS, ht);
        if (pl) a_add64(h.stats + HBHEAP_STAT_POOL_OPS, pl);
        if (sp) a_add64(h.stats + HBHEAP_STAT_SPREAD_OPS, sp);
        if (sl) a_add64(h.stats + HBHEAP_STAT_SLOT_OPS, sl);
    }
}

/* ---------------- geometry ---------------- */

__device__ __forceinline__ int class_of(const hbheap_dev_t& h, uint64_t n)
{
    if (n == 0 || n > (1ull << h.log2_chunk)) return -1;
    if (n <= 16) return 0;
    return 64 - __builtin_clzll(n - 1) - 4; /* ceil(log2 n) - 4 */
}

/* Index of bitmask word w of chunk c.  Words are stored word-major: word 0
 * of every chunk, then word 1 of every chunk, ...  A class with at most 64
 * pages per chunk uses word 0 only, so the lanes of a wave that work on
 * consecutive chunks of it hit neighbouring words -- a few cache lines per
 * instruction instead of one line per chunk. */
__host__ __device__ __forceinline__ uint64_t bit_index(const hbheap_dev_t& h, uint64_t c, uint32_t w)
{
    return (uint64_t)w * h.n_chunks + c;
}

/* Shard owning chunk c: shards own consecutive runs of 2^log2_span chunks. */
__device__ __forceinline__ uint32_t shard_of_chunk(const hbheap_dev_t& h, uint64_t c)
{
    return (uint32_t)(c >> h.log2_span);
}

/* The shard a wave of a user kernel (dev_malloc) tries first.  Chosen from
 * where the wave runs, read from hardware registers (no memory access, any
 * launch shape): the XCD (XCC_ID) picks one of eight equal runs of shards,
 * and the wave's place inside the XCD (CU, SIMD, wave slot: HW_ID) one shard
 * of that run, so a shard's queues are worked by waves of one XCD.  The
 * library's batch kernels pass their linear wave index instead, which
 * spreads a launch over the shards exactly evenly (and, blocks being
 * dispatched to the XCDs in turn, keeps each shard on one XCD).  With
 * HBHEAP_FLAG_HOME0 every wave starts at shard 0 (the deterministic
 * single-lane replay).  Any value in [0, S) is correct: the choice only
 * spreads the load. */
__device__ __forceinline__ uint32_t home_shard(const hbheap_dev_t& h)
{
    const uint32_t S = h.n_shards;
    if (S == 1 || (h.flags & HBHEAP_FLAG_HOME0)) return 0;
    const uint32_t xcc = __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 7u; /* XCC_ID[3:0] */
    const uint32_t hw = __builtin_amdgcn_s_getreg((31 << 11) | (0 << 6) | 4);       /* HW_ID       */
    /* wave slot [3:0], SIMD [5:4], CU [11:8], SH [12], SE [15:13] */
    const uint32_t local = (hw & 0x3Fu) | ((hw >> 2) & 0x3FC0u);
    const uint32_t mix = (local * 0x9E3779B1u) >> 16;
    if (S < 8u) return (xcc + mix) % S;
    const uint32_t lo = xcc * S / 8u, hi = (xcc + 1u) * S / 8u;
    return lo + mix % (hi - lo);
}

/* ---------------- class ring ---------------- */

struct Ring {
    uint64_t* state;
    uint32_t* head;
    uint32_t* tail;
    uint32_t* slots;  /* plain rings: 2^log2q slots, position p at p & mask */
    uint32_t mask;
    /* segmented rings: the shard's segments (nullptr for a plain ring) and
     * the shard; a virtualised array ring's directory (dmask), or a
     * virtualised list ring's front and back words, the shard's segment
     * tags and links, and the queue's index in the shard */
    uint64_t* dir;
    uint32_t* segs;
    uint32_t dmask;
    uint32_t log2g;
    uint32_t j;
    uint64_t* front;
    uint64_t* back;
    uint64_t* vtag;
    uint64_t* vnext;
    uint32_t k;
};

constexpr uint64_t kDirEmpty = ~0ull;
constexpr uint32_t kStoreBlock = 512; /* state, head, tail, committed pages */

__device__ __forceinline__ uint8_t* class_block(const hbheap_dev_t& h, uint32_t j, uint32_t k)
{
    return h.classes + ((uint64_t)j * h.n_classes + k) * kClassBlock;
}

__device__ __forceinline__ Ring ring_of(const hbheap_dev_t& h, uint32_t j, uint32_t k)
{
    uint8_t* cb = class_block(h, j, k);
    Ring r;
    r.state = (uint64_t*)cb;
    r.head = (uint32_t*)(cb + 128);
    r.tail = (uint32_t*)(cb + 256);
    r.j = j;
    r.k = k;
    r.front = r.back = r.vtag = r.vnext = nullptr;
    if (HBHEAP_VARIANT_SEGMENTED(h.variant)) {
        r.slots = nullptr;
        r.mask = 0;
        r.segs = h.slots + (((uint64_t)j * h.vsegs) << h.log2_seg);
        r.log2g = h.log2_seg;
        if (HBHEAP_VARIANT_IS_VA(h.variant)) {
            r.dir = h.vdir + (((uint64_t)j * h.n_classes + k) << h.log2_dir);
            r.dmask = (1u << h.log2_dir) - 1u;
        } else {
            r.dir = nullptr;
            r.dmask = 0;
            r.front = (uint64_t*)(cb + 392);
            r.back = (uint64_t*)(cb + 400);
            r.vtag = h.vdir + (uint64_t)j * h.vsegs;
            r.vnext = h.vdir + (uint64_t)h.n_shards * h.vsegs + (uint64_t)j * h.vsegs;
        }
    } else {
        r.slots = h.slots + (((uint64_t)j * h.n_classes + k) << h.log2q);
        r.mask = (1u << h.log2q) - 1u;
        r.dir = nullptr;
        r.segs = nullptr;
        r.dmask = 0;
        r.log2g = 0;
    }
    return r;
}
/* The segment store of shard j (virtualised array variant): a plain ring
 * of free segment ids. */
__device__ __forceinline__ Ring store_of(const hbheap_dev_t& h, uint32_t j)
{
    uint8_t* sb = h.vstore + (uint64_t)j * kStoreBlock;
    Ring r;
    r.state = (uint64_t*)sb;
    r.head = (uint32_t*)(sb + 128);
    r.tail = (uint32_t*)(sb + 256);
    r.slots = h.vstore_slots + ((uint64_t)j << h.log2_store);
    r.mask = (1u << h.log2_store) - 1u;
    r.dir = nullptr;
    r.segs = nullptr;
    r.dmask = 0;
    r.log2g = 0;
    r.j = j;
    r.k = 0;
    r.front = r.back = r.vtag = r.vnext = nullptr;
    return r;
}
/* Pages the classes of shard j own together (segmented page variants). */
__device__ __forceinline__ uint64_t* committed_of(const hbheap_dev_t& h, uint32_t j)
{
    return (uint64_t*)(h.vstore + (uint64_t)j * kStoreBlock + 384);
}
__device__ __forceinline__ uint64_t* owned_of(const hbheap_dev_t& h, uint32_t j, uint32_t k)
{
    return (uint64_t*)(class_block(h, j, k) + 384);
}
__device__ __forceinline__ int32_t state_count(uint64_t s) { return (int32_t)((uint32_t)s - kBias); }

/* Leader only.  Takes a hold (H += 1) and reserves up to n published
 * entries; returns how many were reserved.  The hold is dropped by
 * ring_release(), which also publishes entries written meanwhile. */
__device__ __forceinline__ uint32_t ring_reserve(const Ring& r, uint32_t n, Tally& t)
{
    fuzz_point(1);
    const uint64_t old = a_add64(r.state, kHold - n);
    const int32_t c = state_count(old);
    const uint32_t got = c <= 0 ? 0u : ((uint32_t)c < n ? (uint32_t)c : n);
    t.state += 1;
    if (got < n) {
        fuzz_point(2);
        a_add64(r.state, (uint64_t)(n - got));
        t.state += 1;
    }
    return got;
}
/* Leader only: take up to n published entries without a hold, for an
 * operation that will publish nothing (the caller knows it cannot refill);
 * a deficit is given back at once. */
__device__ __forceinline__ uint32_t ring_take_published(const Ring& r, uint32_t n, Tally& t)
{
    fuzz_point(3);
    const uint64_t old = a_add64(r.state, (uint64_t)0 - (uint64_t)n);
    const int32_t c = state_count(old);
    const uint32_t got = c <= 0 ? 0u : ((uint32_t)c < n ? (uint32_t)c : n);
    t.state += 1;
    if (got < n) {
        fuzz_point(4);
        a_add64(r.state, (uint64_t)(n - got));
        t.state += 1;
    }
    return got;
}
__device__ __forceinline__ void ring_release(const Ring& r, uint32_t publish, Tally& t)
{
    fuzz_point(5);
    a_add64(r.state, (uint64_t)publish - kHold);
    t.state += 1;
}

__device__ __forceinline__ uint32_t plain_take(const hbheap_dev_t& h, uint32_t* s, Tally& t);
__device__ __forceinline__ bool plain_put(const hbheap_dev_t& h, uint32_t* s, uint32_t v, Tally& t);

/* Per lane, segment store of shard j: take a free segment id (wait, bounded,
 * while none is published); kEmpty on timeout. */
__device__ __forceinline__ uint32_t store_take(const hbheap_dev_t& h, uint32_t j, Tally& t)
{
    const Ring S = store_of(h, j);
    Backoff b;
    for (;;) {
        const uint64_t old = a_add64(S.state, (uint64_t)0 - 1ull);
        t.state += 1;
        if (state_count(old) > 0) break;
        a_add64(S.state, 1ull);
        if (!b.wait(h)) {
            raise_err(h, HBHEAP_ERR_TIMEOUT, HBHEAP_STAT_TIMEOUTS);
            return kEmpty;
        }
    }
    fuzz_point(10);
    const uint32_t pos = a_add32(S.head, 1u);
    t.headtail += 1;
    return plain_take(h, S.slots + (pos & S.mask), t);
}
/* Per lane: return segment id seg to the store of shard j. */
__device__ __forceinline__ void store_put(const hbheap_dev_t& h, uint32_t j, uint32_t seg, Tally& t)
{
    const Ring S = store_of(h, j);
    const uint32_t pos = a_add32(S.tail, 1u);
    t.headtail += 1;
    fuzz_point(11);
    plain_put(h, S.slots + (pos & S.mask), seg, t);
    fuzz_point(12);
    a_add64(S.state, 1ull);
    t.state += 1;
}

/* Per lane, virtualised array ring: the slot of position pos and its
 * segment.  The segment of position p is number s = p >> log2g; directory
 * entry s mod 2^log2_dir holds (s << 32 | id) while it is in use.  The
 * producer of a segment's first position installs it (a segment from the
 * store, all slots empty) once the entry is empty; everyone else waits for
 * the entry to show segment s.  nullptr on timeout. */
__device__ __forceinline__ uint32_t* va_slot(const hbheap_dev_t& h, const Ring& r, uint32_t pos, bool producer,
                                             uint32_t* seg_out, Tally& t)
{
    const uint32_t s = pos >> r.log2g;
    const uint32_t off = pos & ((1u << r.log2g) - 1u);
    uint64_t* e = r.dir + (s & r.dmask);
    Backoff b;
    for (;;) {
        const uint64_t d = a_load64(e);
        if (d != kDirEmpty && (uint32_t)(d >> 32) == s) {
            *seg_out = (uint32_t)d;
            return r.segs + ((uint64_t)(uint32_t)d << r.log2g) + off;
        }
        if (producer && off == 0 && d == kDirEmpty) {
            const uint32_t seg = store_take(h, r.j, t);
            if (seg == kEmpty) return nullptr;
            fuzz_point(13);
            uint64_t expect = kDirEmpty;
            if (__hip_atomic_compare_exchange_strong(e, &expect, ((uint64_t)s << 32) | seg, __ATOMIC_RELAXED,
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                t.spread += 1;
                *seg_out = seg;
                return r.segs + ((uint64_t)seg << r.log2g);
            }
            store_put(h, r.j, seg, t); /* not reached: one installer per segment */
            continue;
        }
        if (!b.wait(h)) {
            raise_err(h, HBHEAP_ERR_TIMEOUT, HBHEAP_STAT_TIMEOUTS);
            return nullptr;
        }
    }
}

constexpr uint64_t kNoLink = ~0ull;

__device__ __forceinline__ uint64_t a_xchg64(uint64_t* p, uint64_t v)
{
    return __hip_atomic_exchange(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

/* Virtualised list ring, at most once per wave and more as needed: unlink
 * fully consumed segments from the front and return them to the store.  A
 * front segment goes once every slot of it is consumed and a successor is
 * linked (the back stays, for the next producer links from it); the
 * compare-and-swap on the front word picks one retirer.  Whoever completes
 * one of those conditions -- the closer that saw the last count, the
 * installer that linked a successor, the retirer of the segment before --
 * runs this loop after it, with reads that follow its own update (each
 * update returns before the reads that depend on it are issued), so the
 * last of them sees all conditions true. */
__device__ __forceinline__ void vl_retire(const hbheap_dev_t& h, const Ring& r, uint32_t after, Tally& t)
{
    const uint32_t G = 1u << r.log2g;
    uint32_t* taken = h.vtaken + (uint64_t)r.j * h.vsegs;
    bool more = true;
    for (uint32_t guard = 0; more && guard <= h.vsegs; ++guard) {
        more = false;
        const uint64_t f = a_load64(r.front + zero_after(after));
        const uint32_t fm = (uint32_t)f;
        const bool fm_ok = fm < h.vsegs;
        const uint32_t c = fm_ok ? a_load32(taken + fm + zero_after((uint32_t)f)) : 0u;
        const uint64_t nx = fm_ok && c == G ? a_load64(r.vnext + fm + zero_after(c)) : kNoLink;
        if (!fm_ok || (nx != kNoLink && (uint32_t)nx >= h.vsegs)) raise_err(h, HBHEAP_ERR_CORRUPT, HBHEAP_STAT_TIMEOUTS);
        if (fm_ok && c == G && nx != kNoLink && (uint32_t)nx < h.vsegs) {
            fuzz_point(16);
            uint64_t expect = f;
            const bool won = __hip_atomic_compare_exchange_strong(
                r.front + zero_after((uint32_t)nx), &expect, (((f >> 32) + 1ull) << 32) | (uint32_t)nx,
                __ATOMIC_RELAXED, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            after = (uint32_t)expect;
            if (won) {
                t.spread += 1;
                /* this retirer owns the segment: reset its count and link,
                 * both performed before the store hands it out again */
                fuzz_point(17);
                const uint32_t was = a_xchg32(taken + fm, 0u);
                const uint64_t lk = a_xchg64(r.vnext + fm, kNoLink);
                store_put(h, r.j + zero_after(was ^ (uint32_t)lk), fm, t);
                after = was;
            }
            more = true;
        }
    }
}

/* Per lane, virtualised list ring: the slot of position pos and its
 * segment (number s = pos >> log2g).  A producer first reads the back: the
 * back's own segment, or -- for the producer of a segment's first position,
 * once the back is segment s-1 -- a new segment from the store, tagged
 * (queue, s), linked after the back, which then moves to it.  Everyone else
 * walks from the front along the links; a link is trusted only if the
 * segment it was read from still carries the tag the walk expects after the
 * read (a segment retired and handed out again carries another tag, since a
 * queue's segment numbers only grow).  nullptr on timeout. */
__device__ __forceinline__ uint32_t* vl_slot(const hbheap_dev_t& h, const Ring& r, uint32_t pos, bool producer,
                                             uint32_t* seg_out, Tally& t)
{
    const uint32_t s = pos >> r.log2g;
    const uint32_t off = pos & ((1u << r.log2g) - 1u);
    const uint64_t qtag = (uint64_t)r.k << 32;
    Backoff b;
    /* the producer of a segment's first slot takes and tags its segment as
     * soon as it knows its position, while earlier segments are still being
     * linked, and waits only to link it: the links of consecutive segments
     * then follow each other one round trip apart.  An unlinked segment is
     * reachable by no walk (links lead only to linked segments). */
    uint32_t prep = kEmpty, pdep = 0;
    for (;;) {
        bool walk = true;
        if (producer) {
            const uint64_t bk = a_load64(r.back);
            const uint32_t bs = (uint32_t)(bk >> 32), bm = (uint32_t)bk;
            if (bm >= h.vsegs) {
                raise_err(h, HBHEAP_ERR_CORRUPT, HBHEAP_STAT_TIMEOUTS);
                return nullptr;
            }
            if (bs == s) {
                *seg_out = bm;
                return r.segs + ((uint64_t)bm << r.log2g) + off;
            }
            if (off == 0 && (int32_t)(s - bs) >= 1) {
                if (prep == kEmpty) {
                    const uint32_t m = store_take(h, r.j, t);
                    if (m == kEmpty) return nullptr;
                    if (m >= h.vsegs) {
                        raise_err(h, HBHEAP_ERR_CORRUPT, HBHEAP_STAT_TIMEOUTS);
                        return nullptr;
                    }
                    fuzz_point(14);
                    const uint64_t w1 = a_xchg64(r.vtag + m, qtag | s);
                    const uint64_t w2 = a_xchg64(r.vnext + m + zero_after((uint32_t)w1), kNoLink);
                    prep = m;
                    pdep = (uint32_t)w2;
                    t.spread += 2;
                }
                if (bs + 1u == s) {
                    /* the back is segment s - 1: link after it, move the back */
                    const uint64_t w3 = a_xchg64(r.vnext + bm + zero_after(pdep), prep);
                    fuzz_point(15);
                    uint64_t expect = bk;
                    const bool moved = __hip_atomic_compare_exchange_strong(
                        r.back + zero_after((uint32_t)w3), &expect, ((uint64_t)s << 32) | prep, __ATOMIC_RELAXED,
                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    t.spread += 2;
                    if (!moved || w3 != kNoLink) raise_err(h, HBHEAP_ERR_CORRUPT, HBHEAP_STAT_TIMEOUTS);
                    vl_retire(h, r, (uint32_t)expect, t);
                    *seg_out = prep;
                    return r.segs + ((uint64_t)prep << r.log2g);
                }
                walk = false; /* wait for the back to reach segment s - 1 */
            } else {
                walk = (int32_t)(bs - s) > 0; /* a late producer of an older segment */
            }
        }
        if (walk) {
            const uint64_t f = a_load64(r.front);
            uint32_t cs = (uint32_t)(f >> 32), cm = (uint32_t)f;
            bool ok = (int32_t)(s - cs) >= 0 && cm < h.vsegs;
            while (ok && cs != s) {
                const uint64_t nx = a_load64(r.vnext + cm);
                const uint64_t tg = a_load64(r.vtag + cm + zero_after((uint32_t)nx));
                if (tg != (qtag | cs) || nx == kNoLink || (uint32_t)nx >= h.vsegs) {
                    ok = false;
                    break;
                }
                cm = (uint32_t)nx;
                ++cs;
            }
            if (ok) {
                *seg_out = cm;
                return r.segs + ((uint64_t)cm << r.log2g) + off;
            }
        }
        if (!b.wait(h)) {
            raise_err(h, HBHEAP_ERR_TIMEOUT, HBHEAP_STAT_TIMEOUTS);
            /* an unlinked segment goes back to the store, after its tag and
             * link writes */
            if (prep != kEmpty) store_put(h, r.j + zero_after(pdep), prep, t);
            return nullptr;
        }
    }
}

/* Per lane: take the entry of ring position pos (wait while its producer is
 * late).  kEmpty on timeout.  Segmented rings: *seg receives the position's
 * segment id, and the caller counts the slot consumed with
 * seg_count_taken() once the lanes of the wave have taken theirs. */
__device__ __forceinline__ uint32_t slot_take(const hbheap_dev_t& h, const Ring& r, uint32_t pos, uint32_t* seg,
                                              Tally& t)
{
    fuzz_point(20);
    if (r.segs) {
        uint32_t* s = HBHEAP_VARIANT_IS_VL(h.variant) ? vl_slot(h, r, pos, false, seg, t)
                                                      : va_slot(h, r, pos, false, seg, t);
        return s ? plain_take(h, s, t) : kEmpty;
    }
    return plain_take(h, r.slots + (pos & r.mask), t);
}
__device__ __forceinline__ uint32_t slot_take(const hbheap_dev_t& h, const Ring& r, uint32_t pos, Tally& t)
{
    uint32_t seg = 0;
    return slot_take(h, r, pos, &seg, t);
}

/* Segmented rings, wave-wide: the lanes with `took` consumed ring position
 * pos of segment seg of ring r.  Runs of adjacent lanes on one segment
 * (their positions rise with the lane) add their number to its consumed
 * count with one atomic.  The run holding the segment's last position is the
 * segment's closer: its last lane gets the count after its add back (every
 * other lane kEmpty, and every other add returns nothing) and closes the
 * segment with seg_close. */
__device__ __forceinline__ uint32_t seg_count_add(const hbheap_dev_t& h, const Ring& r, bool took, uint32_t pos,
                                                  uint32_t seg, Tally& t)
{
    const uint32_t me = lane();
    const Run run = run_combine(took, (uint64_t)r.j * h.vsegs + seg, 1ull << me, 64u);
    if (!(took && me == run.tail)) return kEmpty;
    const uint32_t n = (uint32_t)__popcll(run.incl);
    const uint32_t G = 1u << r.log2g;
    uint32_t* tk = h.vtaken + (uint64_t)r.j * h.vsegs + seg;
    t.spread += 1;
    fuzz_point(18);
    if ((pos & (G - 1u)) != G - 1u) {
        __hip_atomic_fetch_add(tk, n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return kEmpty;
    }
    return a_add32(tk, n) + n;
}

/* Per closer lane (seg_count_add returned c): once the count shows every
 * slot of the segment consumed (each slot was emptied by its consumer before
 * that consumer was counted), close it: a virtualised array ring empties the
 * directory entry and returns the segment to the store; a virtualised list
 * ring unlinks fully consumed segments from its front.  The wait is bounded
 * by the segment's other consumers, which reserved their positions before
 * the closer and count them without waiting on any closer (a wave with
 * several rows counts all of them before it closes any segment). */
__device__ __forceinline__ void seg_close(const hbheap_dev_t& h, const Ring& r, uint32_t pos, uint32_t seg, uint32_t c,
                                          Tally& t)
{
    const uint32_t G = 1u << r.log2g;
    uint32_t* tk = h.vtaken + (uint64_t)r.j * h.vsegs + seg;
    Backoff b;
    while (c != G) {
        if (!b.wait(h)) {
            raise_err(h, HBHEAP_ERR_TIMEOUT, HBHEAP_STAT_TIMEOUTS);
            return;
        }
        c = a_load32(tk);
        if (HBHEAP_VARIANT_IS_VL(h.variant) && c != G) {
            /* a list segment may already be retired by someone else's
             * loop once its count was full: the retirer moved the front
             * past it before resetting the count this load saw */
            const uint64_t f = a_load64(r.front + zero_after(c));
            if ((int32_t)((uint32_t)(f >> 32) - (pos >> r.log2g)) > 0) return;
        }
    }
    if (HBHEAP_VARIANT_IS_VL(h.variant)) {
        vl_retire(h, r, c, t);
        return;
    }
    /* reset the count and empty the directory entry, both performed
     * before the segment can be taken again: exchanges whose returned
     * values the store's first atomic depends on (no cache-wide
     * release fence) */
    fuzz_point(19);
    const uint32_t was = a_xchg32(tk, 0u);
    const uint64_t ent = __hip_atomic_exchange(r.dir + ((pos >> r.log2g) & r.dmask), kDirEmpty,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    store_put(h, r.j + zero_after(was ^ (uint32_t)ent), seg, t);
}

/* Both steps for one row of consumers. */
__device__ __forceinline__ void seg_count_taken(const hbheap_dev_t& h, const Ring& r, bool took, uint32_t pos,
                                                uint32_t seg, Tally& t)
{
    const uint32_t c = seg_count_add(h, r, took, pos, seg, t);
    if (c != kEmpty) seg_close(h, r, pos, seg, c, t);
}

/* Per lane: the waiting part of taking the entry of slot s, after a first
 * exchange found it empty (its producer is late): poll with loads, exchange
 * once it shows an entry; kEmpty on timeout. */
__device__ __forceinline__ uint32_t plain_take_wait(const hbheap_dev_t& h, uint32_t* s, Tally& t)
{
    Backoff b;
    for (;;) {
        if (!b.wait(h)) {
            raise_err(h, HBHEAP_ERR_TIMEOUT, HBHEAP_STAT_TIMEOUTS);
            return kEmpty;
        }
        if (a_load32(s) != kEmpty) {
            const uint32_t v = a_xchg32(s, kEmpty);
            t.slot += 1;
            if (v != kEmpty) return v;
        }
    }
}

/* Per lane: exchange the entry out of slot s (wait while it is empty).  The
 * first attempt exchanges at once (the slot of a published position is
 * normally full; exchanging an empty slot with the empty mark changes
 * nothing); only a late producer makes it poll with loads. */
__device__ __forceinline__ uint32_t plain_take(const hbheap_dev_t& h, uint32_t* s, Tally& t)
{
    const uint32_t v = a_xchg32(s, kEmpty);
    t.slot += 1;
    if (v != kEmpty) return v;
    return plain_take_wait(h, s, t);
}

/* Per lane: fill ring position pos with v (wait while the slot still holds
 * the entry of the previous lap). */
__device__ __forceinline__ bool slot_put(const hbheap_dev_t& h, const Ring& r, uint32_t pos, uint32_t v, Tally& t)
{
    fuzz_point(21);
    if (r.segs) {
        uint32_t seg = 0;
        uint32_t* s = HBHEAP_VARIANT_IS_VL(h.variant) ? vl_slot(h, r, pos, true, &seg, t)
                                                      : va_slot(h, r, pos, true, &seg, t);
        return s ? plain_put(h, s, v, t) : false;
    }
    return plain_put(h, r.slots + (pos & r.mask), v, t);
}

/* Per lane: the waiting part of filling slot s with v, after a first
 * compare-and-swap found it still full (its consumer of the previous lap is
 * late): poll with loads, swap once it shows empty; false on timeout. */
__device__ __forceinline__ bool plain_put_wait(const hbheap_dev_t& h, uint32_t* s, uint32_t v, Tally& t)
{
    Backoff b;
    for (;;) {
        if (!b.wait(h)) {
            raise_err(h, HBHEAP_ERR_TIMEOUT, HBHEAP_STAT_TIMEOUTS);
            return false;
        }
        if (a_load32(s) == kEmpty) {
            t.slot += 1;
            if (a_cas32(s, kEmpty, v)) return true;
        }
    }
}

/* Per lane: compare-and-swap v into slot s (wait while it is still full).
 * The first attempt swaps at once (the slot of a reserved position is
 * normally empty; a failed swap writes nothing); only a late consumer of
 * the previous lap makes it poll with loads. */
__device__ __forceinline__ bool plain_put(const hbheap_dev_t& h, uint32_t* s, uint32_t v, Tally& t)
{
    t.slot += 1;
    if (a_cas32(s, kEmpty, v)) return true;
    return plain_put_wait(h, s, v, t);
}

/* The slot of ring position pos of queue (shard j, class k) in the plain
 * (unsegmented) ring storage. */
__device__ __forceinline__ uint32_t* plain_slot(const hbheap_dev_t& h, uint32_t j, uint32_t k, uint32_t pos)
{
    return h.slots + (((uint64_t)j * h.n_classes + k) << h.log2q) + (pos & ((1u << h.log2q) - 1u));
}

/* ---------------- pool (per shard) ---------------- */

/* Pool block of shard j (128 B): u64 bump, u32 size, u32 first pool index. */
__device__ __forceinline__ uint64_t* pool_block(const hbheap_dev_t& h, uint32_t j) { return h.pool + 16ull * j; }

/* ---------------- eager retirement (chunk variant) ----------------
 *
 * A chunk's free-page count shares one u64 with a token saying where the
 * chunk is listed, so that a chunk whose pages are all free can leave its
 * class at once, while allocators may be about to take it from its queue.
 * The rules, each transition one atomic on that word:
 * - a chunk with free pages has one token: listed (class, queue position)
 *   or held (an allocator took it from its queue); a chunk with no free
 *   page, or an unowned one, has none;
 * - only the token's owner changes the token; frees only add to the count;
 * - a free that finds no token and a zero count owns the chunk from then
 *   on and lists it (or retires it if the free made it whole);
 * - a free that makes the count whole while the chunk is listed retires it
 *   with a compare-and-swap against that listing; if an allocator took it
 *   meanwhile, the allocator finds it whole when it puts it back and
 *   retires it then;
 * - an allocator that takes an entry from a queue checks it against the
 *   token: an entry whose chunk was retired since (or listed elsewhere)
 *   is stale and is dropped.
 * A retired chunk gets zero bits and the unowned class byte, then goes to
 * the tail of its shard's pool ring, from which refills take chunks. */
constexpr uint32_t kTokNone = 0xFFFFFFFFu, kTokHeld = 0xFFFFFFFEu;

__device__ __forceinline__ bool eager(const hbheap_dev_t& h)
{
    return h.variant == HBHEAP_VARIANT_CHUNK && (h.flags & HBHEAP_FLAG_EAGER) != 0;
}
__host__ __device__ __forceinline__ uint32_t tok_listed(uint32_t k, uint32_t pos) { return (k << 28) | (pos & 0x0FFFFFFFu); }
__host__ __device__ __forceinline__ uint64_t ct_word(uint32_t tok, uint32_t cnt) { return ((uint64_t)tok << 32) | cnt; }
/* The count half holds the free pages in bits 0..15 and, in bit 16 + k,
 * whether the chunk has a stale entry in the queue of class k.  A
 * retirement that leaves a stale entry in queue k needs bit k clear and sets
 * it; the taker that drops the entry clears it.  So queue k holds at most one
 * live and one stale entry per chunk of its shard, and its 2 * span slots
 * never overflow.  (A whole chunk whose bit is still set stays listed until
 * an allocation takes it.) */
constexpr uint32_t kCountMask = 0xFFFFu;
__host__ __device__ __forceinline__ uint32_t stale_bit(uint32_t k) { return 1u << (16u + k); }
__device__ __forceinline__ uint32_t ct_count(uint64_t w) { return (uint32_t)w & kCountMask; }
__device__ __forceinline__ uint32_t ct_stale(uint64_t w) { return (uint32_t)w & ~kCountMask; }
__device__ __forceinline__ bool a_cas64(uint64_t* p, uint64_t& expect, uint64_t v)
{
    return __hip_atomic_compare_exchange_strong(p, &expect, v, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
}

/* The pool ring of shard j (eager retirement): state, head and tail in the
 * shard's pool block, slots in its run of pool ids. */
__device__ __forceinline__ Ring pool_ring(const hbheap_dev_t& h, uint32_t j)
{
    uint64_t* pb = pool_block(h, j);
    Ring r;
    r.state = pb;
    r.head = (uint32_t*)pb + 4;
    r.tail = (uint32_t*)pb + 5;
    r.slots = h.pool_ids + ((uint64_t)j << h.log2_span);
    r.mask = (1u << h.log2_span) - 1u;
    r.dir = nullptr;
    r.segs = nullptr;
    r.dmask = 0;
    r.log2g = 0;
    r.j = j;
    r.k = 0;
    r.front = r.back = r.vtag = r.vnext = nullptr;
    return r;
}

/* Read a word by an atomic that changes nothing.  A read-modify-write reads
 * the last value in the word's modification order; the memory model promises
 * that for no load (a relaxed load may return an older value, and only the
 * hardware's coherent service of agent-scope loads rules that out).  Used on
 * rare paths where a decision -- dropping a queue entry as stale -- would
 * lose a chunk if it rested on a value older than another wave's last
 * atomic on the word.  The zero OR-ed in comes from zero_after, so the
 * compiler cannot turn the atomic back into a load. */
__device__ __forceinline__ uint64_t a_read64(uint64_t* p)
{
    return __hip_atomic_fetch_or(p, (uint64_t)zero_after(lane()), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t a_read32(uint32_t* p)
{
    return __hip_atomic_fetch_or(p, zero_after(lane()), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

/* Wave-wide: the class byte of chunk c for the lanes with `have` (eager
 * retirement changes class bytes while kernels run, on any XCD, so they are
 * read coherently).  Adjacent lanes asking for the same 4-byte word form a
 * run; the first lane of each run reads the word, the others take it from
 * that lane, so frees of neighbouring pages do not all hit one word. */
__device__ __forceinline__ uint32_t class_coherent(const hbheap_dev_t& h, bool have, uint64_t c)
{
    const uint32_t me = lane();
    const uint64_t act = exec_mask();
    const uint32_t key = have ? (uint32_t)(c >> 2) : 0xFFFFFFFFu;
    const uint32_t prev = perm32(key, me ? me - 1u : 0u);
    const bool prev_act = me && ((act >> (me - 1u)) & 1ull);
    const bool first = have && (!prev_act || prev != key);
    uint32_t w = 0;
    if (first) w = a_read32((uint32_t*)(h.chunk_class + (c & ~3ull)));
    const uint64_t heads = __ballot(first);
    const uint64_t upto = me == 63u ? ~0ull : ((2ull << me) - 1ull);
    const uint64_t mine = heads & upto;
    w = perm32(w, have && mine ? 63u - (uint32_t)__builtin_clzll(mine) : me);
    return (w >> ((uint32_t)(c & 3u) * 8u)) & 0xFFu;
}

/* Per lane: reset chunk c of class k, all of whose pages are free and
 * which no token names any more -- its bitmask words (those class k uses;
 * the others are always zero) and its class byte -- by atomics.  Returns a
 * value the put that publishes the chunk must depend on, so that any class
 * that takes it finds it reset. */
__device__ __forceinline__ uint32_t retire_reset(const hbheap_dev_t& h, uint32_t c, uint32_t k, Tally& t)
{
    const uint32_t ppc = 1u << (h.log2_chunk - 4u - k);
    const uint32_t nw = ppc >= 64u ? ppc >> 6 : 1u;
    uint64_t acc = 0;
    for (uint32_t w = 0; w < nw; ++w) acc ^= a_xchg64(h.bits + bit_index(h, c, w), 0ull);
    const uint32_t sh = (c & 3u) * 8u;
    t.spread += nw + 1u;
    return (uint32_t)acc ^ (uint32_t)(acc >> 32) ^ a_or32((uint32_t*)(h.chunk_class + (c & ~3u)), 0xFFu << sh);
}

/* Per lane: retire chunk c of class k -- reset it, then put it at the tail
 * of its shard's pool ring and publish it. */
__device__ __forceinline__ void retire_chunk(const hbheap_dev_t& h, uint32_t c, uint32_t k, Tally& t)
{
    const uint32_t dep = retire_reset(h, c, k, t);
    const Ring P = pool_ring(h, shard_of_chunk(h, c));
    const uint32_t pos = a_add32(P.tail, 1u) + zero_after(dep);
    plain_put(h, P.slots + (pos & P.mask), c, t);
    a_add64(P.state, 1ull);
    t.pool += 2;
    if (h.flags & HBHEAP_FLAG_STATS) a_add64(h.stats + HBHEAP_STAT_RETIRED, 1);
}

/* Wave-wide (every active lane calls it): the lanes with `want` retire
 * their chunk c of class k.  Chunks of one shard go to its pool ring with
 * one tail add and one publish for the group. */
__device__ __forceinline__ void retire_wave(const hbheap_dev_t& h, bool want, uint32_t c, uint32_t k, Tally& t)
{
    uint64_t pend = __ballot(want);
    if (!pend) return;
    uint32_t dep = 0;
    fuzz_point(47);
    if (want) dep = retire_reset(h, c, k, t);
    const uint32_t me = lane();
    const uint32_t j = want ? shard_of_chunk(h, c) : 0u;
    while (pend) {
        const uint32_t leader = ctz64(pend);
        const uint32_t jj = bcast(j, leader);
        const uint64_t grp = __ballot(want && j == jj) & pend;
        const uint32_t n = (uint32_t)__popcll(grp);
        const Ring P = pool_ring(h, jj);
        uint32_t t0 = 0;
        if (me == leader) {
            t0 = a_add32(P.tail, n);
            t.pool += 1;
        }
        t0 = bcast(t0, leader);
        if ((grp >> me) & 1ull) plain_put(h, P.slots + ((t0 + rank_in(grp) + zero_after(dep)) & P.mask), c, t);
        if (me == leader) {
            a_add64(P.state, (uint64_t)n);
            t.pool += 1;
            if (h.flags & HBHEAP_FLAG_STATS) a_add64(h.stats + HBHEAP_STAT_RETIRED, n);
        }
        pend &= ~grp;
    }
}

/* Per lane, by the owner of chunk c's token (a free that found none, or
 * the allocator holding it, which also takes `take` pages off the count
 * here): list the chunk at position pos of its class queue, or retire it if
 * its pages are all free by now.  The caller then fills the slot either way
 * (a retired chunk's entry is stale).  The first value tried is a plain
 * load; a failed compare-and-swap returns the word's current value. */
__device__ __forceinline__ void list_or_retire(const hbheap_dev_t& h, uint32_t c, uint32_t k, uint32_t ppc, uint32_t pos,
                                               uint32_t take, Tally& t)
{
    uint64_t* w = h.chunk_ct + c;
    fuzz_point(46);
    uint64_t v = a_load64(w);
    for (;;) {
        const uint32_t n = ct_count(v) - take;
        t.spread += 1;
        /* retiring leaves the entry the caller puts stale: only without one
         * outstanding in this queue (else the whole chunk stays listed) */
        if (n >= ppc && !(ct_stale(v) & stale_bit(k))) {
            if (a_cas64(w, v, ct_word(kTokNone, ct_stale(v) | stale_bit(k)))) {
                retire_chunk(h, c, k, t);
                return;
            }
        } else if (a_cas64(w, v, ct_word(tok_listed(k, pos), n | ct_stale(v)))) {
            return;
        }
        /* a concurrent free raised the count, or a stale entry was dropped:
         * look again */
    }
}


/* Leader only: take up to m unowned chunks of shard j; *first receives the
 * index in pool_ids of the first one, the return value how many. */
__device__ __forceinline__ uint32_t pool_take(const hbheap_dev_t& h, uint32_t j, uint32_t m, uint64_t* first, Tally& t)
{
    uint64_t* pb = pool_block(h, j);
    if (h.variant == HBHEAP_VARIANT_CHUNK && (h.flags & HBHEAP_FLAG_EAGER)) {
        /* pool ring: *first is the ring position of the first entry taken;
         * the lanes take the entries themselves (pool_entry) */
        if (state_count(a_load64(pb)) <= 0) return 0;
        const uint32_t got = ring_take_published(pool_ring(h, j), m, t);
        if (got) *first = a_add32((uint32_t*)pb + 4, got);
        t.pool += 1;
        return got;
    }
    const uint32_t size = ((const uint32_t*)pb)[2];
    const uint32_t start = ((const uint32_t*)pb)[3];
    if (a_load64(pb) >= size) return 0; /* exhausted: no need to move the bump */
    const uint64_t b = a_add64(pb, m);
    t.pool += 1;
    *first = start + b;
    if (b >= size) return 0;
    return (uint32_t)((size - b) < m ? (size - b) : m);
}
__device__ __forceinline__ bool pool_empty(const hbheap_dev_t& h, uint32_t j)
{
    uint64_t* pb = pool_block(h, j);
    if (h.variant == HBHEAP_VARIANT_CHUNK && (h.flags & HBHEAP_FLAG_EAGER)) return state_count(a_load64(pb)) <= 0;
    return a_load64(pb) >= ((const uint32_t*)pb)[2];
}

/* Page variant: a class may own at most (ring capacity / pages per chunk)
 * chunks of a shard, so its ring can always hold every free page it owns. */
__device__ __forceinline__ uint64_t page_max_chunks(const hbheap_dev_t& h, uint32_t lppc)
{
    return (1ull << h.log2q) >> lppc;
}

__device__ __forceinline__ void count_refill(const hbheap_dev_t& h, uint32_t grabbed)
{
    if (h.flags & HBHEAP_FLAG_STATS) {
        a_add64(h.stats + HBHEAP_STAT_REFILLS, 1);
        if (grabbed) a_add64(h.stats + HBHEAP_STAT_CHUNK_GRABS, grabbed);
    }
}

/* Bitmask words covering pages [u, ppc) of a class, for word w. */
__device__ __forceinline__ uint64_t free_mask_word(uint32_t w, uint32_t u, uint32_t ppc)
{
    const uint32_t lo = w * 64u, hi = lo + 64u;
    const uint32_t a = u > lo ? u : lo, e = ppc < hi ? ppc : hi;
    if (a >= e) return 0;
    const uint64_t upto = (e - lo) == 64 ? ~0ull : ((1ull << (e - lo)) - 1ull);
    return upto & ~((a - lo) == 0 ? 0ull : ((1ull << (a - lo)) - 1ull));
}

__device__ __forceinline__ uint64_t lowest_bits(uint64_t x, uint32_t n)
{
    if ((uint32_t)__popcll(x) <= n) return x;
    uint64_t r = 0;
    for (uint32_t i = 0; i < n; ++i) {
        r |= x & (~x + 1ull);
        x &= x - 1ull;
    }
    return r;
}

/* Per helper lane (chunk variant): clear t free bits of chunk c (class k),
 * lowest first, writing the pages' byte offsets to out[0..t).  The caller
 * already took t from the chunk's count, so t set bits exist; bits lost to a
 * concurrent claimer are looked for again. */
__device__ __forceinline__ uint32_t claim_pages(const hbheap_dev_t& h, uint32_t c, uint32_t k, uint32_t t, uint64_t* out,
                                                Tally& tl)
{
    const uint32_t shift = 4u + k;
    const uint32_t ppc = 1u << (h.log2_chunk - shift);
    const uint32_t nw = ppc >= 64u ? ppc >> 6 : 1u;
    const uint64_t base = (uint64_t)c << h.log2_chunk;
    uint32_t got = 0;
    Backoff b;
    while (got < t) {
        for (uint32_t w = 0; w < nw && got < t; ++w) {
            uint64_t* word = h.bits + bit_index(h, c, w);
            uint64_t x = a_load64(word);
            while (x && got < t) {
                const uint64_t pick = lowest_bits(x, t - got);
                const uint64_t old = a_and64(word, ~pick);
                tl.spread += 1;
                uint64_t won = old & pick;
                while (won) {
                    const uint32_t bit = ctz64(won);
                    won &= won - 1ull;
                    out[got++] = base + ((uint64_t)(w * 64u + bit) << shift);
                }
                x = old & ~pick;
            }
        }
        if (got < t && !b.wait(h)) {
            raise_err(h, HBHEAP_ERR_TIMEOUT, HBHEAP_STAT_TIMEOUTS);
            break;
        }
    }
    return got;
}

/* LDS staging of the chunk variants' page offsets: 64 per wave for one
 * request per lane (up to 16 waves per block), 64 R per wave for R requests
 * per lane (the batch kernels: blocks of at most kRowsBlockWaves waves). */
constexpr uint32_t kRowsBlockWaves = 4;
static __shared__ uint64_t hbheap_stage_lds[kMaxWavesPerBlock * 64];
static __shared__ uint64_t hbheap_stage_lds4[kRowsBlockWaves * 64 * 4];

/* Per-workgroup out-of-memory proof states of a class (batch launches). */
constexpr uint32_t kShareFree = 0, kShareProving = 1, kShareProved = 2;
constexpr uint32_t kShareSlots = 16; /* >= classes of any chunk size */

template <uint32_t R = 1>
__device__ __forceinline__ uint64_t* stage_for_wave()
{
    static_assert(R == 1 || R == 4, "rows per lane: 1 or 4");
    const uint32_t lin = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    if constexpr (R == 1) return hbheap_stage_lds + (lin >> 6) * 64u;
    return hbheap_stage_lds4 + (lin >> 6) * 64u * R;
}

/* ---------------- one class group of one wave ---------------- */

/* The requests one call serves: R per lane ("rows"; request (lane l, row
 * r)).  Requests of one class (inside aligned segments of `width` lanes)
 * form a group; gid is a request's group and rank its place in the group,
 * rows first (row 0's requests in lane order, then row 1's, ...), so that
 * consecutive ranks sit on consecutive lanes of a row.  k < 0: no request
 * there (an invalid size, or a row past the end of the batch).  off
 * receives the page offsets (kNoPage: none). */
template <uint32_t R>
struct Rows {
    int32_t k[R];
    uint32_t gid[R];
    uint32_t rank[R];
    uint64_t off[R];
};

template <uint32_t R>
__device__ __forceinline__ bool in_group(const Rows<R>& q, uint32_t id, uint32_t r)
{
    return q.k[r] >= 0 && q.gid[r] == id;
}

/* Wave-uniform facts about one group of requests.  The leader is the lowest
 * active lane; helpers are the active lanes by rank. */
struct Group {
    uint64_t act;
    uint32_t me, leader, nact, arank;
    uint32_t id;
    uint32_t k, shift, lppc, ppc;
};

__device__ __forceinline__ Group make_group(const hbheap_dev_t& h, uint32_t k, uint32_t id)
{
    Group g;
    g.act = exec_mask();
    g.me = lane();
    g.leader = ctz64(g.act);
    g.nact = (uint32_t)__popcll(g.act);
    g.arank = rank_in(g.act);
    g.id = id;
    g.k = k;
    g.shift = 4u + k;
    g.lppc = h.log2_chunk - g.shift;
    g.ppc = 1u << g.lppc;
    return g;
}

/* The lane that acts for group g in a wave's first pass: the g-th active
 * lane (there are never more groups than active lanes: with one row each
 * lane asks once; with several rows all 64 lanes are active and the width
 * is at least 16, so at most 4 segments x 13 classes). */
__device__ __forceinline__ uint32_t agent_lane(uint64_t act, uint32_t g)
{
    return act == ~0ull ? g : lane_of_rank(act, g);
}

/* Per lane: give unowned chunk c to class k, by an atomic AND on the word
 * holding its class byte (0xFF while unowned); the returned value is not
 * needed, only that the atomic is performed before the chunk's pages are
 * published (write_free_bits waits for it). */
__device__ __forceinline__ void set_class(const hbheap_dev_t& h, uint32_t c, uint32_t k, Tally& tl)
{
    const uint32_t sh = (c & 3u) * 8u;
    (void)a_and32((uint32_t*)(h.chunk_class + (c & ~3u)), ~(0xFFu << sh) | (k << sh));
    tl.spread += 1;
}

/* Wave-wide (the group's lanes): a refill keeps pages [u, ppc) of chunk cl
 * for its queue; set their bits by returning exchanges spread over the
 * lanes, then wait for every access the wave has in flight -- these and the
 * class words -- so that they are performed before the pages are published.
 * (Plain stores would need an agent-scope release fence, which writes back
 * the whole L2 of the XCD.) */
__device__ __forceinline__ void write_free_bits(const hbheap_dev_t& h, uint32_t cl, uint32_t u, const Group& g, Tally& tl)
{
    const uint32_t nw = g.ppc >= 64u ? g.ppc >> 6 : 1u;
    uint64_t acc = 0;
    for (uint32_t w = g.arank; w < nw; w += g.nact) {
        acc ^= a_xchg64(h.bits + bit_index(h, cl, w), free_mask_word(w, u, g.ppc));
        tl.spread += 1;
    }
    __asm__ volatile("" ::"v"((uint32_t)acc), "v"((uint32_t)(acc >> 32)) : "memory");
    wait_own_accesses();
}

/* Rows, per lane: the requests with tk[r] take ring position pos[r] of
 * queue (shard j, class kr[r]); v[r] receives the entry (kEmpty: none, or a
 * wait that timed out).  Plain rings: every row's exchange is issued before
 * any is waited for, so a lane's rows cost one round trip.  Segmented
 * rings: row by row, each row's consumed slots counted once its lanes have
 * taken theirs, and segments closed only after every row is counted
 * (wave-wide: every active lane calls this). */
template <uint32_t R>
__device__ __forceinline__ void take_rows(const hbheap_dev_t& h, uint32_t j, const uint32_t (&kr)[R],
                                          const bool (&tk)[R], const uint32_t (&pos)[R], uint32_t (&v)[R],
                                          Tally& tl)
{
    if (!HBHEAP_VARIANT_SEGMENTED(h.variant)) {
        /* v[r] is left unset where no row takes (and set to kEmpty only after
         * every exchange is issued), so that no copy of a returned value
         * stands between two exchanges and makes the wave wait for the
         * first */
        uint32_t x[R];
#pragma unroll
        for (uint32_t r = 0; r < R; ++r) {
            if (tk[r]) {
                x[r] = a_xchg32(plain_slot(h, j, kr[r], pos[r]), kEmpty);
                tl.slot += 1;
            }
        }
#pragma unroll
        for (uint32_t r = 0; r < R; ++r) {
            v[r] = tk[r] ? x[r] : kEmpty;
            if (tk[r] && v[r] == kEmpty) v[r] = plain_take_wait(h, plain_slot(h, j, kr[r], pos[r]), tl);
        }
        return;
    }
    /* every row's slots taken and counted before any segment is closed: a
     * closer waits for the segment's other consumers to count, and those may
     * be this wave's later rows or another wave that is itself closing a
     * segment of another queue */
    uint32_t seg[R], cl[R];
#pragma unroll
    for (uint32_t r = 0; r < R; ++r) {
        const Ring Q = ring_of(h, j, kr[r]);
        seg[r] = 0;
        v[r] = tk[r] ? slot_take(h, Q, pos[r], &seg[r], tl) : kEmpty;
        cl[r] = seg_count_add(h, Q, tk[r] && v[r] != kEmpty, pos[r], seg[r], tl);
    }
#pragma unroll
    for (uint32_t r = 0; r < R; ++r)
        if (cl[r] != kEmpty) seg_close(h, ring_of(h, j, kr[r]), pos[r], seg[r], cl[r], tl);
}

/* Shared-budget variants: a shard's committed-pages word holds the pages
 * its classes own (bits 0..39) and, above them, the number of refills whose
 * reservation is in flight (added, excess not yet given back). */
constexpr uint32_t kPendShift = 40;
constexpr uint64_t kPendOne = 1ull << kPendShift;
constexpr uint64_t kPagesMask = kPendOne - 1ull;

/* Page variants: reserve room for up to m more chunks of class k in shard j
 * under the cap, by adding first and giving back what passed it.  Returns
 * the number reserved; unused reservations are returned by the caller only
 * when the pool ran dry.
 *  - The page variant keeps one counter per class.  A reader can see it
 *    above the truth only while some adder's excess is still out, and that
 *    adder saw the counter below the cap and took all the room left: so a
 *    reading at or above the cap means no room in truth, and one below it
 *    carries no excess and is exact.
 *  - The shared-budget variants keep one page budget for all classes of a
 *    shard, and an excess of one class could hide a remainder that a class
 *    with fewer pages per chunk could still use.  So each adder also counts
 *    itself in flight in the same atomic and leaves with its give-back: a
 *    reading with nobody in flight is exact, and readers that need the truth
 *    (the exhaustion scan) treat one with adders in flight as undecided.
 * (A compare-and-swap loop gives exact answers too, but with every
 * refilling wave of a shard on one word it retires one success per round
 * trip.) */
__device__ __forceinline__ uint32_t owned_reserve(const hbheap_dev_t& h, uint32_t j, uint32_t k, uint32_t lppc, uint32_t m,
                                                  Tally& tl)
{
    if (HBHEAP_VARIANT_SHARED_PAGES(h.variant)) {
        uint64_t* cm = committed_of(h, j);
        const uint64_t want = (uint64_t)m << lppc;
        const uint64_t c = a_add64(cm, want + kPendOne) & kPagesMask;
        uint32_t allow = m;
        if (c + want > h.vbudget) allow = c < h.vbudget ? (uint32_t)((h.vbudget - c) >> lppc) : 0u;
        a_add64(cm, (uint64_t)0 - (want - ((uint64_t)allow << lppc)) - kPendOne);
        tl.pool += 2;
        if (allow) a_add64(owned_of(h, j, k), allow);
        return allow;
    }
    uint64_t* owned = owned_of(h, j, k);
    const uint64_t maxc = page_max_chunks(h, lppc);
    const uint64_t o = a_add64(owned, m);
    tl.pool += 1;
    if (o + m <= maxc) return m;
    const uint32_t allow = o < maxc ? (uint32_t)(maxc - o) : 0u;
    a_add64(owned, (uint64_t)0 - (uint64_t)(m - allow));
    tl.pool += 1;
    return allow;
}

/* Page variants: may class k of shard j take another chunk?  0: no (exact at
 * the read), 1: yes, 2: undecided (shared budget with refills in flight). */
__device__ __forceinline__ uint32_t class_room(const hbheap_dev_t& h, uint32_t j, uint32_t k, uint32_t lppc)
{
    if (h.variant == HBHEAP_VARIANT_PAGE) return a_load64(owned_of(h, j, k)) < page_max_chunks(h, lppc) ? 1u : 0u;
    if (HBHEAP_VARIANT_SHARED_PAGES(h.variant)) {
        const uint64_t c = a_load64(committed_of(h, j));
        if (c >> kPendShift) return 2u;
        return (c & kPagesMask) + (1ull << lppc) <= h.vbudget ? 1u : 0u;
    }
    return 1u;
}
/* Does shard j show entries or room to grow for class k?  (Pool and room
 * counter read before the state word.)  A wave skips a shard that shows
 * neither instead of taking a hold on it, so waves that find nothing do not
 * keep the shard's hold count busy; undecided room counts as room. */
__device__ __forceinline__ bool class_has_room(const hbheap_dev_t& h, uint32_t j, uint32_t k, uint32_t lppc)
{
    return class_room(h, j, k, lppc) != 0u;
}
__device__ __forceinline__ bool shard_has_something(const hbheap_dev_t& h, uint32_t j, uint32_t k, uint32_t lppc)
{
    bool grow = !pool_empty(h, j);
    if (grow) grow = class_has_room(h, j, k, lppc);
    return grow || state_count(a_load64(ring_of(h, j, k).state)) > 0;
}

/* One look at every shard's queue for the group's class, spread over the
 * active lanes (rank r looks at shards home+r, home+r+nact, ...).  Per
 * shard the pool is read before the state word, head and tail: a pool once
 * empty stays empty until the next trim (with eager retirement, until a free
 * retires a chunk into it, so within a launch that frees nothing it stays
 * empty as well), so "pool empty, then no hold, no
 * entry and head = tail" means the shard had nothing for the class at the
 * moment head was read (no refill in flight, every published entry taken).
 * Returns the rotated rank (from home) of the first shard with published
 * entries or room to grow, or S; *busy tells whether any shard had a hold
 * or a head/tail gap in flight. */
__device__ __forceinline__ uint32_t scan_shards(const hbheap_dev_t& h, const Group& g, uint32_t home, bool* busy)
{
    const uint32_t S = h.n_shards;
    bool anybusy = false;
    for (uint32_t base = 0; base < S; base += g.nact) {
        const uint32_t r = base + g.arank;
        bool avail = false, hold = false;
        if (r < S) {
            const uint32_t j = home + r < S ? home + r : home + r - S;
            /* read in this order (each load's address depends on the value
             * before it): pool, state word, head, tail.  Head before tail:
             * both only grow, so an equal pair means that no published entry
             * was left untaken when head was read; a gap is an operation in
             * flight (a free publishing, or a taker that over-asked without
             * a hold and has not yet given the excess back, while the count
             * can hide entries published meanwhile).  The room counter may
             * be read in any order: a reading of no room is true when read
             * and stays true until the pool runs dry (the only give-back of
             * real room before a trim); an undecided one (refills in flight
             * on a shared budget) counts as an operation in flight. */
            uint64_t* pb = pool_block(h, j);
            const uint64_t bump = a_load64(pb);
            bool grow = eager(h) ? state_count(bump) > 0 : bump < ((const uint32_t*)pb)[2];
            uint32_t room = 1u;
            if (grow) {
                room = class_room(h, j, g.k, g.lppc);
                grow = room == 1u;
            }
            const Ring R = ring_of(h, j, g.k);
            fuzz_point(35);
            const uint64_t st = a_load64(R.state + zero_after((uint32_t)bump));
            fuzz_point(36);
            const uint32_t hd = a_load32(R.head + zero_after((uint32_t)st));
            fuzz_point(37);
            const uint32_t tl_ = a_load32(R.tail + zero_after(hd));
            hold = (st >> 32) != 0 || hd != tl_ || room == 2u;
            avail = state_count(st) > 0 || grow;
        }
        const uint64_t av = __ballot(avail);
        anybusy = anybusy || __ballot(hold) != 0;
        if (av) {
            *busy = anybusy;
            return bcast(r, ctz64(av));
        }
    }
    *busy = anybusy;
    return S;
}

template <uint32_t R>
__device__ __forceinline__ void put_rows(const hbheap_dev_t& h, const uint32_t (&jr)[R], const uint32_t (&kr)[R],
                                         const bool (&pt)[R], const uint32_t (&pos)[R], const uint32_t (&val)[R],
                                         Tally& tl);

/* Wave-wide (chunk variants, a full wave): the helper of rank i (lane i)
 * takes t free bits of its chunk c, lowest first, writing the pages' byte
 * offsets to out[tpre .. tpre + t), as claim_pages does -- but with the
 * (helper, word) pairs spread over the lanes, so that a helper whose pages
 * span several bitmask words reads and clears them all in one round trip
 * each instead of one word after another.  A lane reads its word, takes its
 * share of the helper's t (the lowest set bits, words in order) with one
 * atomicAnd and writes what it won; bits a concurrent claimer took first are
 * looked for again by the helper alone (claim_pages).  Pairs that do not fit
 * the wave fall back to claim_pages per helper. */
__device__ __forceinline__ void claim_wave(const hbheap_dev_t& h, const Group& g, uint32_t nh, uint32_t c, uint32_t t,
                                           uint32_t tpre, uint64_t* out, Tally& tl)
{
    const uint32_t nw = g.ppc >= 64u ? g.ppc >> 6 : 1u;
    if (nh == 0) return;
    if (g.act != ~0ull || nh * nw > 64u) {
        if (t) claim_pages(h, c, g.k, t, out + tpre, tl);
        return;
    }
    const uint32_t me = g.me;
    const uint32_t hi = me / nw, w = me % nw;  /* pair (helper hi, word w) */
    const bool on = hi < nh;
    const uint32_t ch = perm32(c, hi), th = perm32(t, hi), tph = perm32(tpre, hi);
    const bool valid = on && th > 0u;
    uint64_t* word = h.bits + bit_index(h, valid ? ch : 0u, w);
    uint64_t x = 0;
    if (valid) x = a_load64(word);
    const uint32_t pop = valid ? (uint32_t)__popcll(x) : 0u;
    uint32_t tot;
    const uint32_t gp = excl_scan<7>(pop, &tot);
    const uint32_t before = gp - perm32(gp, hi * nw); /* set bits of the helper's lower words */
    const uint32_t q = valid && th > before ? (th - before < pop ? th - before : pop) : 0u;
    uint64_t won = 0;
    if (q) {
        const uint64_t pick = lowest_bits(x, q);
        won = a_and64(word, ~pick) & pick;
        tl.spread += 1;
    }
    const uint32_t nwon = (uint32_t)__popcll(won);
    const uint32_t gw = excl_scan<7>(nwon, &tot);
    uint32_t idx = tph + (gw - perm32(gw, hi * nw));
    const uint64_t cbase = (uint64_t)ch << h.log2_chunk;
    while (won) {
        const uint32_t b = ctz64(won);
        won &= won - 1ull;
        out[idx++] = cbase + ((uint64_t)(w * 64u + b) << g.shift);
    }
    /* helper lanes: what their pairs won in all; the rest alone */
    const uint32_t first = me * nw < 64u ? me * nw : 0u, last = me * nw + nw - 1u < 64u ? me * nw + nw - 1u : 0u;
    const uint32_t mine = perm32(gw + nwon, last) - perm32(gw, first);
    if (t && mine < t) claim_pages(h, c, g.k, t - mine, out + tpre + mine, tl);
}

/* Eager refills, wave-wide: the chunk of refill rank q (< RQ nact), held in
 * slot q / nact of the lane of rank q mod nact (every lane calls this: the
 * lanes read from must be active). */
template <uint32_t RQ>
__device__ __forceinline__ uint32_t refill_chunk(const Group& g, const uint32_t (&mine)[RQ], uint32_t q)
{
    const uint32_t slot = RQ == 1 ? 0u : q / g.nact;
    const uint32_t src = lane_of_rank(g.act, q - slot * g.nact);
    uint32_t ci = kEmpty;
#pragma unroll
    for (uint32_t b = 0; b < RQ; ++b) {
        const uint32_t v = perm32(mine[b], src);
        if (b == slot) ci = v;
    }
    return ci;
}

/* Chunk variant, shard j: serve up to `need` pages of the group's class,
 * writing their byte offsets to stage[served..).  Returns when need is met
 * or when shard j's queue and pool could not supply more. */
template <uint32_t RQ, uint32_t RW>
__device__ __forceinline__ void chunk_serve_shard(const hbheap_dev_t& h, const Group& g, uint32_t j, uint32_t& need,
                                                  uint32_t& served, uint64_t* stage, bool look_first, Tally& tl)
{
    const Ring R = ring_of(h, j, g.k);
    /* RQ requests per lane, RW queue entries per lane and pass.  Several
     * entries per lane (RW > 1) only without eager retirement: there a lane
     * takes at most one entry per pass (it takes the entry's token by a
     * compare-and-swap), whatever its number of requests */
    static_assert(RW == 1 || RW == RQ, "queue entries per lane: 1 or one per request");
    const bool ev = RW == 1 && eager(h);
    /* a group's need is at most 64 RQ: scans of per-lane page counts */
    constexpr int kBits = RQ == 1 ? 7 : 9;
    /* look before reserving, except on a first pass the caller vouches for
     * (a home shard whose pool still had chunks, or a shard a scan just found
     * something in): there an empty queue costs only a hold taken and given
     * back, while on a dry shard such holds would keep scanning waves waiting */
    bool first_pass = !look_first;
    while (need > 0) {
        if (!first_pass) {
            uint32_t some = 0;
            if (g.me == g.leader) some = shard_has_something(h, j, g.k, g.lppc);
            if (!bcast(some, g.leader)) return;
        }
        first_pass = false;
        const uint32_t want0 = (need + g.ppc - 1u) >> g.lppc;
        /* each lane takes up to K queue entries (K = requests per lane:
         * entry i * nact + rank of the reservation), all in flight together */
        constexpr uint32_t K = RW;
        const uint32_t want = want0 < g.nact * K ? want0 : g.nact * K;
        uint32_t got = 0, h0 = 0;
        if (g.me == g.leader) {
            got = ring_reserve(R, want, tl);
            if (got) {
                h0 = a_add32(R.head, got);
                tl.headtail += 1;
            }
        }
        got = bcast(got, g.leader);
        h0 = bcast(h0, g.leader);

        /* helpers take their chunks (segmented rings: every slot counted
         * consumed before any segment is closed) and read their free counts */
        uint32_t c[K], kq[K], qpos[K];
        bool tk[K];
        int32_t v[K];
#pragma unroll
        for (uint32_t i = 0; i < K; ++i) {
            tk[i] = i * g.nact + g.arank < got;
            qpos[i] = h0 + i * g.nact + g.arank;
            kq[i] = g.k;
            v[i] = 0;
        }
        take_rows<K>(h, j, kq, tk, qpos, c, tl);
        bool stale = false;
#pragma unroll
        for (uint32_t i = 0; i < K; ++i) {
            if (!tk[i]) c[i] = kEmpty;
            if (c[i] != kEmpty && (c[i] >= h.n_chunks || shard_of_chunk(h, c[i]) != j)) {
                raise_err(h, HBHEAP_ERR_CORRUPT, HBHEAP_STAT_TIMEOUTS);
                c[i] = kEmpty;
            }
        }
        if (ev && c[0] != kEmpty) {
            /* take the chunk's token from its listing; an entry the token
             * does not name is stale: dropped.  A listing is matched by its
             * class and its position modulo the ring capacity: a slow taker
             * of position p - Q and the taker of p take from the same slot and
             * may get each other's entries, which leaves each entry in the
             * slot its position maps to.  Only one taker can win the token,
             * whichever copy it came by. */
            uint64_t* w = h.chunk_ct + c[0];
            uint64_t x = a_load64(w);   /* a guess: an entry is dropped only on a coherent value */
            bool sure = false;
            const uint32_t mine = tok_listed(g.k, h0 + g.arank);
            for (;;) {
                const uint32_t tk0 = (uint32_t)(x >> 32);
                if (tk0 >= kTokHeld || (tk0 >> 28) != g.k || ((tk0 ^ mine) & R.mask) != 0) {
                    if (!sure) {
                        x = a_read64(w);
                        sure = true;
                        tl.spread += 1;
                        continue;
                    }
                    stale = true;
                    /* the chunk's stale entry in this queue is gone */
                    __hip_atomic_fetch_and(w, ~(uint64_t)stale_bit(g.k), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    tl.spread += 1;
                    break;
                }
                tl.spread += 1;
                if (a_cas64(w, x, ct_word(kTokHeld, (uint32_t)x))) {
                    v[0] = (int32_t)ct_count(x);
                    break;
                }
                sure = true;
            }
            if (!stale && v[0] <= 0) raise_err(h, HBHEAP_ERR_CORRUPT, HBHEAP_STAT_TIMEOUTS);
        } else if (!ev) {
#pragma unroll
            for (uint32_t i = 0; i < K; ++i)
                if (c[i] != kEmpty) v[i] = a_loadi(h.chunk_cnt + c[i]);
#pragma unroll
            for (uint32_t i = 0; i < K; ++i)
                if (c[i] != kEmpty && v[i] <= 0) raise_err(h, HBHEAP_ERR_CORRUPT, HBHEAP_STAT_TIMEOUTS);
        }
        fuzz_point(28);
        /* stale entries dropped: progress even if nothing was served */
        const bool dropped = ev && __ballot(stale) != 0;
        /* pages each chunk gives, in entry order (entry i * nact + rank) */
        uint32_t t[K], tpre[K], vc[K];
        bool keep[K];
        uint32_t base = 0;
        /* rows of entries in use (wave-uniform): the rest skip their scans */
        const uint32_t rows = (got + g.nact - 1u) / g.nact;
#pragma unroll
        for (uint32_t i = 0; i < K; ++i) {
            vc[i] = v[i] > 0 ? ((uint32_t)v[i] < need ? (uint32_t)v[i] : need) : 0u;
            t[i] = 0;
            if (i < rows) {
                uint32_t tot;
                const uint32_t pre = base + excl_scan<kBits>(vc[i], &tot);
                base += tot;
                t[i] = pre < need ? ((need - pre) < vc[i] ? (need - pre) : vc[i]) : 0u;
            }
        }
        int32_t cnt[K];
#pragma unroll
        for (uint32_t i = 0; i < K; ++i) {
            if (!ev && t[i]) {
                fuzz_point(29);
                cnt[i] = a_addi(h.chunk_cnt + c[i], -(int32_t)t[i]);
                tl.spread += 1;
            }
        }
#pragma unroll
        for (uint32_t i = 0; i < K; ++i) {
            keep[i] = false;
            if (vc[i] > 0) {
                /* eager: the count is lowered by t when the token is put
                 * back (list_or_retire, or the release below): while it is
                 * held nobody else takes pages from the chunk and frees only
                 * add */
                if (t[i] && ev) keep[i] = (uint32_t)v[i] > t[i];
                else if (t[i]) keep[i] = cnt[i] - (int32_t)t[i] > 0;
                else keep[i] = true;
            }
        }
        uint32_t took = 0;
#pragma unroll
        for (uint32_t i = 0; i < K; ++i) {
            tpre[i] = took;
            if (i < rows) {
                uint32_t tt;
                tpre[i] = took + excl_scan<kBits>(t[i], &tt);
                took += tt;
            }
        }
        /* a pass that will not refill (its reservations cover the need, or
         * the queue gave every chunk asked for) puts its kept chunks back
         * and releases the queue before it claims its pages' bits, so other
         * waves can take those chunks meanwhile: the pages it claims are
         * already taken off the counts, which stay within the free bits */
        const bool early = !(got < want && need > took);
        fuzz_point(30);
        if (!early) {
#pragma unroll
            for (uint32_t i = 0; i < K; ++i) {
                const uint32_t nh = got > i * g.nact ? (got - i * g.nact < g.nact ? got - i * g.nact : g.nact) : 0u;
                claim_wave(h, g, nh, c[i], t[i], tpre[i], stage + served, tl);
            }
        }

        /* chunks that still hold free pages go back to the tail */
        uint32_t nrq = 0, rpos[K], jq[K];
#pragma unroll
        for (uint32_t i = 0; i < K; ++i) {
            rpos[i] = 0;
            jq[i] = j;
            if (i < rows) {
                const uint64_t rq = __ballot(keep[i]);
                rpos[i] = nrq + rank_in(rq);
                nrq += (uint32_t)__popcll(rq);
            }
        }
        uint32_t t0 = 0;
        fuzz_point(31);
        if (nrq && g.me == g.leader) {
            t0 = a_add32(R.tail, nrq);
            tl.headtail += 1;
        }
        t0 = bcast(t0, g.leader);
#pragma unroll
        for (uint32_t i = 0; i < K; ++i) rpos[i] += t0;
        if (ev) {
            if (keep[0]) {
                list_or_retire(h, c[0], g.k, g.ppc, rpos[0], t[0], tl);
                slot_put(h, R, rpos[0], c[0], tl);
            }
        } else {
            put_rows<K>(h, jq, kq, keep, rpos, c, tl);
        }
        if (ev && vc[0] > 0 && !keep[0]) {
            /* every free page taken: give the token up -- unless frees came
             * in while it was held, which left it to this lane to list the
             * chunk again (or retire it) */
            uint64_t x = a_load64(h.chunk_ct + c[0]);
            bool released = false;
            tl.spread += 1;
            /* held, and no page freed meanwhile: give it up (keep the stale flag) */
            while (ct_count(x) == t[0] && (uint32_t)(x >> 32) == kTokHeld)
                if ((released = a_cas64(h.chunk_ct + c[0], x, ct_word(kTokNone, ct_stale(x))))) break;
            if (!released) {
                const uint32_t pos = a_add32(R.tail, 1u);
                tl.headtail += 1;
                list_or_retire(h, c[0], g.k, g.ppc, pos, t[0], tl);
                slot_put(h, R, pos, c[0], tl);
                a_add64(R.state, 1ull);
                tl.state += 1;
            }
        }
        if (early) {
            if (g.me == g.leader) ring_release(R, nrq, tl);
#pragma unroll
            for (uint32_t i = 0; i < K; ++i) {
                const uint32_t nh = got > i * g.nact ? (got - i * g.nact < g.nact ? got - i * g.nact : g.nact) : 0u;
                claim_wave(h, g, nh, c[i], t[i], tpre[i], stage + served, tl);
            }
            need -= took;
            served += took;
            /* entries reserved but nothing served: a wait gave up (error raised) */
            if (got > 0 && took == 0 && !dropped) return;
            continue;
        }
        need -= took;
        served += took;

        uint32_t publish = nrq;
        bool exhausted = false;
        if (got < want && need > 0) {
            /* refill from the shard's pool while still holding the queue
             * (eager retirement: at most RQ chunks per active lane, each lane
             * taking its own from the pool ring, all in flight together; a
             * need beyond that takes further passes) */
            uint32_t m = (need + g.ppc - 1u) >> g.lppc;
            if (ev && m > g.nact * RQ) m = g.nact * RQ;
            uint64_t first = 0;
            uint32_t gm = 0;
            if (g.me == g.leader) {
                gm = pool_take(h, j, m, &first, tl);
                count_refill(h, gm);
            }
            gm = bcast(gm, g.leader);
            first = bcast64(first, g.leader);
            exhausted = gm < m;
            fuzz_point(32);
            /* the chunk of rank q among those taken: a pool id (bump pool),
             * or what the lane of rank q mod nact took from the pool ring
             * into its slot q / nact */
            uint32_t mine[RQ];
#pragma unroll
            for (uint32_t b = 0; b < RQ; ++b) mine[b] = kEmpty;
            if (ev) {
                const Ring P = pool_ring(h, j);
                uint32_t x[RQ];
                bool fail = false;
#pragma unroll
                for (uint32_t b = 0; b < RQ; ++b) {
                    const uint32_t q = g.arank + b * g.nact;
                    if (q < gm) {
                        x[b] = a_xchg32(P.slots + (((uint32_t)first + q) & P.mask), kEmpty);
                        tl.slot += 1;
                    }
                }
#pragma unroll
                for (uint32_t b = 0; b < RQ; ++b) {
                    const uint32_t q = g.arank + b * g.nact;
                    if (q < gm) {
                        mine[b] = x[b] != kEmpty ? x[b]
                                                 : plain_take_wait(h, P.slots + (((uint32_t)first + q) & P.mask), tl);
                        fail = fail || mine[b] == kEmpty;
                    }
                }
                if (__ballot(fail)) { /* a wait gave up (error raised) */
                    gm = 0;
                    exhausted = true;
                }
#pragma unroll
                for (uint32_t b = 0; b < RQ; ++b)
                    if (g.arank + b * g.nact < gm) set_class(h, mine[b], g.k, tl);
                wait_own_accesses();
            } else {
                for (uint32_t i = g.arank; i < gm; i += g.nact) set_class(h, h.pool_ids[first + i], g.k, tl);
            }
            const uint32_t cap = gm << g.lppc;
            const uint32_t r = cap < need ? cap : need;
            if (ev && gm) {
                /* page i of the refill (i < r <= 64 RQ) is in chunk i >> lppc:
                 * RQ uniform rounds, so every lane read from is active */
#pragma unroll
                for (uint32_t b = 0; b < RQ; ++b) {
                    const uint32_t i = g.arank + b * g.nact;
                    const uint32_t q = (i >> g.lppc) < gm ? (i >> g.lppc) : gm - 1u;
                    const uint32_t ci = refill_chunk<RQ>(g, mine, q);
                    if (i < r)
                        stage[served + i] = ((uint64_t)ci << h.log2_chunk) + ((uint64_t)(i & (g.ppc - 1u)) << g.shift);
                }
            } else {
                for (uint32_t i = g.arank; i < r; i += g.nact) {
                    const uint32_t ci = h.pool_ids[first + (i >> g.lppc)];
                    stage[served + i] = ((uint64_t)ci << h.log2_chunk) + ((uint64_t)(i & (g.ppc - 1u)) << g.shift);
                }
            }
            if (cap > need) {
                /* last chunk keeps pages [u, ppc): set their bits, publish it */
                const uint32_t last = gm - 1u;
                const uint32_t u = need - (last << g.lppc);
                const uint32_t cl = ev ? refill_chunk<RQ>(g, mine, last) : h.pool_ids[first + last];
                /* the free count (lazy retirement; with eager retirement it
                 * is set with the listing below) and the bit words by
                 * returning exchanges, waited for: performed before the chunk
                 * is listed, with no write-back of the L2 */
                uint32_t pos = 0;
                if (g.me == g.leader) {
                    if (!ev) {
                        (void)a_xchg32((uint32_t*)(h.chunk_cnt + cl), g.ppc - u);
                        tl.spread += 1;
                    }
                    /* its tail position, reserved in the same round trip */
                    pos = a_add32(R.tail, 1u);
                    tl.headtail += 1;
                }
                write_free_bits(h, cl, u, g, tl);
                fuzz_point(33);
                if (g.me == g.leader) {
                    if (ev) {
                        /* listed at pos, with pages [u, ppc) free */
                        /* keep the stale flag, which a taker dropping an entry
                         * of this chunk may clear meanwhile */
                        uint64_t was = a_load64(h.chunk_ct + cl);
                        while (!a_cas64(h.chunk_ct + cl, was, ct_word(tok_listed(g.k, pos), (g.ppc - u) | ct_stale(was))))
                            tl.spread += 1;
                        tl.spread += 1;
                        pos += zero_after((uint32_t)was);
                    }
                    slot_put(h, R, pos, cl, tl);
                }
                publish += 1u;
            }
            need -= r;
            served += r;
        }
        if (g.me == g.leader) ring_release(R, publish, tl);
        if (need > 0 && got < want && exhausted) return;
        /* entries reserved but nothing served: a wait gave up (error raised) */
        if (got > 0 && took == 0 && !dropped) return;
    }
}

/* Page variant: lanes with `have` clear `bit` of bitmask word `widx` (the
 * page is theirs: they took it from the queue); each run of adjacent lanes
 * on one word clears its bits with one atomicAnd, and `off` becomes the
 * lane's page offset `o`.  With HBHEAP_FLAG_VERIFY the old word is waited
 * for and a page whose bit was already clear (a heap fault) is not handed
 * out; without it the clearing atomic returns nothing, so the allocation
 * does not wait for it. */
__device__ __forceinline__ void clear_bits_grouped(const hbheap_dev_t& h, bool have, uint64_t widx, uint64_t bit,
                                                   uint64_t o, uint32_t shift, uint32_t p, uint64_t& off, Tally& tl)
{
    Run r;
    if (!run_consecutive(have, o, shift, 1u << (h.log2_chunk - shift), p, r)) r = run_combine(have, widx, bit, 64u);
    if (!(h.flags & HBHEAP_FLAG_VERIFY)) {
        if (have && lane() == r.tail) {
            __hip_atomic_fetch_and(h.bits + widx, ~r.incl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            tl.spread += 1;
        }
        if (have) off = o;
        return;
    }
    uint64_t old = 0;
    if (have && lane() == r.tail) {
        old = a_and64(h.bits + widx, ~r.incl);
        tl.spread += 1;
    }
    old = perm64(old, r.tail);
    if (have) {
        if (old & bit) off = o;
        else raise_err(h, HBHEAP_ERR_CORRUPT, HBHEAP_STAT_TIMEOUTS);
    }
}

/* Page variants, wave-wide: a lane that took entry v (kEmpty: none) from a
 * queue of shard j gets that page (off) and its bit is cleared, one
 * atomicAnd per run of lanes on one bitmask word. */
__device__ __forceinline__ void page_took(const hbheap_dev_t& h, uint32_t j, uint32_t shift, uint32_t v, uint64_t& off,
                                          Tally& tl)
{
    bool took = false;
    uint64_t widx = 0, bit = 0, o = 0;
    uint32_t p = 0;
    if (v != kEmpty) {
        o = (uint64_t)v << 4;
        if (o >= h.data_bytes || shard_of_chunk(h, o >> h.log2_chunk) != j) {
            raise_err(h, HBHEAP_ERR_CORRUPT, HBHEAP_STAT_TIMEOUTS);
        } else {
            const uint64_t c = o >> h.log2_chunk;
            p = (uint32_t)((o & ((1ull << h.log2_chunk) - 1ull)) >> shift);
            widx = bit_index(h, c, p >> 6);
            bit = 1ull << (p & 63u);
            took = true;
        }
    }
    clear_bits_grouped(h, took, widx, bit, o, shift, p, off, tl);
}

/* Page variant, shard j: the group's requests of ranks [served,
 * served+need) receive pages (q.off). */
template <uint32_t R>
__device__ __forceinline__ void page_serve_shard(const hbheap_dev_t& h, const Group& g, Rows<R>& q, uint32_t j,
                                                 uint32_t& need, uint32_t& served, bool dry, bool check_first,
                                                 Tally& tl, bool hold_first = false)
{
    const Ring Q = ring_of(h, j, g.k);
    /* The first pass (which looks first only if check_first) takes published
     * entries without a hold: it never refills, so it has nothing to publish
     * and a scanning wave need not wait on it (an over-ask it gives back is
     * covered by the scan's head/tail test instead).  Short of pages, the
     * next passes look first and hold the queue, so they may refill -- except
     * on a shard the caller saw with a dry pool (dry stays dry until a trim):
     * there the caller scans instead.  hold_first: the caller has just made
     * that first pass itself and saw the pool not dry, so the first pass here
     * holds at once, without a look (a look could only say that the pool has
     * chunks; should it have run dry meanwhile, the held pass finds it so and
     * returns, and the caller scans). */
    bool look = check_first && !hold_first, held = hold_first;
    while (need > 0) {
        if (look) {
            uint32_t some = 0;
            if (g.me == g.leader) some = shard_has_something(h, j, g.k, g.lppc);
            if (!bcast(some, g.leader)) return;
        }
        look = true;
        uint32_t got = 0, h0 = 0;
        if (g.me == g.leader) {
            got = held ? ring_reserve(Q, need, tl) : ring_take_published(Q, need, tl);
            if (got) {
                fuzz_point(22);
                h0 = a_add32(Q.head, got);
                tl.headtail += 1;
            }
        }
        got = bcast(got, g.leader);
        h0 = bcast(h0, g.leader);
        /* takers read their slots (all rows at once); then the bits of taken
         * pages are cleared, one atomicAnd per run of lanes on one word */
        bool tk[R];
        uint32_t pos[R], kr[R], v[R];
#pragma unroll
        for (uint32_t r = 0; r < R; ++r) {
            tk[r] = in_group(q, g.id, r) && q.rank[r] >= served && q.rank[r] < served + got;
            pos[r] = h0 + (q.rank[r] - served);
            kr[r] = g.k;
        }
        take_rows<R>(h, j, kr, tk, pos, v, tl);
        fuzz_point(23);
#pragma unroll
        for (uint32_t r = 0; r < R; ++r) page_took(h, j, g.shift, v[r], q.off[r], tl);
        need -= got;
        served += got;

        uint32_t publish = 0;
        bool exhausted = !held && dry;
        if (need > 0 && held) {
            const uint32_t m = (need + g.ppc - 1u) >> g.lppc;
            uint64_t first = 0;
            uint32_t gm = 0;
            if (g.me == g.leader) {
                if (!pool_empty(h, j)) {
                    const uint32_t allow = owned_reserve(h, j, g.k, g.lppc, m, tl);
                    fuzz_point(24);
                    gm = allow ? pool_take(h, j, allow, &first, tl) : 0u;
                    if (gm < allow) {
                        /* the pool ran dry: give back what was not taken */
                        a_add64(owned_of(h, j, g.k), (uint64_t)0 - (uint64_t)(allow - gm));
                        if (HBHEAP_VARIANT_SHARED_PAGES(h.variant))
                            a_add64(committed_of(h, j), (uint64_t)0 - ((uint64_t)(allow - gm) << g.lppc));
                        tl.pool += 1;
                    }
                }
                count_refill(h, gm);
            }
            gm = bcast(gm, g.leader);
            first = bcast64(first, g.leader);
            exhausted = gm < m;
            fuzz_point(25);
            /* the chunks' class bytes, by atomics on their words (an unowned
             * chunk's byte is 0xFF, so an AND sets it): like every word other
             * waves read during a kernel, written where device atomics are
             * performed */
            for (uint32_t i = g.arank; i < gm; i += g.nact) set_class(h, h.pool_ids[first + i], g.k, tl);
            const uint32_t cap = gm << g.lppc;
            const uint32_t rr = cap < need ? cap : need;
#pragma unroll
            for (uint32_t r = 0; r < R; ++r) {
                if (in_group(q, g.id, r) && q.rank[r] >= served && q.rank[r] < served + rr) {
                    const uint32_t qq = q.rank[r] - served;
                    const uint32_t ci = h.pool_ids[first + (qq >> g.lppc)];
                    q.off[r] = ((uint64_t)ci << h.log2_chunk) + ((uint64_t)(qq & (g.ppc - 1u)) << g.shift);
                }
            }
            if (cap > need) {
                const uint32_t last = gm - 1u;
                const uint32_t u = need - (last << g.lppc);
                const uint32_t cl = h.pool_ids[first + last];
                /* its free bits by returning exchanges, and the wave waits for
                 * them (and the class words): performed before any of its pages
                 * is published, with no write-back of the L2.  The tail
                 * positions are reserved in the same round trip (a reserved
                 * position is taken by nobody before its count is published) */
                const uint32_t L = g.ppc - u;
                uint32_t t0 = 0;
                fuzz_point(26);
                if (g.me == g.leader) {
                    t0 = a_add32(Q.tail, L);
                    tl.headtail += 1;
                }
                write_free_bits(h, cl, u, g, tl);
                t0 = bcast(t0, g.leader);
                const uint64_t cbase = ((uint64_t)cl << h.log2_chunk) >> 4;
                const uint32_t step = 1u << (g.shift - 4u);
                fuzz_point(27);
                if (!Q.segs) {
                    /* eight compare-and-swaps per lane in flight at a time */
                    for (uint32_t i0 = g.arank; i0 < L; i0 += 8u * g.nact) {
                        uint32_t was[8];
#pragma unroll
                        for (uint32_t b = 0; b < 8u; ++b) {
                            const uint32_t i = i0 + b * g.nact;
                            was[b] = kEmpty;
                            if (i < L) {
                                was[b] = a_cas32_old(Q.slots + ((t0 + i) & Q.mask), kEmpty,
                                                     (uint32_t)cbase + (u + i) * step);
                                tl.slot += 1;
                            }
                        }
#pragma unroll
                        for (uint32_t b = 0; b < 8u; ++b) {
                            const uint32_t i = i0 + b * g.nact;
                            if (i < L && was[b] != kEmpty)
                                plain_put_wait(h, Q.slots + ((t0 + i) & Q.mask), (uint32_t)cbase + (u + i) * step, tl);
                        }
                    }
                } else {
                    for (uint32_t i = g.arank; i < L; i += g.nact)
                        slot_put(h, Q, t0 + i, (uint32_t)cbase + (u + i) * step, tl);
                }
                publish = L;
            }
            need -= rr;
            served += rr;
        }
        if (held && g.me == g.leader) ring_release(Q, publish, tl);
        if (need > 0 && exhausted) return;
        held = true;
    }
}

/* Serve one class group (id, class k, tot requests): the home shard first;
 * then, while requests remain, scan every shard at once and serve from the
 * first one (after home) that has entries or room to grow; give up only when
 * a scan finds every shard without entries, without room and without holds
 * in flight.  The group's requests receive their page offsets in q.off
 * (unchanged: kNoPage).  Chunk variants stage the group's offsets in LDS
 * (64 R per wave) and hand them out by rank at the end. */
template <uint32_t R>
__device__ __forceinline__ void chunk_serve(const hbheap_dev_t& h, const Group& g, uint32_t j, uint32_t& need,
                                            uint32_t& served, uint64_t* stage, bool look_first, Tally& tl)
{
    if constexpr (R > 1) {
        if (eager(h)) {
            chunk_serve_shard<R, 1>(h, g, j, need, served, stage, look_first, tl);
            return;
        }
    }
    chunk_serve_shard<R, R>(h, g, j, need, served, stage, look_first, tl);
}

template <uint32_t R>
__device__ __forceinline__ void alloc_group(const hbheap_dev_t& h, Rows<R>& q, uint32_t id, uint32_t k, uint32_t tot,
                                            uint64_t* stage, uint32_t home, bool home_dry, uint32_t served0,
                                            bool home_tried, uint32_t* share, Tally& tl)
{
    const Group g = make_group(h, k, id);
    const bool chunk = HBHEAP_VARIANT_LISTS_CHUNKS(h.variant);
    if (chunk) {
        for (uint32_t i = g.arank; i < tot; i += g.nact) stage[i] = kNoPage;
        wave_sync_lds();
    }
    /* ranks below served0 were served already (page variant: the wave's
     * first pass over all its groups at once, on the home shard; after it,
     * home_tried makes the home shard hold at once where its pool was not
     * dry, and look before it reserves again where it was) */
    uint32_t need = tot - served0, served = served0;
    const uint32_t S = h.n_shards;
    if (chunk) chunk_serve<R>(h, g, home, need, served, stage, home_dry, tl);
    else page_serve_shard<R>(h, g, q, home, need, served, home_dry && !home_tried, home_tried, tl,
                             home_tried && !home_dry);
    Backoff wb;
    bool timed_out = false;
    /* share != nullptr (a batch launch, whose requests were all issued when
     * it began): the waves of one workgroup share out-of-memory proofs of a
     * class through LDS.  One of them (the prover) scans; its finding that
     * every shard was exhausted at some instant -- an instant inside the
     * interval of every request of the launch still unanswered -- answers
     * its workgroup mates too, who wait for it instead of scanning the same
     * hot queue words.  A prover that finds entries instead gives up the
     * claim; a wait that runs out scans on its own. */
    bool prover = false;
    while (need > 0) {
        if (share && !prover) {
            uint32_t* sk = share + k;
            Backoff pb;
            bool answered = false;
            for (;;) {
                const uint32_t v = __hip_atomic_load(sk, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (v == kShareProved) {
                    answered = true;
                    break;
                }
                if (v == kShareFree) {
                    uint32_t won = 0;
                    if (g.me == g.leader) {
                        uint32_t expect = kShareFree;
                        won = __hip_atomic_compare_exchange_strong(sk, &expect, kShareProving, __ATOMIC_RELAXED,
                                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                    if (bcast(won, g.leader)) {
                        prover = true;
                        break;
                    }
                }
                if (!pb.wait(h)) break;
            }
            if (answered) break;
        }
        bool busy = false;
        const uint32_t r = scan_shards(h, g, home, &busy);
        if (r == S && !busy) { /* every shard empty for this class: out of memory */
            if (prover && g.me == g.leader)
                __hip_atomic_store(share + k, kShareProved, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            break;
        }
        if (prover && r < S) {
            if (g.me == g.leader)
                __hip_atomic_store(share + k, kShareFree, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            prover = false;
        }
        if (r < S) {
            const uint32_t j = home + r < S ? home + r : home + r - S;
            const uint32_t before = need;
            if (chunk) chunk_serve<R>(h, g, j, need, served, stage, false, tl);
            else page_serve_shard<R>(h, g, q, j, need, served, false, false, tl);
            if (need < before) continue;
        }
        /* holds in flight, or the shard was drained under us: wait, bounded */
        if (g.me == g.leader) a_add64(shard_stats(h, home) + 1, 1);
        if (!wb.wait(h)) {
            timed_out = true;
            break;
        }
    }
    if (prover && need == 0 && g.me == g.leader)
        __hip_atomic_store(share + k, kShareFree, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (prover && timed_out && g.me == g.leader)
        __hip_atomic_store(share + k, kShareFree, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (need > 0 && g.me == g.leader) {
        if (timed_out) raise_err(h, HBHEAP_ERR_TIMEOUT, HBHEAP_STAT_TIMEOUTS);
        a_add64(shard_stats(h, home), need);
    }
    if (chunk) {
        wave_sync_lds();
#pragma unroll
        for (uint32_t r = 0; r < R; ++r)
            if (in_group(q, id, r)) q.off[r] = stage[q.rank[r]];
        wave_sync_lds();
    }
}

/* ---------------- wave entry points ---------------- */

/* Whether the home shard's pool has run dry.  A plain load: the bump only
 * grows until a (quiescent) trim, so a stale value can only make the pool
 * look less consumed, never dry when it is not.  With eager retirement the
 * ring's count also rises as frees retire chunks, so a stale reading can say
 * dry when it is not; that only makes the chunk path look at the queue before
 * reserving, and the scan over shards reads every count afresh.  Callers that
 * load their request sizes issue this first, so that both loads are in flight
 * together. */
__device__ __forceinline__ bool home_pool_dry(const hbheap_dev_t& h, uint32_t home)
{
    const uint64_t* hp = pool_block(h, home);
    if (eager(h)) return state_count(hp[0]) <= 0;
    return hp[0] >= ((const uint32_t*)hp)[2];
}

template <uint32_t R>
__device__ __forceinline__ void malloc_rows(const hbheap_dev_t& h, Rows<R>& q, const uint64_t (&n)[R],
                                            const bool (&has)[R], uint32_t home_in, bool dry_in,
                                            uint32_t* share = nullptr);

/* Rows served one after another, one request per lane each (row r a
 * compile-time index, so that q stays in registers). */
template <uint32_t R, uint32_t r>
__device__ __forceinline__ void malloc_rows_one_by_one(const hbheap_dev_t& h, Rows<R>& q, const uint64_t (&n)[R],
                                                       const bool (&has)[R], uint32_t home_in, bool dry_in,
                                                       uint32_t* share)
{
    if constexpr (r < R) {
        Rows<1> one;
        const uint64_t n1[1] = {n[r]};
        const bool h1[1] = {has[r]};
        malloc_rows<1>(h, one, n1, h1, home_in, dry_in, share);
        q.k[r] = one.k[0];
        q.gid[r] = 0;
        q.rank[r] = 0;
        q.off[r] = one.off[0];
        malloc_rows_one_by_one<R, r + 1>(h, q, n, has, home_in, dry_in, share);
    }
}

/* Every active lane calls this with R requests (n[r] bytes where has[r]);
 * requests are grouped by class (inside aligned segments of `width` lanes)
 * and each group is served by queue operations of one lane for the whole
 * group.  q.off receives the page offsets.  With R > 1 every lane of the
 * wave must be active and the block at most kRowsBlockWaves waves (the
 * batch kernels see to it); below width 16 the rows are served one after
 * another.  A chunk heap with eager retirement serves a group's rows
 * together, one queue entry per lane and pass. */
template <uint32_t R>
__device__ __forceinline__ void malloc_rows(const hbheap_dev_t& h, Rows<R>& q, const uint64_t (&n)[R],
                                            const bool (&has)[R], uint32_t home_in, bool dry_in,
                                            uint32_t* share)
{
    if constexpr (R > 1) {
        if (h.width < 16u) {
            malloc_rows_one_by_one<R, 0>(h, q, n, has, home_in, dry_in, share);
            return;
        }
    }
    /* the home shard and its hint act for the whole wave: take the first
     * active lane's (a caller whose lanes disagree would otherwise make the
     * leader reserve on one queue and its lanes take from another) */
    const uint32_t home = (uint32_t)__builtin_amdgcn_readfirstlane((int)home_in);
    const bool home_dry = __builtin_amdgcn_readfirstlane((int)dry_in) != 0;
    const uint32_t me = lane();
    const uint64_t act = exec_mask();
    const uint32_t arank = rank_in(act);
    uint64_t* stage = stage_for_wave<R>();
    Tally tl;
    if constexpr (R > 1) {
        /* Every request of a full wave in one class (a batch of one size,
         * aggregated over the whole wave): one group, ranked rows first,
         * with no grouping loop; lane 0 acts for it.  Its first pass takes
         * published entries on the home shard without a hold, as below. */
        if (!HBHEAP_VARIANT_LISTS_CHUNKS(h.variant) && h.width >= 64u && act == ~0ull) {
            const int32_t k0 = __builtin_amdgcn_readfirstlane(has[0] ? class_of(h, n[0]) : -1);
            bool same = k0 >= 0;
#pragma unroll
            for (uint32_t r = 0; r < R; ++r) same = same && has[r] && class_of(h, n[r]) == k0;
            if (__ballot(!same) == 0) {
                constexpr uint32_t tot = 64u * R;
#pragma unroll
                for (uint32_t r = 0; r < R; ++r) {
                    q.k[r] = k0;
                    q.gid[r] = 0;
                    q.rank[r] = 64u * r + me;
                    q.off[r] = kNoPage;
                }
                uint32_t got = 0, h0 = 0;
                if (me == 0) {
                    const Ring Q = ring_of(h, home, (uint32_t)k0);
                    got = ring_take_published(Q, tot, tl);
                    if (got) {
                        fuzz_point(22);
                        h0 = a_add32(Q.head, got);
                        tl.headtail += 1;
                    }
                }
                got = (uint32_t)__builtin_amdgcn_readfirstlane((int)got);
                h0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)h0);
                bool tk[R];
                uint32_t pos[R], kr[R], v[R];
#pragma unroll
                for (uint32_t r = 0; r < R; ++r) {
                    tk[r] = q.rank[r] < got;
                    pos[r] = h0 + q.rank[r];
                    kr[r] = (uint32_t)k0;
                }
                take_rows<R>(h, home, kr, tk, pos, v, tl);
                fuzz_point(23);
#pragma unroll
                for (uint32_t r = 0; r < R; ++r) page_took(h, home, 4u + (uint32_t)k0, v[r], q.off[r], tl);
                if (got < tot) alloc_group<R>(h, q, 0, (uint32_t)k0, tot, stage, home, home_dry, got, true, share, tl);
                tally_flush(h, tl);
                return;
            }
        }
    }
    /* groups: requests of one class (inside aligned segments of `width`
     * lanes), ranked rows first; the g-th active lane keeps group g's class
     * and size */
    bool pend[R];
#pragma unroll
    for (uint32_t r = 0; r < R; ++r) {
        q.k[r] = has[r] ? class_of(h, n[r]) : -1;
        q.gid[r] = 0;
        q.rank[r] = 0;
        q.off[r] = kNoPage;
        pend[r] = q.k[r] >= 0;
    }
    uint32_t ngroups = 0, my_k = 0, my_tot = 0;
    for (;;) {
        /* the first pending request, rows first */
        uint32_t kk = 0, first = 0;
        bool found = false;
#pragma unroll
        for (uint32_t r = 0; r < R; ++r) {
            const uint64_t m = __ballot(pend[r]);
            if (!found && m) {
                first = ctz64(m);
                kk = bcast((uint32_t)q.k[r], first);
                found = true;
            }
        }
        if (!found) break;
        const bool in_seg = h.width >= 64u || ((me ^ first) & ~(h.width - 1u)) == 0u;
        uint32_t base = 0;
#pragma unroll
        for (uint32_t r = 0; r < R; ++r) {
            const bool mine = pend[r] && q.k[r] == (int32_t)kk && in_seg;
            const uint64_t m = __ballot(mine);
            if (mine) {
                q.gid[r] = ngroups;
                q.rank[r] = base + rank_in(m);
                pend[r] = false;
            }
            base += (uint32_t)__popcll(m);
        }
        if (arank == ngroups) {
            my_k = kk;
            my_tot = base;
        }
        ++ngroups;
    }
    /* Page variants, several groups or rows: one first pass for all of them
     * at once on the home shard -- every group's agent lane reserves on its
     * own queue in the same instructions, the requests take their slots
     * together (every row's exchange in flight at once) and the bits are
     * cleared in one combined step per row -- instead of one group after
     * another.  It publishes nothing (no refill); groups left short continue
     * below, each on its own. */
    const bool fast = !HBHEAP_VARIANT_LISTS_CHUNKS(h.variant) && (ngroups > 1 || R > 1);
    uint32_t got = 0;
    if (fast) {
        uint32_t h0 = 0;
        if (arank < ngroups) {
            const Ring Q = ring_of(h, home, my_k);
            got = ring_take_published(Q, my_tot, tl);
            if (got) {
                h0 = a_add32(Q.head, got);
                tl.headtail += 1;
            }
        }
        bool tk[R];
        uint32_t pos[R], kr[R], v[R];
#pragma unroll
        for (uint32_t r = 0; r < R; ++r) {
            const uint32_t al = agent_lane(act, q.k[r] >= 0 ? q.gid[r] : 0u);
            const uint32_t gg = perm32(got, al), hh = perm32(h0, al);
            tk[r] = q.k[r] >= 0 && q.rank[r] < gg;
            pos[r] = hh + q.rank[r];
            kr[r] = q.k[r] >= 0 ? (uint32_t)q.k[r] : 0u;
        }
        take_rows<R>(h, home, kr, tk, pos, v, tl);
#pragma unroll
        for (uint32_t r = 0; r < R; ++r) page_took(h, home, 4u + kr[r], v[r], q.off[r], tl);
    }
    /* groups left short, one after another */
    for (uint32_t gi = 0; gi < ngroups; ++gi) {
        const uint32_t al = agent_lane(act, gi);
        const uint32_t kk = bcast(my_k, al), tot = bcast(my_tot, al);
        const uint32_t done = fast ? bcast(got, al) : 0u;
        if (done >= tot) continue;
        alloc_group<R>(h, q, gi, kk, tot, stage, home, home_dry, done, fast, share, tl);
    }
    tally_flush(h, tl);
}

/* One request per lane: every active lane calls this. */
__device__ __forceinline__ void* malloc_wave(const hbheap_dev_t& h, uint64_t n, uint32_t home_in, bool dry_in,
                                             uint32_t* share = nullptr)
{
    Rows<1> q;
    const uint64_t n1[1] = {n};
    const bool h1[1] = {true};
    malloc_rows<1>(h, q, n1, h1, home_in, dry_in, share);
    return q.off[0] == kNoPage ? nullptr : (void*)(h.data + q.off[0]);
}

/* Every active lane calls this with its pointer (NULL allowed).  size_hint:
 * when check_size, the request size the block was allocated with; a size of
 * another class makes the free invalid.  Returns kFree* status. */
__device__ __forceinline__ uint32_t free_wave(const hbheap_dev_t& h, void* p, uint64_t size_hint, bool check_size)
{
    const uint32_t me = lane();
    uint32_t status = kFreeNull;
    bool enq = false, cand = false;
    Tally tl;
    uint32_t val = 0, key = 0, k = 0, jv = 0;
    uint64_t c = 0, widx = 0, bit = 0, o = 0;
    bool inr = false;
    if (p != nullptr) {
        status = kFreeInvalid;
        o = (uint64_t)((uint8_t*)p - h.data);
        inr = (uint8_t*)p >= h.data && o < h.data_bytes;
        if (inr) c = o >> h.log2_chunk;
    }
    uint32_t kc = 0;
    if (eager(h)) kc = class_coherent(h, inr, c);
    if (p != nullptr) {
        if (inr) {
            k = eager(h) ? kc : h.chunk_class[c];
            const uint32_t shift = 4u + k;
            bool ok = k < h.n_classes && (o & ((1ull << shift) - 1ull)) == 0;
            if (ok && check_size) ok = class_of(h, size_hint) == (int)k;
            if (ok) {
                const uint32_t pg = (uint32_t)((o & ((1ull << h.log2_chunk) - 1ull)) >> shift);
                widx = bit_index(h, c, pg >> 6);
                bit = 1ull << (pg & 63u);
                jv = shard_of_chunk(h, c);
                key = jv * h.n_classes + k;
                cand = true;
            }
        }
    }
    /* Set the free bits.  Each run of adjacent lanes freeing pages of one
     * bitmask word sets its bits with one atomicOr by its last lane (the
     * run's bits are combined first, which also finds the same page twice in
     * one run); in the chunk variant that lane also raises the chunk's count
     * once by the number of newly set bits, and the run enqueues the chunk
     * once if the count left zero.  Pages of one word in separate runs are
     * set by separate atomics: the returned old word tells each run which of
     * its bits were already set. */
    const Run run = run_combine(cand, widx, bit, h.width < 64u ? h.width : 64u);
    uint64_t old = 0;
    uint32_t cold = 1, nnew = 0;
    bool retire = false;
    if (cand && me == run.tail) {
        old = a_or64(h.bits + widx, run.incl);
        nnew = (uint32_t)__popcll(run.incl & ~old);
        tl.spread += 1;
        if (eager(h) && nnew) {
            /* count and token in one word: a free that finds neither a token
             * nor a free page owns the chunk (it lists it below, cold = 0);
             * one that makes a listed chunk whole retires it, unless an
             * allocator takes it first */
            const uint32_t ppc = 1u << (h.log2_chunk - 4u - k);
            const uint64_t ow = a_add64(h.chunk_ct + c, nnew);
            const uint32_t otok = (uint32_t)(ow >> 32), n = ct_count(ow) + nnew, st = ct_stale(ow);
            tl.spread += 1;
            if (otok == kTokNone && ct_count(ow) == 0) {
                if (n >= ppc) {
                    /* whole at once, never listed: no stale entry left */
                    uint64_t x = ct_word(kTokNone, n | st);
                    retire = a_cas64(h.chunk_ct + c, x, ct_word(kTokNone, st));
                } else {
                    cold = 0;
                }
            } else if (otok < kTokHeld && n >= ppc && !(st & stale_bit(k))) {
                /* its entry becomes stale: only without one outstanding in
                 * its queue */
                uint64_t x = ct_word(otok, n | st);
                retire = a_cas64(h.chunk_ct + c, x, ct_word(kTokNone, st | stale_bit(k)));
            }
        } else if (HBHEAP_VARIANT_LISTS_CHUNKS(h.variant) && nnew) {
            cold = (uint32_t)a_addi(h.chunk_cnt + c, (int32_t)nnew);
            tl.spread += 1;
        }
    }
    fuzz_point(38);
    if (eager(h)) retire_wave(h, retire, (uint32_t)c, k, tl);
    old = perm64(old, run.tail);
    cold = perm32(cold, run.tail);
    nnew = perm32(nnew, run.tail);
    if (cand) {
        status = ((run.prior & bit) || (old & bit)) ? kFreeDouble : kFreeOk;
        if (HBHEAP_VARIANT_LISTS_CHUNKS(h.variant)) {
            /* the chunk's count left zero: the run enqueues it once */
            enq = me == run.tail && nnew > 0 && cold == 0;
            val = (uint32_t)c;
        } else {
            enq = status == kFreeOk;
            val = (uint32_t)(o >> 4);
        }
    }
    /* rare paths: one report per wave */
    const uint64_t dbl = __ballot(status == kFreeDouble), inv = __ballot(status == kFreeInvalid);
    if ((dbl | inv) && me == ctz64(exec_mask())) {
        if (dbl) { a_or32(h.err, HBHEAP_ERR_DOUBLE_FREE); a_add64(h.stats + HBHEAP_STAT_DOUBLE_FREE, (uint64_t)__popcll(dbl)); }
        if (inv) { a_or32(h.err, HBHEAP_ERR_INVALID_FREE); a_add64(h.stats + HBHEAP_STAT_INVALID_FREE, (uint64_t)__popcll(inv)); }
    }
    /* aggregated enqueue by (shard, class): one tail and one state add per
     * group.  Once a group of fewer than 4 lanes shows up (frees scattered
     * over many queues), the remaining lanes enqueue one entry each, all in
     * the same instructions, instead of one queue after another. */
    uint64_t pend = __ballot(enq);
    bool first_group = true;
    while (pend) {
        const uint32_t leader = ctz64(pend);
        const uint32_t kk = bcast(key, leader);
        uint64_t grp = __ballot(enq && key == kk) & pend;
        if (h.width < 64u) {
            const uint32_t seg = leader & ~(h.width - 1u);
            grp &= ((1ull << h.width) - 1ull) << seg;
        }
        if (!first_group && __popcll(grp) < 4) break;
        first_group = false;
        const uint32_t n = (uint32_t)__popcll(grp);
        const Ring R = ring_of(h, kk / h.n_classes, kk % h.n_classes);
        uint32_t t0 = 0;
        fuzz_point(39);
        if (me == leader) {
            t0 = a_add32(R.tail, n);
            tl.headtail += 1;
        }
        t0 = bcast(t0, leader);
        if ((grp >> me) & 1ull) {
            const uint32_t pos = t0 + rank_in(grp);
            if (eager(h)) list_or_retire(h, val, k, 1u << (h.log2_chunk - 4u - k), pos, 0u, tl);
            slot_put(h, R, pos, val, tl);
        }
        fuzz_point(40);
        if (me == leader) {
            a_add64(R.state, (uint64_t)n);
            tl.state += 1;
        }
        pend &= ~grp;
    }
    if ((pend >> me) & 1ull) {
        const Ring R = ring_of(h, jv, k);
        const uint32_t t0 = a_add32(R.tail, 1u);
        tl.headtail += 1;
        if (eager(h)) list_or_retire(h, val, k, 1u << (h.log2_chunk - 4u - k), t0, 0u, tl);
        slot_put(h, R, t0, val, tl);
        fuzz_point(41);
        a_add64(R.state, 1ull);
        tl.state += 1;
    }
    tally_flush(h, tl);
    return status;
}

/* Rows, per lane: the requests with pt[r] fill ring position pos[r] of
 * queue (shard jr[r], class kr[r]) with val[r].  Plain rings: every row's
 * compare-and-swap is issued before any is waited for; segmented rings: row
 * by row. */
template <uint32_t R>
__device__ __forceinline__ void put_rows(const hbheap_dev_t& h, const uint32_t (&jr)[R], const uint32_t (&kr)[R],
                                         const bool (&pt)[R], const uint32_t (&pos)[R], const uint32_t (&val)[R],
                                         Tally& tl)
{
    if (!HBHEAP_VARIANT_SEGMENTED(h.variant)) {
        /* was[r] is read only where the row swapped (see take_rows) */
        uint32_t was[R];
#pragma unroll
        for (uint32_t r = 0; r < R; ++r) {
            if (pt[r]) {
                was[r] = a_cas32_old(plain_slot(h, jr[r], kr[r], pos[r]), kEmpty, val[r]);
                tl.slot += 1;
            }
        }
#pragma unroll
        for (uint32_t r = 0; r < R; ++r)
            if (pt[r] && was[r] != kEmpty) plain_put_wait(h, plain_slot(h, jr[r], kr[r], pos[r]), val[r], tl);
        return;
    }
#pragma unroll
    for (uint32_t r = 0; r < R; ++r)
        if (pt[r]) slot_put(h, ring_of(h, jr[r], kr[r]), pos[r], val[r], tl);
}

/* R frees per lane (p[r], NULL allowed), for heaps without eager
 * retirement and with aggregation width 64 (others go row by row through
 * free_wave).  The same steps as free_wave, each taken for every row before
 * the next: runs of lanes on one bitmask word set their bits with one
 * atomicOr per row (all rows' in flight together), and the entries to
 * enqueue are grouped by (shard, class) over all rows, one tail add and one
 * state add per group.  status[r] receives kFree* status. */
template <uint32_t R>
__device__ __forceinline__ void free_rows(const hbheap_dev_t& h, void* const (&p)[R], const uint64_t (&size_hint)[R],
                                          bool check_size, uint32_t (&status)[R])
{
    if (R == 1 || eager(h) || h.width < 64u) {
#pragma unroll
        for (uint32_t r = 0; r < R; ++r) status[r] = free_wave(h, p[r], size_hint[r], check_size);
        return;
    }
    const uint32_t me = lane();
    Tally tl;
    bool cand[R], inr[R], enq[R];
    uint32_t key[R], k[R], val[R], pg[R];
    uint64_t c[R], widx[R], bit[R], o[R];
#pragma unroll
    for (uint32_t r = 0; r < R; ++r) {
        status[r] = kFreeNull;
        cand[r] = inr[r] = enq[r] = false;
        key[r] = k[r] = val[r] = pg[r] = 0;
        c[r] = widx[r] = bit[r] = o[r] = 0;
        if (p[r] != nullptr) {
            status[r] = kFreeInvalid;
            o[r] = (uint64_t)((const uint8_t*)p[r] - h.data);
            inr[r] = (const uint8_t*)p[r] >= h.data && o[r] < h.data_bytes;
            if (inr[r]) c[r] = o[r] >> h.log2_chunk;
        }
    }
    uint32_t kc[R];
#pragma unroll
    for (uint32_t r = 0; r < R; ++r) kc[r] = inr[r] ? h.chunk_class[c[r]] : 0u;
#pragma unroll
    for (uint32_t r = 0; r < R; ++r) {
        if (!inr[r]) continue;
        k[r] = kc[r];
        const uint32_t shift = 4u + k[r];
        bool ok = k[r] < h.n_classes && (o[r] & ((1ull << shift) - 1ull)) == 0;
        if (ok && check_size) ok = class_of(h, size_hint[r]) == (int)k[r];
        if (ok) {
            pg[r] = (uint32_t)((o[r] & ((1ull << h.log2_chunk) - 1ull)) >> shift);
            widx[r] = bit_index(h, c[r], pg[r] >> 6);
            bit[r] = 1ull << (pg[r] & 63u);
            key[r] = shard_of_chunk(h, c[r]) * h.n_classes + k[r];
            cand[r] = true;
        }
    }
    /* set the free bits: one atomicOr per run of lanes on one word, every
     * row's in flight together; chunk variant: then one count add per run */
    Run run[R];
    uint64_t old[R];
    uint32_t cold[R], nnew[R];
#pragma unroll
    for (uint32_t r = 0; r < R; ++r) {
        const uint32_t shift = cand[r] ? 4u + k[r] : h.log2_chunk;
        if (!run_consecutive(cand[r], o[r], shift, 1u << (h.log2_chunk - shift), pg[r], run[r]))
            run[r] = run_combine(cand[r], widx[r], bit[r], 64u);
    }
    /* (returned values are left unset on lanes that issue nothing, and
     * masked only after every row's atomic is issued, so that the rows'
     * atomics are in flight together) */
    bool tail[R];
#pragma unroll
    for (uint32_t r = 0; r < R; ++r) {
        tail[r] = cand[r] && me == run[r].tail;
        if (tail[r]) {
            old[r] = a_or64(h.bits + widx[r], run[r].incl);
            tl.spread += 1;
        }
    }
#pragma unroll
    for (uint32_t r = 0; r < R; ++r) {
        old[r] = tail[r] ? old[r] : 0ull;
        nnew[r] = tail[r] ? (uint32_t)__popcll(run[r].incl & ~old[r]) : 0u;
        if (HBHEAP_VARIANT_LISTS_CHUNKS(h.variant) && nnew[r]) {
            cold[r] = (uint32_t)a_addi(h.chunk_cnt + c[r], (int32_t)nnew[r]);
            tl.spread += 1;
        }
    }
#pragma unroll
    for (uint32_t r = 0; r < R; ++r) cold[r] = nnew[r] ? cold[r] : 1u;
    fuzz_point(42);
    uint32_t ndbl = 0, ninv = 0;
#pragma unroll
    for (uint32_t r = 0; r < R; ++r) {
        old[r] = perm64(old[r], run[r].tail);
        cold[r] = perm32(cold[r], run[r].tail);
        nnew[r] = perm32(nnew[r], run[r].tail);
        if (cand[r]) {
            status[r] = ((run[r].prior & bit[r]) || (old[r] & bit[r])) ? kFreeDouble : kFreeOk;
            if (HBHEAP_VARIANT_LISTS_CHUNKS(h.variant)) {
                /* the chunk's count left zero: the run enqueues it once */
                enq[r] = me == run[r].tail && nnew[r] > 0 && cold[r] == 0;
                val[r] = (uint32_t)c[r];
            } else {
                enq[r] = status[r] == kFreeOk;
                val[r] = (uint32_t)(o[r] >> 4);
            }
        }
        ndbl += (uint32_t)__popcll(__ballot(status[r] == kFreeDouble));
        ninv += (uint32_t)__popcll(__ballot(status[r] == kFreeInvalid));
    }
    /* rare paths: one report per wave */
    if ((ndbl | ninv) && me == ctz64(exec_mask())) {
        if (ndbl) { a_or32(h.err, HBHEAP_ERR_DOUBLE_FREE); a_add64(h.stats + HBHEAP_STAT_DOUBLE_FREE, ndbl); }
        if (ninv) { a_or32(h.err, HBHEAP_ERR_INVALID_FREE); a_add64(h.stats + HBHEAP_STAT_INVALID_FREE, ninv); }
    }
    /* aggregated enqueue by (shard, class) over all rows: one tail and one
     * state add per group, ranks rows first.  Once a group of fewer than 4
     * entries shows up (frees scattered over many queues), the remaining
     * entries are enqueued one by one, all in the same instructions. */
    uint32_t jr[R], kr[R];
#pragma unroll
    for (uint32_t r = 0; r < R; ++r) {
        jr[r] = cand[r] ? shard_of_chunk(h, c[r]) : 0u;
        kr[r] = cand[r] ? k[r] : 0u;
    }
    {
        /* every request of a full wave enqueues into one queue (frees of
         * one size from one shard): one group, ranked rows first, with no
         * grouping loop; lane 0 acts for it */
        const uint32_t k0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)key[0]);
        bool one = exec_mask() == ~0ull;
#pragma unroll
        for (uint32_t r = 0; r < R; ++r) one = one && enq[r] && key[r] == k0;
        if (__ballot(!one) == 0) {
            const uint32_t jj = (uint32_t)__builtin_amdgcn_readfirstlane((int)jr[0]);
            const uint32_t kc = (uint32_t)__builtin_amdgcn_readfirstlane((int)kr[0]);
            const Ring Q = ring_of(h, jj, kc);
            uint32_t t0 = 0;
            fuzz_point(43);
            if (me == 0) {
                t0 = a_add32(Q.tail, 64u * R);
                tl.headtail += 1;
            }
            t0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)t0);
            uint32_t ju[R], ku[R], pos[R];
#pragma unroll
            for (uint32_t r = 0; r < R; ++r) {
                ju[r] = jj;
                ku[r] = kc;
                pos[r] = t0 + 64u * r + me;
            }
            put_rows<R>(h, ju, ku, enq, pos, val, tl);
            fuzz_point(44);
            if (me == 0) {
                a_add64(Q.state, 64ull * R);
                tl.state += 1;
            }
            tally_flush(h, tl);
            return;
        }
    }
    bool first_group = true;
    for (;;) {
        uint32_t kk = 0, leader = 0, jj = 0, kc = 0;
        bool found = false;
#pragma unroll
        for (uint32_t r = 0; r < R; ++r) {
            const uint64_t m = __ballot(enq[r]);
            if (!found && m) {
                leader = ctz64(m);
                kk = bcast(key[r], leader);
                jj = bcast(jr[r], leader);
                kc = bcast(kr[r], leader);
                found = true;
            }
        }
        if (!found) break;
        bool mem[R];
        uint32_t pos[R], nn = 0;
#pragma unroll
        for (uint32_t r = 0; r < R; ++r) {
            mem[r] = enq[r] && key[r] == kk;
            const uint64_t m = __ballot(mem[r]);
            pos[r] = nn + rank_in(m);
            nn += (uint32_t)__popcll(m);
        }
        if (!first_group && nn < 4u) break;
        first_group = false;
        const Ring Q = ring_of(h, jj, kc);
        uint32_t t0 = 0;
        fuzz_point(43);
        if (me == leader) {
            t0 = a_add32(Q.tail, nn);
            tl.headtail += 1;
        }
        t0 = bcast(t0, leader);
#pragma unroll
        for (uint32_t r = 0; r < R; ++r) pos[r] += t0;
        put_rows<R>(h, jr, kr, mem, pos, val, tl);
        fuzz_point(44);
        if (me == leader) {
            a_add64(Q.state, (uint64_t)nn);
            tl.state += 1;
        }
#pragma unroll
        for (uint32_t r = 0; r < R; ++r) enq[r] = enq[r] && !mem[r];
    }
    /* the rest: one entry per request, each with its own tail and state add */
    if (HBHEAP_VARIANT_SEGMENTED(h.variant)) {
        /* row by row: a producer in a segmented ring may wait for whoever
         * installs its segment, which holds a lower position of the ring.
         * Positions taken and filled one row at a time keep every such wait
         * on a position reserved earlier -- this row's or another wave's --
         * never on a later row of this wave, which would not run before the
         * wait ends. */
#pragma unroll
        for (uint32_t r = 0; r < R; ++r) {
            if (enq[r]) {
                const Ring Q = ring_of(h, jr[r], kr[r]);
                const uint32_t t = a_add32(Q.tail, 1u);
                tl.headtail += 1;
                slot_put(h, Q, t, val[r], tl);
                a_add64(Q.state, 1ull);
                tl.state += 1;
            }
        }
        tally_flush(h, tl);
        return;
    }
    uint32_t pos[R];
#pragma unroll
    for (uint32_t r = 0; r < R; ++r) {
        pos[r] = 0;
        if (enq[r]) {
            pos[r] = a_add32(ring_of(h, jr[r], kr[r]).tail, 1u);
            tl.headtail += 1;
        }
    }
    put_rows<R>(h, jr, kr, enq, pos, val, tl);
    fuzz_point(45);
#pragma unroll
    for (uint32_t r = 0; r < R; ++r) {
        if (enq[r]) {
            a_add64(ring_of(h, jr[r], kr[r]).state, 1ull);
            tl.state += 1;
        }
    }
    tally_flush(h, tl);
}

}  // namespace detail
}  // namespace hbheap

/* Allocate n bytes from the heap; NULL when n == 0, n exceeds the chunk
 * size, or no page of the class and no chunk is left in any shard. */
__device__ __forceinline__ void* dev_malloc(hbheap_dev_t h, size_t n)
{
    const uint32_t home = hbheap::detail::home_shard(h);
    return hbheap::detail::malloc_wave(h, (uint64_t)n, home, hbheap::detail::home_pool_dry(h, home));
}

/* Return a block to the heap.  NULL is ignored; an invalid pointer or a
 * double free is ignored and recorded in the sticky error word. */
__device__ __forceinline__ void dev_free(hbheap_dev_t h, void* p)
{
    hbheap::detail::fence_release();
    (void)hbheap::detail::free_wave(h, p, 0, false);
}

#endif
