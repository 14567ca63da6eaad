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
 *     a request returns NULL only after it saw the pool exhausted, then the
 *     state with H == 0 and count <= 0 (exact out-of-memory).
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
 *     back to the pool only through heap_trim() at quiescence.
 *   - Every wait is bounded: past spin_cap iterations the wait gives up,
 *     sets HBHEAP_ERR_TIMEOUT and the request returns NULL.
 *   - Metadata atomics are agent-scope and relaxed; ordering comes from
 *     issuing a dependent atomic only after the previous one returned, plus
 *     one release fence before a refill publishes freshly written bitmasks.
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

/* ---------------- scoped atomics ---------------- */

#define HBH_A(order) order, __HIP_MEMORY_SCOPE_AGENT
__device__ __forceinline__ uint64_t a_add64(uint64_t* p, uint64_t v) { return __hip_atomic_fetch_add(p, v, HBH_A(__ATOMIC_RELAXED)); }
__device__ __forceinline__ uint32_t a_add32(uint32_t* p, uint32_t v) { return __hip_atomic_fetch_add(p, v, HBH_A(__ATOMIC_RELAXED)); }
__device__ __forceinline__ int32_t a_addi(int32_t* p, int32_t v) { return __hip_atomic_fetch_add(p, v, HBH_A(__ATOMIC_RELAXED)); }
__device__ __forceinline__ uint64_t a_or64(uint64_t* p, uint64_t v) { return __hip_atomic_fetch_or(p, v, HBH_A(__ATOMIC_RELAXED)); }
__device__ __forceinline__ uint64_t a_and64(uint64_t* p, uint64_t v) { return __hip_atomic_fetch_and(p, v, HBH_A(__ATOMIC_RELAXED)); }
__device__ __forceinline__ uint32_t a_or32(uint32_t* p, uint32_t v) { return __hip_atomic_fetch_or(p, v, HBH_A(__ATOMIC_RELAXED)); }
__device__ __forceinline__ uint32_t a_xchg32(uint32_t* p, uint32_t v) { return __hip_atomic_exchange(p, v, HBH_A(__ATOMIC_RELAXED)); }
__device__ __forceinline__ bool a_cas32(uint32_t* p, uint32_t expect, uint32_t v)
{
    return __hip_atomic_compare_exchange_strong(p, &expect, v, __ATOMIC_RELAXED, HBH_A(__ATOMIC_RELAXED));
}
__device__ __forceinline__ uint64_t a_load64(uint64_t* p) { return __hip_atomic_load(p, HBH_A(__ATOMIC_RELAXED)); }
__device__ __forceinline__ uint32_t a_load32(uint32_t* p) { return __hip_atomic_load(p, HBH_A(__ATOMIC_RELAXED)); }
__device__ __forceinline__ int32_t a_loadi(int32_t* p) { return __hip_atomic_load(p, HBH_A(__ATOMIC_RELAXED)); }
#undef HBH_A

__device__ __forceinline__ void fence_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
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

/* Atomics issued, by target, when HBHEAP_FLAG_STATS is set: class state
 * words, class head/tail words, the pool counter, and per-lane atomics on
 * slots, bitmasks and chunk counts. */
struct Tally {
    uint32_t state = 0, headtail = 0, pool = 0, spread = 0;
};

__device__ __forceinline__ void tally_flush(const hbheap_dev_t& h, const Tally& t)
{
    if (!(h.flags & HBHEAP_FLAG_STATS)) return;
    uint32_t s, ht, pl, sp;
    (void)excl_scan<20>(t.state, &s);
    (void)excl_scan<20>(t.headtail, &ht);
    (void)excl_scan<20>(t.pool, &pl);
    (void)excl_scan<20>(t.spread, &sp);
    if (lane() == ctz64(exec_mask())) {
        if (s) a_add64(h.stats + HBHEAP_STAT_STATE_OPS, s);
        if (ht) a_add64(h.stats + HBHEAP_STAT_HEADTAIL_OPS, ht);
        if (pl) a_add64(h.stats + HBHEAP_STAT_POOL_OPS, pl);
        if (sp) a_add64(h.stats + HBHEAP_STAT_SPREAD_OPS, sp);
    }
}

/* ---------------- geometry ---------------- */

__device__ __forceinline__ int class_of(const hbheap_dev_t& h, uint64_t n)
{
    if (n == 0 || n > (1ull << h.log2_chunk)) return -1;
    if (n <= 16) return 0;
    return 64 - __builtin_clzll(n - 1) - 4; /* ceil(log2 n) - 4 */
}

/* ---------------- class ring ---------------- */

struct Ring {
    uint64_t* state;
    uint32_t* head;
    uint32_t* tail;
    uint32_t* slots;
    uint32_t mask;
};

__device__ __forceinline__ Ring ring_of(const hbheap_dev_t& h, uint32_t k)
{
    uint8_t* cb = h.classes + (uint64_t)k * kClassBlock;
    Ring r;
    r.state = (uint64_t*)cb;
    r.head = (uint32_t*)(cb + 128);
    r.tail = (uint32_t*)(cb + 256);
    r.slots = h.slots + ((uint64_t)k << h.log2q);
    r.mask = (1u << h.log2q) - 1u;
    return r;
}
__device__ __forceinline__ uint64_t* owned_of(const hbheap_dev_t& h, uint32_t k)
{
    return (uint64_t*)(h.classes + (uint64_t)k * kClassBlock + 384);
}
__device__ __forceinline__ int32_t state_count(uint64_t s) { return (int32_t)((uint32_t)s - kBias); }

/* Leader only.  Takes a hold (H += 1) and reserves up to n published
 * entries; returns how many were reserved.  The hold is dropped by
 * ring_release(), which also publishes entries written meanwhile. */
__device__ __forceinline__ uint32_t ring_reserve(const Ring& r, uint32_t n, Tally& t)
{
    const uint64_t old = a_add64(r.state, kHold - n);
    const int32_t c = state_count(old);
    const uint32_t got = c <= 0 ? 0u : ((uint32_t)c < n ? (uint32_t)c : n);
    t.state += 1;
    if (got < n) {
        a_add64(r.state, (uint64_t)(n - got));
        t.state += 1;
    }
    return got;
}
__device__ __forceinline__ void ring_release(const Ring& r, uint32_t publish, Tally& t)
{
    a_add64(r.state, (uint64_t)publish - kHold);
    t.state += 1;
}

/* Per lane: take the entry of ring position pos (wait while its producer is
 * late).  kEmpty on timeout. */
__device__ __forceinline__ uint32_t slot_take(const hbheap_dev_t& h, const Ring& r, uint32_t pos, Tally& t)
{
    uint32_t* s = r.slots + (pos & r.mask);
    Backoff b;
    for (;;) {
        if (a_load32(s) != kEmpty) {
            const uint32_t v = a_xchg32(s, kEmpty);
            t.spread += 1;
            if (v != kEmpty) return v;
        }
        if (!b.wait(h)) {
            raise_err(h, HBHEAP_ERR_TIMEOUT, HBHEAP_STAT_TIMEOUTS);
            return kEmpty;
        }
    }
}

/* Per lane: fill ring position pos with v (wait while the slot still holds
 * the entry of the previous lap). */
__device__ __forceinline__ bool slot_put(const hbheap_dev_t& h, const Ring& r, uint32_t pos, uint32_t v, Tally& t)
{
    uint32_t* s = r.slots + (pos & r.mask);
    Backoff b;
    for (;;) {
        if (a_load32(s) == kEmpty) {
            t.spread += 1;
            if (a_cas32(s, kEmpty, v)) return true;
        }
        if (!b.wait(h)) {
            raise_err(h, HBHEAP_ERR_TIMEOUT, HBHEAP_STAT_TIMEOUTS);
            return false;
        }
    }
}

/* ---------------- pool ---------------- */

/* Leader only: take up to m unowned chunks; returns the first pool index in
 * *first and the number granted. */
__device__ __forceinline__ uint32_t pool_take(const hbheap_dev_t& h, uint32_t m, uint64_t* first, Tally& t)
{
    const uint64_t size = (uint32_t)h.pool[1];
    const uint64_t b = a_add64(h.pool, m);
    t.pool += 1;
    *first = b;
    if (b >= size) return 0;
    return (uint32_t)((size - b) < m ? (size - b) : m);
}
__device__ __forceinline__ bool pool_empty(const hbheap_dev_t& h)
{
    return a_load64(h.pool) >= (uint32_t)h.pool[1];
}

/* Page variant: a class may own at most (ring capacity / pages per chunk)
 * chunks, so its ring can always hold every free page it owns. */
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
    uint64_t* words = h.bits + (uint64_t)c * h.words_per_chunk;
    const uint64_t base = (uint64_t)c << h.log2_chunk;
    uint32_t got = 0;
    Backoff b;
    while (got < t) {
        for (uint32_t w = 0; w < nw && got < t; ++w) {
            uint64_t x = a_load64(&words[w]);
            while (x && got < t) {
                const uint64_t pick = lowest_bits(x, t - got);
                const uint64_t old = a_and64(&words[w], ~pick);
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

/* LDS staging: 64 page offsets per wave, for up to 16 waves per block. */
static __shared__ uint64_t hbheap_stage_lds[kMaxWavesPerBlock * 64];

__device__ __forceinline__ uint64_t* stage_for_wave()
{
    const uint32_t lin = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    return hbheap_stage_lds + (lin >> 6) * 64u;
}

/* Out-of-memory decision, leader only, after this group saw the pool (or
 * the class cap) exhausted: wait until no operation holds the class queue,
 * then retry if entries were published, else report out of memory.  For the
 * page variant the cap and pool are read again once nothing is in flight. */
__device__ __forceinline__ bool oom_should_retry(const hbheap_dev_t& h, const Ring& R, uint32_t k, Backoff& b)
{
    a_add64(h.stats + HBHEAP_STAT_OOM_WAITS, 1);
    /* every decision spends from the same budget, so retries are bounded */
    if (!b.wait(h)) {
        raise_err(h, HBHEAP_ERR_TIMEOUT, HBHEAP_STAT_TIMEOUTS);
        return false;
    }
    for (;;) {
        const uint64_t s = a_load64(R.state);
        if (state_count(s) > 0) return true;
        if ((s >> 32) == 0) {
            if (h.variant == HBHEAP_VARIANT_PAGE)
                return !pool_empty(h) && a_load64(owned_of(h, k)) < page_max_chunks(h, h.log2_chunk - 4u - k);
            return false;
        }
        if (!b.wait(h)) {
            raise_err(h, HBHEAP_ERR_TIMEOUT, HBHEAP_STAT_TIMEOUTS);
            return false;
        }
    }
}

/* ---------------- chunk variant: serve one class group ---------------- */

__device__ __forceinline__ uint64_t alloc_group_chunk(const hbheap_dev_t& h, uint32_t k, uint64_t grp, uint64_t* stage,
                                                      Tally& tl)
{
    const uint64_t act = exec_mask();
    const uint32_t me = lane();
    const uint32_t leader = ctz64(act);
    const uint32_t nact = (uint32_t)__popcll(act);
    const uint32_t arank = rank_in(act);
    const bool req = (grp >> me) & 1ull;
    const uint32_t qrank = rank_in(grp);
    const uint32_t shift = 4u + k;
    const uint32_t lppc = h.log2_chunk - shift;
    const uint32_t ppc = 1u << lppc;
    const Ring R = ring_of(h, k);

    stage[arank] = kNoPage;
    wave_sync_lds();

    uint32_t need = (uint32_t)__popcll(grp), served = 0;
    Backoff oom;
    while (need > 0) {
        const uint32_t want0 = (need + ppc - 1u) >> lppc;
        const uint32_t want = want0 < nact ? want0 : nact;
        uint32_t got = 0, h0 = 0;
        if (me == leader) {
            got = ring_reserve(R, want, tl);
            if (got) {
                h0 = a_add32(R.head, got);
                tl.headtail += 1;
            }
        }
        got = bcast(got, leader);
        h0 = bcast(h0, leader);

        /* helpers take one chunk each and read its free count */
        const bool helper = arank < got;
        uint32_t c = kEmpty;
        int32_t v = 0;
        if (helper) {
            c = slot_take(h, R, h0 + arank, tl);
            if (c != kEmpty && c >= h.n_chunks) {
                raise_err(h, HBHEAP_ERR_CORRUPT, HBHEAP_STAT_TIMEOUTS);
                c = kEmpty;
            }
            if (c != kEmpty) {
                v = a_loadi(h.chunk_cnt + c);
                if (v <= 0) raise_err(h, HBHEAP_ERR_CORRUPT, HBHEAP_STAT_TIMEOUTS);
            }
        }
        const uint32_t vc = v > 0 ? ((uint32_t)v < need ? (uint32_t)v : need) : 0u;
        uint32_t tot;
        const uint32_t pre = excl_scan<7>(vc, &tot);
        const uint32_t t = pre < need ? ((need - pre) < vc ? (need - pre) : vc) : 0u;

        bool keep = false;
        if (vc > 0) {
            if (t) {
                keep = a_addi(h.chunk_cnt + c, -(int32_t)t) - (int32_t)t > 0;
                tl.spread += 1;
            }
            else keep = true;
        }
        uint32_t took;
        const uint32_t tpre = excl_scan<7>(t, &took);
        if (t) claim_pages(h, c, k, t, stage + served + tpre, tl);

        /* chunks that still hold free pages go back to the tail */
        const uint64_t rq = __ballot(keep);
        const uint32_t nrq = (uint32_t)__popcll(rq);
        uint32_t t0 = 0;
        if (nrq && me == leader) {
            t0 = a_add32(R.tail, nrq);
            tl.headtail += 1;
        }
        t0 = bcast(t0, leader);
        if (keep) slot_put(h, R, t0 + rank_in(rq), c, tl);
        need -= took;
        served += took;

        uint32_t publish = nrq;
        bool exhausted = false;
        if (got < want && need > 0) {
            /* refill from the pool while still holding the queue */
            const uint32_t m = (need + ppc - 1u) >> lppc;
            uint64_t first = 0;
            uint32_t gm = 0;
            if (me == leader) {
                gm = pool_take(h, m, &first, tl);
                count_refill(h, gm);
            }
            gm = bcast(gm, leader);
            first = bcast64(first, leader);
            exhausted = gm < m;
            if (arank < gm) h.chunk_class[h.pool_ids[first + arank]] = (uint8_t)k;
            const uint32_t cap = gm << lppc;
            const uint32_t r = cap < need ? cap : need;
            if (arank < r) {
                const uint32_t ci = h.pool_ids[first + (arank >> lppc)];
                stage[served + arank] = ((uint64_t)ci << h.log2_chunk) + ((uint64_t)(arank & (ppc - 1u)) << shift);
            }
            if (cap > need) {
                /* last chunk keeps pages [u, ppc): set their bits, publish it */
                const uint32_t last = gm - 1u;
                const uint32_t u = need - (last << lppc);
                const uint32_t cl = h.pool_ids[first + last];
                const uint32_t nw = ppc >= 64u ? ppc >> 6 : 1u;
                for (uint32_t w = arank; w < nw; w += nact)
                    h.bits[(uint64_t)cl * h.words_per_chunk + w] = free_mask_word(w, u, ppc);
                if (me == leader) h.chunk_cnt[cl] = (int32_t)(ppc - u);
                fence_release();
                if (me == leader) {
                    const uint32_t pos = a_add32(R.tail, 1u);
                    tl.headtail += 1;
                    slot_put(h, R, pos, cl, tl);
                }
                publish += 1u;
            }
            need -= r;
            served += r;
        }
        if (me == leader) ring_release(R, publish, tl);
        if (need > 0 && exhausted) {
            bool retry = false;
            if (me == leader) retry = oom_should_retry(h, R, k, oom);
            if (!bcast((uint32_t)retry, leader)) break;
        }
        /* entries reserved but nothing served: a wait gave up (error raised) */
        if (got > 0 && took == 0) break;
    }
    if (need > 0 && me == leader) a_add64(h.stats + HBHEAP_STAT_OOM, need);
    wave_sync_lds();
    return req ? stage[qrank] : kNoPage;
}

/* ---------------- page variant: serve one class group ---------------- */

__device__ __forceinline__ uint64_t alloc_group_page(const hbheap_dev_t& h, uint32_t k, uint64_t grp, Tally& tl)
{
    const uint64_t act = exec_mask();
    const uint32_t me = lane();
    const uint32_t leader = ctz64(act);
    const uint32_t nact = (uint32_t)__popcll(act);
    const uint32_t arank = rank_in(act);
    const bool req = (grp >> me) & 1ull;
    const uint32_t qrank = rank_in(grp);
    const uint32_t shift = 4u + k;
    const uint32_t lppc = h.log2_chunk - shift;
    const uint32_t ppc = 1u << lppc;
    const Ring R = ring_of(h, k);

    uint64_t off = kNoPage;
    uint32_t need = (uint32_t)__popcll(grp), served = 0;
    Backoff oom;
    while (need > 0) {
        uint32_t got = 0, h0 = 0;
        if (me == leader) {
            got = ring_reserve(R, need, tl);
            if (got) {
                h0 = a_add32(R.head, got);
                tl.headtail += 1;
            }
        }
        got = bcast(got, leader);
        h0 = bcast(h0, leader);
        if (req && qrank >= served && qrank < served + got) {
            const uint32_t v = slot_take(h, R, h0 + (qrank - served), tl);
            if (v != kEmpty && ((uint64_t)v << 4) >= h.data_bytes) raise_err(h, HBHEAP_ERR_CORRUPT, HBHEAP_STAT_TIMEOUTS);
            else if (v != kEmpty) {
                const uint64_t o = (uint64_t)v << 4;
                const uint64_t c = o >> h.log2_chunk;
                const uint32_t p = (uint32_t)((o & ((1ull << h.log2_chunk) - 1ull)) >> shift);
                const uint64_t bit = 1ull << (p & 63u);
                const uint64_t old = a_and64(h.bits + c * h.words_per_chunk + (p >> 6), ~bit);
                tl.spread += 1;
                if (old & bit) off = o;
                else raise_err(h, HBHEAP_ERR_CORRUPT, HBHEAP_STAT_TIMEOUTS);
            }
        }
        need -= got;
        served += got;

        uint32_t publish = 0;
        bool exhausted = false;
        if (need > 0) {
            const uint32_t m = (need + ppc - 1u) >> lppc;
            uint64_t first = 0;
            uint32_t gm = 0;
            if (me == leader) {
                uint64_t* owned = owned_of(h, k);
                const uint64_t maxc = page_max_chunks(h, lppc);
                const uint64_t o = a_add64(owned, m);
                const uint32_t allow = o >= maxc ? 0u : (uint32_t)((maxc - o) < m ? (maxc - o) : m);
                gm = allow ? pool_take(h, allow, &first, tl) : 0u;
                tl.pool += 1;
                if (gm < m) {
                    a_add64(owned, (uint64_t)0 - (uint64_t)(m - gm));
                    tl.pool += 1;
                }
                count_refill(h, gm);
            }
            gm = bcast(gm, leader);
            first = bcast64(first, leader);
            exhausted = gm < m;
            if (arank < gm) h.chunk_class[h.pool_ids[first + arank]] = (uint8_t)k;
            const uint32_t cap = gm << lppc;
            const uint32_t r = cap < need ? cap : need;
            if (req && qrank >= served && qrank < served + r) {
                const uint32_t q = qrank - served;
                const uint32_t ci = h.pool_ids[first + (q >> lppc)];
                off = ((uint64_t)ci << h.log2_chunk) + ((uint64_t)(q & (ppc - 1u)) << shift);
            }
            if (cap > need) {
                const uint32_t last = gm - 1u;
                const uint32_t u = need - (last << lppc);
                const uint32_t cl = h.pool_ids[first + last];
                const uint32_t nw = ppc >= 64u ? ppc >> 6 : 1u;
                for (uint32_t w = arank; w < nw; w += nact)
                    h.bits[(uint64_t)cl * h.words_per_chunk + w] = free_mask_word(w, u, ppc);
                fence_release();
                const uint32_t L = ppc - u;
                uint32_t t0 = 0;
                if (me == leader) {
                    t0 = a_add32(R.tail, L);
                    tl.headtail += 1;
                }
                t0 = bcast(t0, leader);
                const uint64_t cbase = (uint64_t)cl << h.log2_chunk;
                for (uint32_t j = arank; j < L; j += nact)
                    slot_put(h, R, t0 + j, (uint32_t)((cbase + ((uint64_t)(u + j) << shift)) >> 4), tl);
                publish = L;
            }
            need -= r;
            served += r;
        }
        if (me == leader) ring_release(R, publish, tl);
        if (need > 0 && exhausted) {
            bool retry = false;
            if (me == leader) retry = oom_should_retry(h, R, k, oom);
            if (!bcast((uint32_t)retry, leader)) break;
        }
    }
    if (need > 0 && me == leader) a_add64(h.stats + HBHEAP_STAT_OOM, need);
    return req ? off : kNoPage;
}

/* ---------------- wave entry points ---------------- */

/* Every active lane calls this; lanes are grouped by class (restricted to
 * aligned segments of `width` lanes) and each group is served by one queue
 * operation of its leader. */
__device__ __forceinline__ void* malloc_wave(const hbheap_dev_t& h, uint64_t n)
{
    const int k = class_of(h, n);
    const uint32_t me = lane();
    uint64_t pending = __ballot(k >= 0);
    uint64_t* stage = stage_for_wave();
    uint64_t off = kNoPage;
    Tally tl;
    while (pending) {
        const uint32_t leader = ctz64(pending);
        const uint32_t kk = bcast((uint32_t)k, leader);
        uint64_t grp = __ballot(k == (int)kk) & pending;
        if (h.width < 64u) {
            const uint32_t seg = leader & ~(h.width - 1u);
            grp &= ((1ull << h.width) - 1ull) << seg;
        }
        const uint64_t o = h.variant == HBHEAP_VARIANT_CHUNK ? alloc_group_chunk(h, kk, grp, stage, tl)
                                                              : alloc_group_page(h, kk, grp, tl);
        if ((grp >> me) & 1ull) off = o;
        pending &= ~grp;
    }
    tally_flush(h, tl);
    return off == kNoPage ? nullptr : (void*)(h.data + off);
}

/* Every active lane calls this with its pointer (NULL allowed).  size_hint:
 * when check_size, the request size the block was allocated with; a size of
 * another class makes the free invalid.  Returns kFree* status. */
__device__ __forceinline__ uint32_t free_wave(const hbheap_dev_t& h, void* p, uint64_t size_hint, bool check_size)
{
    const uint32_t me = lane();
    uint32_t status = kFreeNull;
    bool enq = false;
    Tally tl;
    uint32_t val = 0, k = 0;
    if (p != nullptr) {
        status = kFreeInvalid;
        const uint64_t o = (uint64_t)((uint8_t*)p - h.data);
        if ((uint8_t*)p >= h.data && o < h.data_bytes) {
            const uint64_t c = o >> h.log2_chunk;
            k = h.chunk_class[c];
            const uint32_t shift = 4u + k;
            bool ok = k < h.n_classes && (o & ((1ull << shift) - 1ull)) == 0;
            if (ok && check_size) ok = class_of(h, size_hint) == (int)k;
            if (ok) {
                const uint32_t pg = (uint32_t)((o & ((1ull << h.log2_chunk) - 1ull)) >> shift);
                const uint64_t bit = 1ull << (pg & 63u);
                const uint64_t old = a_or64(h.bits + c * h.words_per_chunk + (pg >> 6), bit);
                tl.spread += 1;
                if (old & bit) {
                    status = kFreeDouble;
                } else {
                    status = kFreeOk;
                    if (h.variant == HBHEAP_VARIANT_CHUNK) {
                        enq = a_addi(h.chunk_cnt + c, 1) == 0;
                        tl.spread += 1;
                        val = (uint32_t)c;
                    } else {
                        enq = true;
                        val = (uint32_t)(o >> 4);
                    }
                }
            }
        }
    }
    /* rare paths: one report per wave */
    const uint64_t dbl = __ballot(status == kFreeDouble), inv = __ballot(status == kFreeInvalid);
    if ((dbl | inv) && me == ctz64(exec_mask())) {
        if (dbl) { a_or32(h.err, HBHEAP_ERR_DOUBLE_FREE); a_add64(h.stats + HBHEAP_STAT_DOUBLE_FREE, (uint64_t)__popcll(dbl)); }
        if (inv) { a_or32(h.err, HBHEAP_ERR_INVALID_FREE); a_add64(h.stats + HBHEAP_STAT_INVALID_FREE, (uint64_t)__popcll(inv)); }
    }
    /* aggregated enqueue by class */
    uint64_t pend = __ballot(enq);
    while (pend) {
        const uint32_t leader = ctz64(pend);
        const uint32_t kk = bcast(k, leader);
        uint64_t grp = __ballot(enq && k == kk) & pend;
        if (h.width < 64u) {
            const uint32_t seg = leader & ~(h.width - 1u);
            grp &= ((1ull << h.width) - 1ull) << seg;
        }
        const uint32_t n = (uint32_t)__popcll(grp);
        const Ring R = ring_of(h, kk);
        uint32_t t0 = 0;
        if (me == leader) {
            t0 = a_add32(R.tail, n);
            tl.headtail += 1;
        }
        t0 = bcast(t0, leader);
        if ((grp >> me) & 1ull) slot_put(h, R, t0 + rank_in(grp), val, tl);
        if (me == leader) {
            a_add64(R.state, (uint64_t)n);
            tl.state += 1;
        }
        pend &= ~grp;
    }
    tally_flush(h, tl);
    return status;
}

}  // namespace detail
}  // namespace hbheap

/* Allocate n bytes from the heap; NULL when n == 0, n exceeds the chunk
 * size, or no page of the class and no chunk is left. */
__device__ __forceinline__ void* dev_malloc(hbheap_dev_t h, size_t n)
{
    return hbheap::detail::malloc_wave(h, (uint64_t)n);
}

/* Return a block to the heap.  NULL is ignored; an invalid pointer or a
 * double free is ignored and recorded in the sticky error word. */
__device__ __forceinline__ void dev_free(hbheap_dev_t h, void* p)
{
    hbheap::detail::fence_release();
    (void)hbheap::detail::free_wave(h, p, 0, false);
}

#endif
