/*
 * hbheap_types.h -- plain-C types shared by the host C ABI (hbheap.h) and
 * the device API (hbheap_device.h).
 *
 * The heap follows the paper's statement of the problem (Introduction): the
 * host preallocates one block of device memory that acts as the heap, and a
 * heap algorithm running on the device serves allocation requests from
 * threads of running kernels.  The block is cut into chunks of one fixed
 * size C, and a chunk handed to a size class is split into pages of that
 * class (Results, "Page allocator" and "Chunk allocator").
 */
#ifndef HBHEAP_TYPES_H
#define HBHEAP_TYPES_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Queue variants (Results): "chunk" queues list chunks that have free
 * pages; "page" queues list free pages; the "virtualised array" variants
 * keep the same queues in storage taken on demand, segment by segment, from
 * a store the class queues of a shard share ("Virtualised array and list
 * allocators"). */
#define HBHEAP_VARIANT_CHUNK    0u
#define HBHEAP_VARIANT_PAGE     1u
#define HBHEAP_VARIANT_VA_PAGE  2u
#define HBHEAP_VARIANT_VA_CHUNK 3u
#define HBHEAP_VARIANT_VL_PAGE  4u
#define HBHEAP_VARIANT_VL_CHUNK 5u

/* Virtualised array variants: a queue finds its segments in a directory. */
#define HBHEAP_VARIANT_IS_VA(v) ((v) == HBHEAP_VARIANT_VA_PAGE || (v) == HBHEAP_VARIANT_VA_CHUNK)
/* Virtualised list variants: a queue's segments form a linked list. */
#define HBHEAP_VARIANT_IS_VL(v) ((v) == HBHEAP_VARIANT_VL_PAGE || (v) == HBHEAP_VARIANT_VL_CHUNK)
/* Queues in segmented storage drawn from a per-shard store. */
#define HBHEAP_VARIANT_SEGMENTED(v) (HBHEAP_VARIANT_IS_VA(v) || HBHEAP_VARIANT_IS_VL(v))
/* Queues of chunk ids (a chunk is listed while it has free pages), as
 * opposed to queues of free pages. */
#define HBHEAP_VARIANT_LISTS_CHUNKS(v) \
    ((v) == HBHEAP_VARIANT_CHUNK || (v) == HBHEAP_VARIANT_VA_CHUNK || (v) == HBHEAP_VARIANT_VL_CHUNK)
/* Page queues in segmented storage: a shard's classes share one page budget. */
#define HBHEAP_VARIANT_SHARED_PAGES(v) ((v) == HBHEAP_VARIANT_VA_PAGE || (v) == HBHEAP_VARIANT_VL_PAGE)

/* Return codes of every host entry point. */
#define HBHEAP_OK          0
#define HBHEAP_E_INVAL    -1   /* bad argument                              */
#define HBHEAP_E_NOMEM    -2   /* device memory for the heap not available  */
#define HBHEAP_E_HIP      -3   /* a HIP runtime call failed                 */
#define HBHEAP_E_RANGE    -4   /* buffer too small for the requested data   */
#define HBHEAP_E_UNSUP    -5   /* feature not available on this device      */

/* Bits of the sticky device error word (heap_get_error). */
#define HBHEAP_ERR_DOUBLE_FREE  0x1u  /* a page freed while already free     */
#define HBHEAP_ERR_INVALID_FREE 0x2u  /* pointer outside the heap, misaligned
                                         for its class, in an unowned chunk,
                                         or with a size of another class     */
#define HBHEAP_ERR_TIMEOUT      0x4u  /* a bounded wait gave up: the heap is
                                         inconsistent and must be destroyed  */
#define HBHEAP_ERR_CORRUPT      0x8u  /* a queue entry contradicted the
                                         bitmasks: the heap is inconsistent  */

/* Indices of the device statistics counters (heap_stats). */
#define HBHEAP_STAT_CHUNK_GRABS   0   /* chunks taken from the pool (FLAG_STATS) */
#define HBHEAP_STAT_REFILLS       1   /* refills of a class queue (FLAG_STATS)   */
#define HBHEAP_STAT_OOM           2   /* requests that returned NULL on OOM  */
#define HBHEAP_STAT_OOM_WAITS     3   /* OOM checks that had to wait         */
#define HBHEAP_STAT_DOUBLE_FREE   4
#define HBHEAP_STAT_INVALID_FREE  5
#define HBHEAP_STAT_TIMEOUTS      6
/* atomics issued, by target (FLAG_STATS): class state words, class head and
 * tail words, the pool counters, per-lane bitmask/count atomics (spread);
 * per-lane ring slot atomics are counted apart (SLOT_OPS) */
#define HBHEAP_STAT_STATE_OPS     8
#define HBHEAP_STAT_HEADTAIL_OPS  9
#define HBHEAP_STAT_POOL_OPS      10
#define HBHEAP_STAT_SPREAD_OPS    11
#define HBHEAP_STAT_RETIRED       12  /* chunks retired eagerly (FLAG_STATS)     */
#define HBHEAP_STAT_SLOT_OPS      13  /* per-lane ring slot atomics (FLAG_STATS) */
#define HBHEAP_STAT_COUNT         16

/*
 * Device handle: plain data passed by value as a kernel argument.  All
 * pointers are device pointers into memory the library owns.  Obtain it with
 * heap_device_handle(); it stays valid until heap_destroy().
 */
typedef struct hbheap_dev {
    uint8_t*  data;            /* data region: n_chunks * 2^log2_chunk bytes  */
    uint8_t*  state;           /* state region (snapshot layout, version 4)  */
    uint64_t* pool;            /* n_shards pool blocks of 128 bytes: u64 bump,
                                  u32 size, u32 first index into pool_ids    */
    uint8_t*  classes;         /* n_shards * n_classes blocks of 512 bytes   */
    uint8_t*  chunk_class;     /* class of each chunk, 0xFF when unowned     */
    int32_t*  chunk_cnt;       /* free pages per chunk (chunk variant)       */
    uint64_t* bits;            /* words_per_chunk words per chunk, 1 = free;
                                  word-major: word w of chunk c at
                                  w * n_chunks + c                           */
    uint32_t* pool_ids;        /* ids of unowned chunks, consumed by bump    */
    uint32_t* slots;           /* n_shards * n_classes rings of 2^log2q u32  */
    uint32_t* err;             /* sticky error word                          */
    uint64_t* stats;           /* HBHEAP_STAT_COUNT counters                 */
    uint64_t  data_bytes;
    uint32_t  n_chunks;
    uint32_t  log2_chunk;
    uint32_t  n_classes;       /* log2_chunk - 3: pages 16 B .. chunk        */
    uint32_t  variant;
    uint32_t  words_per_chunk; /* chunk / 1024                               */
    uint32_t  log2q;           /* capacity of each (shard, class) ring, log2 */
    uint32_t  width;           /* aggregation width: 1, 16, 32 or 64 lanes   */
    uint32_t  spin_cap;        /* bounded-wait iterations before TIMEOUT     */
    uint32_t  backoff_max;     /* largest s_sleep backoff, in s_sleep(1)s    */
    uint32_t  flags;           /* HBHEAP_FLAG_* bits                         */
    uint32_t  n_shards;        /* shards; shard j owns chunks
                                  [j << log2_span, (j+1) << log2_span)       */
    uint32_t  log2_span;
    /* segmented variants (all zero / NULL otherwise): the slot region
     * holds, per shard, vsegs segments of 2^log2_seg slots; free segment ids
     * wait in the shard's store, a ring of 2^log2_store u32 with its own
     * state/head/tail block (512 B; u64 pages the shard's classes own @384).
     * Virtualised array: a class queue finds the segment of ring position p
     * in its directory entry (p >> log2_seg) mod 2^log2_dir, a u64 (segment
     * number << 32 | segment id), all ones when empty.  Virtualised list:
     * vdir holds, per segment, a u64 tag (queue index << 32 | segment
     * number) and then, for all segments, a u64 link to the next segment id
     * (all ones for none); each queue's class block keeps front and back
     * words (segment number << 32 | id) at +392 and +400. */
    uint64_t* vdir;            /* directories, or tags then links            */
    uint32_t* vtaken;          /* per segment: slots consumed so far          */
    uint8_t*  vstore;          /* n_shards store blocks of 512 bytes          */
    uint32_t* vstore_slots;    /* n_shards rings of 2^log2_store u32          */
    uint32_t  log2_seg;
    uint32_t  log2_dir;
    uint32_t  log2_store;
    uint32_t  vsegs;           /* segments per shard                         */
    uint64_t  vbudget;         /* pages the classes of one shard may own     */
    /* eager retirement (chunk variant created with HBHEAP_FLAG_EAGER; NULL
     * otherwise): per chunk a u64.  Low half: free pages in bits 0..15, and
     * in bit 16 + k whether the chunk has a stale entry in the queue of
     * class k.  High half: where the chunk is listed: (class << 28 | queue
     * position mod 2^28), held by an allocator (0xFFFFFFFE) or nowhere
     * (0xFFFFFFFF).
     * Each shard's pool is then a ring: u64 state (free chunks + 2^31) at
     * +0, u32 head at +16, u32 tail at +20 of its pool block, and slots
     * pool_ids[(j << log2_span) + (position mod 2^log2_span)]. */
    uint64_t* chunk_ct;
} hbheap_dev_t;

/* Count refills, chunk grabs and atomics by target in the statistics
 * counters (extra atomics: for measurement runs only; errors and
 * out-of-memory are always counted). */
#define HBHEAP_FLAG_STATS 0x1u
/* Page variant: check that every page taken from a queue still had its
 * free bit set, raising HBHEAP_ERR_CORRUPT otherwise (the allocation then
 * waits for the bit-clearing atomic to return; without the flag it does
 * not). */
#define HBHEAP_FLAG_VERIFY 0x2u
/* Every wave starts at shard 0 instead of a shard of its XCD (used by the
 * single-lane replay, whose outcome is then deterministic). */
#define HBHEAP_FLAG_HOME0 0x4u
/* Chunk variant, fixed at creation (heap_create_ex): a chunk whose pages
 * are all free again leaves its class at once and returns to its shard's
 * pool, where any class can take it, instead of waiting for a trim. */
#define HBHEAP_FLAG_EAGER 0x8u

#ifdef __cplusplus
}
#endif
#endif
