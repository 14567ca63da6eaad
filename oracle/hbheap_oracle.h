/*
 * hbheap_oracle.h -- CPU oracle for the device heap allocator.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library,
 * its Python binding, the timed part of the benchmark) may include, link or
 * call this code; only the tests, the smoke check and the benchmark's CPU
 * baseline leg do.  It shares no code, header, table or constant generator
 * with the HIP path: every definition below is written out again here from
 * the paper and from the documented snapshot format.
 *
 * What the paper fixes (Standish, "Dynamic Memory Management on GPUs with
 * SYCL"):
 *   - Introduction: the host preallocates a block that acts as the heap and
 *     a heap algorithm runs on the device; the block is divided into chunks,
 *     each served through a lock-free queue dedicated to one size.
 *   - Results, "Page allocator": pages of one fixed size per queue; the heap
 *     is divided among the queues.
 *   - Results, "Chunk allocator": queues hold chunks that have free pages;
 *     an allocation first obtains a chunk index, then scans the chunk for a
 *     free page.  Queues are per power-of-two size.
 * Where the paper is silent this file takes these readings: smallest page
 * 16 B, one fixed chunk size, ceil-to-power-of-two rounding, NULL for 0 or
 * > chunk, metadata outside the heap bytes, a page-variant queue budget of
 * bytes/8, and a heap split into shards (runs of chunks with their own pool
 * and queues) where a request is served from any shard that can.
 *
 * Offsets, not pointers: a block is reported as its byte offset from the
 * start of the heap's data region; -1 stands for NULL.
 */
#ifndef HBHEAP_ORACLE_H
#define HBHEAP_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_CLASSES 16

enum {
    ORC_VARIANT_CHUNK = 0, ORC_VARIANT_PAGE = 1, ORC_VARIANT_VA_PAGE = 2, ORC_VARIANT_VA_CHUNK = 3,
    ORC_VARIANT_VL_PAGE = 4, ORC_VARIANT_VL_CHUNK = 5
};
/* LOWEST: canonical legal outcome (lowest chunk id, then lowest page).
 * FIFO:   the order a single device thread observes (queue order). */
enum { ORC_POLICY_LOWEST = 0, ORC_POLICY_FIFO = 1 };
enum { ORC_FREE_OK = 0, ORC_FREE_DOUBLE = 1, ORC_FREE_INVALID = 2, ORC_FREE_NULL = 3 };

/* ---- closed forms of the geometry (Results: page and chunk allocators) ---- */
int      orc_class_of(uint64_t n, uint64_t chunk_bytes);   /* -1: NULL request */
void     orc_classes(const uint64_t* sizes, uint64_t n, uint64_t chunk_bytes, int8_t* out);
uint32_t orc_num_classes(uint64_t chunk_bytes);
uint64_t orc_page_bytes(uint32_t k);
uint64_t orc_pages_per_chunk(uint64_t chunk_bytes, uint32_t k);
void     orc_shard_geometry(uint64_t n_chunks, uint32_t requested, uint32_t* shards, uint32_t* log2_span);
uint64_t orc_page_ring_entries(uint64_t bytes, uint64_t chunk_bytes, uint32_t shards);
uint64_t orc_page_max_chunks(uint64_t bytes, uint64_t chunk_bytes, uint32_t k, uint32_t shards);
int      orc_geometry_ok(uint64_t bytes, uint64_t chunk_bytes);
/* virtualised array page variant: segment size (log2 entries), segments and
 * page budget per shard */
uint32_t orc_va_log2_seg(uint64_t bytes, uint64_t chunk_bytes, uint32_t shards);
uint64_t orc_va_segments(uint64_t bytes, uint64_t chunk_bytes, uint32_t shards);
uint64_t orc_va_budget(uint64_t bytes, uint64_t chunk_bytes, uint32_t shards);
/* Virtualised array chunk variant (shards as requested of orc_create_ex):
 * log2 of the segment size and the segments per shard. */
uint32_t orc_va_chunk_log2_seg(uint64_t bytes, uint64_t chunk_bytes, uint32_t shards);
uint64_t orc_va_chunk_segments(uint64_t bytes, uint64_t chunk_bytes, uint32_t shards);

/* ---- sequential allocator ---- */
typedef struct orc_heap orc_heap;

typedef struct {
    uint32_t n_classes;
    uint32_t pad;
    uint64_t n_chunks;
    uint64_t free_chunks;                      /* chunks owned by no class */
    uint64_t live[ORC_MAX_CLASSES];            /* allocated pages per class */
    uint64_t chunks[ORC_MAX_CLASSES];          /* chunks owned per class    */
    uint64_t free_pages[ORC_MAX_CLASSES];      /* free pages inside owned chunks */
    uint64_t n_alloc_ok, n_alloc_null, n_free_ok, n_free_double, n_free_invalid;
} orc_acct;

/* shards: power of two <= 64, 0 for one per 256 chunks (up to 64) */
orc_heap* orc_create_ex(uint64_t bytes, uint64_t chunk_bytes, int variant, int policy, uint32_t shards);
orc_heap* orc_create(uint64_t bytes, uint64_t chunk_bytes, int variant, int policy); /* one shard */
/* Eager retirement (chunk variant, before any request): a chunk whose pages
 * are all free again returns to its shard's pool at once instead of at the
 * next trim (LOWEST: the unowned set; FIFO: the back of the shard's pool
 * queue).  Returns 0, or -1 for another variant or a heap already used. */
int orc_set_eager(orc_heap* h);
uint32_t  orc_shards(const orc_heap* h);
void      orc_destroy(orc_heap* h);
int64_t   orc_alloc(orc_heap* h, uint64_t n);
int       orc_free(orc_heap* h, int64_t off);
void      orc_trim(orc_heap* h);
void      orc_alloc_batch(orc_heap* h, const uint64_t* sizes, int64_t* offs, uint64_t n);
void      orc_free_batch(orc_heap* h, const int64_t* offs, uint64_t n, int32_t* status);
void      orc_accounting(const orc_heap* h, orc_acct* out);
/* replay of a mixed op list: op[i] >= 0 is an allocation of op[i] bytes whose
 * offset goes to out[i]; op[i] < 0 frees the block allocated by op index
 * (-op[i] - 1), and out[i] receives the free status. */
void      orc_replay(orc_heap* h, const int64_t* op, uint64_t n, int64_t* out);

/* ---- pattern written into every block (harness) ---- */
uint32_t orc_fmix32(uint32_t x);
uint32_t orc_pattern_word(uint32_t seed, uint32_t req, uint32_t i);
void     orc_pattern_fill(uint32_t seed, uint32_t req, uint8_t* dst, uint64_t nbytes);
/* 32-bit wrap-around sum of the little-endian words of the first nbytes of
 * the pattern (a partial last word zero-extended); batch form per request */
uint32_t orc_pattern_sum(uint32_t seed, uint32_t req, uint64_t nbytes);
void     orc_pattern_sums(uint32_t seed, const uint64_t* reqs, const uint64_t* sizes, uint64_t n, uint32_t* out);

/* ---- invariant checker ---- */
typedef struct {
    uint64_t n, n_null, n_nonnull;
    uint64_t n_null_valid;        /* NULL for a request that had a valid size */
    uint64_t n_bad_size_nonnull;  /* non-NULL for size 0 or size > chunk      */
    uint64_t n_oob, n_misaligned, n_straddle;
    uint64_t n_overlap;           /* overlapping neighbour pairs after sorting */
    uint64_t live[ORC_MAX_CLASSES];
} orc_blocks_report;

int orc_check_blocks(uint64_t data_bytes, uint64_t chunk_bytes, const uint64_t* sizes,
                     const int64_t* offs, uint64_t n, orc_blocks_report* rep);

typedef struct {
    int32_t  ok_header;
    uint32_t n_classes;
    uint64_t bad_class_byte, bad_free_chunk, bad_stray_bits, bad_count;
    uint64_t bad_pool, bad_ring_ctl, bad_ring_entry, bad_ring_missing, bad_ring_dup;
    uint64_t bad_conservation, bad_owned;
    uint64_t bad_vdir, bad_vtaken, bad_vstore, bad_committed; /* virtualised array */
    uint64_t free_chunks;
    uint64_t live[ORC_MAX_CLASSES], chunks[ORC_MAX_CLASSES], free_pages[ORC_MAX_CLASSES];
    uint64_t stale_entries;       /* eager retirement: queue entries no token names */
    uint32_t eager, pad;
    uint64_t whole_owned;         /* eager retirement: owned chunks with every page free
                                     (kept while a stale entry of theirs blocked it) */
} orc_snap_report;

/* Quiescent-state consistency of a snapshot (documented layout, version 4). */
int orc_check_snapshot(const uint8_t* snap, uint64_t len, orc_snap_report* rep);

/* Blocks against a snapshot: each live block must lie in a chunk of its
 * request's class with its page bit clear (allocated).  Returns the number
 * of blocks that fail. */
uint64_t orc_check_blocks_in_snapshot(const uint8_t* snap, uint64_t len, const uint64_t* sizes,
                                      const int64_t* offs, uint64_t n);

/* ---- step-level model of the concurrent algorithm (hbheap_model.c) ---- */
#define ORC_MODEL_MAXL 3
#define ORC_MODEL_MAXOPS 3
enum { ORC_OP_NONE = 0, ORC_OP_ALLOC = 1, ORC_OP_FREE_OWN = 2, ORC_OP_FREE_GIVEN = 3 };

/* ALLOC: a = pages wanted (group size <= 4); FREE_OWN: a = index of an
 * earlier ALLOC op of the same leader whose pages are freed; FREE_GIVEN:
 * free prefill pages [a, a+b). */
typedef struct { int32_t kind, a, b; } orc_model_op;

typedef struct {
    int32_t variant;           /* 0 chunk, 1 page                         */
    int32_t n_chunks;          /* <= 4                                    */
    int32_t ppc;               /* pages per chunk, <= 8                   */
    int32_t maxc;              /* page variant: chunks the class may own  */
    int32_t n_leaders;         /* <= 3                                    */
    int32_t n_ops[ORC_MODEL_MAXL];
    orc_model_op ops[ORC_MODEL_MAXL][ORC_MODEL_MAXOPS];
    int32_t prefill;           /* pages allocated before exploration      */
    int32_t freeze;            /* also run the freeze analysis            */
    int32_t mutation;          /* planted mistake, 0 for none             */
    int32_t dry_hint;          /* page alloc reads the pool first and skips
                                  the hold on a dry pool                  */
    int32_t fast_first;        /* page alloc: the first pass never refills */
    int32_t first_nohold;      /* page alloc: every first pass takes without
                                  a hold and never refills                */
    int32_t early_requeue;     /* chunk alloc: a pass that will not refill
                                  requeues and releases before it claims  */
    int32_t pad2_;
    int64_t max_states;
} orc_model_params;

typedef struct {
    int64_t states, terminals, violations, deadlocks;
    int64_t token_violations, oom_violations, final_violations, grant_violations;
    int64_t blocked_freezes;   /* freeze points where others cannot finish */
    int64_t null_outcomes;     /* final states where some request got NULL */
    int32_t truncated;
    int32_t first_violation;
    uint32_t blocking_pcs;     /* bit mask of the frozen leader's pcs mod 32 */
    uint32_t dry_starts;       /* page allocs that started on a dry pool   */
    uint64_t blocking_set[4];  /* the same pcs, all 256 of them, exactly    */
} orc_model_result;

/* 0 on success, negative for bad parameters. */
int orc_model_run(const orc_model_params* p, orc_model_result* r);

/* ---- step-level model of the page variant across shards
 *      (hbheap_shards_model.c): home passes, the scan of every shard,
 *      stealing, and the out-of-memory answer ---- */
#define ORC_SHARDS_MAXL 3
enum { ORC_SOP_ALLOC = 1, ORC_SOP_FREE = 2 };

/* ALLOC: a = pages wanted (<= ppc), b = home shard; FREE: free the
 * pre-allocated pages [a, a + b) (page v = (shard * chunks + chunk) * ppc
 * + page). */
typedef struct { int32_t kind, a, b; } orc_shards_op;

typedef struct {
    int32_t n_shards;          /* <= 3                                     */
    int32_t chunks;            /* chunks per shard, <= 2                   */
    int32_t ppc;               /* pages per chunk, <= 4                    */
    int32_t n_leaders;         /* <= 3, one operation each                 */
    orc_shards_op ops[ORC_SHARDS_MAXL];
    int32_t taken[3];          /* chunks of shard j owned by the class at the start */
    uint32_t prealloc[3];      /* of those, pages allocated (bit c*ppc + p); the
                                  others are free and published in order   */
    int32_t mutation;          /* planted mistake, 0 for none              */
    int32_t room;              /* most chunks the class may own per shard
                                  (a cap on the room counter), 0 for none  */
    int64_t max_states;
} orc_shards_params;

typedef struct {
    int64_t states, terminals, violations, deadlocks;
    int64_t oom_violations, final_violations, grant_violations;
    int64_t null_outcomes;     /* final states where some request got NULL */
    int32_t truncated;
    int32_t first_violation;
} orc_shards_result;

int orc_shards_model_run(const orc_shards_params* p, orc_shards_result* r);

/* ---- step-level model of the virtualised queues (hbheap_seg_model.c):
 *      segments from a shared store, the array form's directory and the
 *      list form's links, tags and front retirement ---- */
#define ORC_SEG_MAXL 3
#define ORC_SEG_MAXOPS 6
enum { ORC_GOP_PUT = 1, ORC_GOP_GET = 2 };

/* PUT: enqueue `value` (< 32, distinct over the run) on `queue`; GET:
 * dequeue one entry of `queue` (waits for a published one). */
typedef struct { int32_t kind, queue, value; } orc_seg_op;

typedef struct {
    int32_t list;              /* 0: array form, 1: list form              */
    int32_t n_queues;          /* <= 2, sharing the store                  */
    int32_t segments;          /* ids in the store (list: one per queue
                                  starts in use), 2 .. 4; 2 slots each      */
    int32_t n_leaders;         /* <= 3                                     */
    int32_t n_ops[ORC_SEG_MAXL];
    orc_seg_op ops[ORC_SEG_MAXL][ORC_SEG_MAXOPS];
    int32_t consume_all;       /* every value put is also taken            */
    int32_t mutation;          /* planted mistake, 0 for none              */
    int64_t max_states;
} orc_seg_params;

typedef struct {
    int64_t states, terminals, violations, deadlocks;
    int64_t value_violations, segment_violations, final_violations;
    int32_t truncated;
    int32_t first_violation;
} orc_seg_result;

int orc_seg_model_run(const orc_seg_params* p, orc_seg_result* r);

#ifdef __cplusplus
}
#endif
#endif
