/*
 * hbheap.h -- C ABI of the device heap allocator (host side).
 *
 * The paper's problem statement (Introduction): dynamic allocation inside
 * running device kernels, served by a heap that the host preallocates once
 * and that a heap algorithm on the device manages; the block is cut into
 * chunks, each size served through its own lock-free queue.  The paper's
 * driver (Methods) allocates many blocks in parallel, writes data into them,
 * checks it on read-back and frees them, timing allocation and free.
 *
 * Conventions for every entry point:
 *   - Return 0 (HBHEAP_OK) or a negative HBHEAP_E_* code; nothing aborts the
 *     process.  Arguments are validated on the host before any launch.
 *   - "device buffer" = memory from hipMalloc (or a torch CUDA tensor)
 *     that the caller owns and keeps alive until the work on `stream` ends.
 *   - Calls that take a stream are asynchronous and stream-ordered unless
 *     said otherwise.  A NULL stream is the null stream.
 *   - The library owns every byte of the heap; `heap_t` is opaque.
 */
#ifndef HBHEAP_H
#define HBHEAP_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#include "hbheap_types.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hbheap_heap* heap_t;

/* Tunables of heap_create_ex.  Zero fields take the defaults. */
typedef struct heap_config {
    uint32_t variant;      /* HBHEAP_VARIANT_CHUNK (default), _PAGE, _VA_PAGE,
                              _VA_CHUNK, _VL_PAGE or _VL_CHUNK               */
    uint32_t width;        /* lanes aggregated per queue operation: power of
                              two in [1, 64], default 64                     */
    uint32_t spin_cap;     /* bounded-wait iterations, default 1 << 18        */
    uint32_t backoff_max;  /* longest backoff in s_sleep(1) units, default 64 */
    uint32_t flags;        /* HBHEAP_FLAG_*; HBHEAP_FLAG_EAGER (chunk variant
                              only) is fixed for the heap's lifetime         */
    uint32_t shards;       /* queue shards: power of two <= 64; 0 = about one
                              per 256 chunks, at most 64                     */
    uint32_t rows;         /* requests per lane of the batch kernels: 1 or 4,
                              0 = 4.  With 4, a wave serves 256 requests
                              and each of its queue operations covers all of
                              them.  Applies at widths of 16 or more to
                              every variant but the virtualised-list page
                              variant, which always uses 1                   */
} heap_config_t;

/* Geometry and placement of a heap (heap_info). */
typedef struct heap_info {
    void*    data;            /* device address of the data region           */
    uint64_t data_bytes;      /* n_chunks * chunk_bytes                      */
    uint64_t chunk_bytes;
    uint64_t n_chunks;
    uint32_t n_classes;       /* pages 16 B * 2^k, k < n_classes             */
    uint32_t variant;
    uint64_t ring_entries;    /* capacity of each (shard, class) queue; for
                                 the virtualised array page variant, the
                                 pages the classes of one shard may own
                                 together (virtualised array chunk variant:
                                 the chunks of a shard, which its queues
                                 always have room for)                      */
    uint64_t state_bytes;     /* size of the state region (= snapshot size)  */
    uint64_t metadata_bytes;  /* all device memory besides the data region   */
    uint32_t n_shards;        /* shards actually used (chunk runs of a power
                                 of two, the last one possibly shorter)      */
    uint32_t reserved;
} heap_info_t;

/*
 * Create a heap of floor(bytes / chunk_bytes) chunks (Introduction: the host
 * preallocates the heap).  Metadata is allocated separately and is not
 * counted in `bytes`.  chunk_bytes: power of two in [4 KiB, 64 KiB]; bytes
 * >= chunk_bytes; page variants: data region at most 64 GiB.  Blocking: the
 * heap is initialised when the call returns.  *out is untouched on error.
 * cfg->flags with HBHEAP_FLAG_EAGER (chunk variant only; at most 2^27 chunks
 * per shard): a chunk whose pages are all free again leaves its class at
 * once and goes back to its shard's pool -- the paper leaves open when a
 * chunk changes class; the default keeps it with its class until
 * heap_trim.  Out of memory stays exact for launches without frees (no
 * chunk retires during them).
 * Errors: HBHEAP_E_INVAL (geometry, config, out == NULL), HBHEAP_E_NOMEM
 * (hipMalloc failed), HBHEAP_E_HIP.
 */
int heap_create(size_t bytes, size_t chunk_bytes, heap_t* out);
int heap_create_ex(size_t bytes, size_t chunk_bytes, const heap_config_t* cfg, heap_t* out);

/* Free all device memory of the heap.  The caller guarantees no work on the
 * heap is in flight; every block becomes invalid.  NULL is a no-op. */
int heap_destroy(heap_t h);

/*
 * Batch allocation: thread i of one launch sets ptrs[i] to a block of at
 * least sizes[i] bytes, or NULL when sizes[i] is 0, exceeds chunk_bytes, or
 * neither a page of its class nor an unowned chunk is left at some instant
 * between the start of the launch and the request's answer (all requests of
 * a launch are issued together; a proof of exhaustion found by one wave of
 * a workgroup answers the others of the same class).  sizes (u64) and
 * ptrs are device buffers of n entries.  256-thread blocks; the lanes of each
 * wave are aggregated by size class (Porting section: warp votes let several
 * allocations of one warp proceed together).
 * Errors: HBHEAP_E_INVAL (h NULL, or a NULL buffer with n > 0), HBHEAP_E_HIP.
 */
int heap_alloc_batch(heap_t h, const size_t* sizes, void** ptrs, size_t n, hipStream_t stream);

/*
 * Batch free of ptrs[0..n) (device buffer).  NULL entries are skipped.
 * sizes may be NULL; if given, each must be the size the block was
 * requested with (same class), else the free is invalid.  Invalid pointers
 * and double frees are ignored and set bits of the sticky error word.
 */
int heap_free_batch(heap_t h, const size_t* sizes, void* const* ptrs, size_t n, hipStream_t stream);

/* As heap_free_batch; status (device buffer of n int32, may be NULL)
 * receives 0 ok, 1 double free, 2 invalid, 3 NULL pointer per entry. */
int heap_free_batch_ex(heap_t h, const size_t* sizes, void* const* ptrs, size_t n, int32_t* status,
                       hipStream_t stream);

/* Replace the HBHEAP_FLAG_* bits used by launches issued after this call
 * (and by handles obtained after it).  HBHEAP_FLAG_EAGER is kept as the
 * heap was created, whatever `flags` says. */
int heap_set_flags(heap_t h, uint32_t flags);

/* Device handle for user kernels calling dev_malloc/dev_free
 * (hbheap_device.h).  Valid until heap_destroy. */
int heap_device_handle(heap_t h, hbheap_dev_t* out);

/* Geometry, placement and metadata size. */
int heap_info(heap_t h, heap_info_t* out);

/*
 * Quiescent trim (stream-ordered; no other work on the heap may overlap):
 * chunks whose pages are all free return to the pool, and the pool and the
 * class queues are rewritten in ascending order with head = 0.  After every
 * block is freed, trim makes the state region byte-identical to a fresh
 * heap's.  With eager retirement (HBHEAP_FLAG_EAGER) no owned chunk is ever
 * whole at quiescence; trim then only compacts the queues (dropping their
 * stale entries) and the pool rings.
 */
int heap_trim(heap_t h, hipStream_t stream);

/*
 * Copy the state region into host memory `dst` of `cap` bytes.  Layout
 * version 4: a 256-byte header (magic 0x48424850, version, geometry, the
 * variant, and the byte offset of every section: pools, class blocks, class
 * bytes, free counts, bitmask words, pool ids, queue slots, and for the
 * segmented variants the directories or segment tags and links, consumed
 * counts and segment stores), then the sections.  Bitmask words are
 * word-major: word w of chunk c at index w * n_chunks + c.  Eager retirement: header
 * u32 at 168 is 1 and u64 at 176 the offset of the per-chunk count/token
 * words (hbheap_types.h, chunk_ct); pools are rings (state, head, tail) over
 * pool ids padded to S << log2_span; queues have twice the slots (room for
 * stale entries); the u32 free counts stay zero.  Synchronises `stream`.
 * *len receives the size (also when cap is too small, which returns
 * HBHEAP_E_RANGE).  dst may be NULL to query the size.
 */
int heap_snapshot(heap_t h, void* dst, size_t cap, size_t* len, hipStream_t stream);

/* Sticky device error word (HBHEAP_ERR_* bits); synchronises the device
 * copy with a blocking read.  heap_clear_error resets it to 0. */
int heap_get_error(heap_t h, uint32_t* err);
int heap_clear_error(heap_t h);

/* Device statistics counters, one field per HBHEAP_STAT_* index (field i is
 * counter i).  The failure and timeout counters are always kept; the refill,
 * grab, retirement and atomics-by-target counters only on heaps created with
 * HBHEAP_FLAG_STATS (else they stay 0). */
typedef struct heap_stats_t {
    uint64_t chunk_grabs;   /* chunks taken from a pool                          */
    uint64_t refills;       /* refills of a class queue                          */
    uint64_t oom;           /* requests answered NULL because the heap was full  */
    uint64_t oom_waits;     /* exhaustion proofs that had to wait for holds      */
    uint64_t double_free;   /* frees of a block that was already free            */
    uint64_t invalid_free;  /* frees of an address that is no block of the heap  */
    uint64_t timeouts;      /* bounded waits that gave up (HBHEAP_ERR_TIMEOUT)   */
    uint64_t reserved7;
    uint64_t state_ops;     /* atomics on class state words                      */
    uint64_t headtail_ops;  /* atomics on class head and tail words              */
    uint64_t pool_ops;      /* atomics on pool counters                          */
    uint64_t spread_ops;    /* per-lane bitmask and chunk-count atomics          */
    uint64_t retired;       /* chunks retired eagerly                            */
    uint64_t slot_ops;      /* per-lane ring slot atomics                        */
    uint64_t reserved14;
    uint64_t reserved15;
} heap_stats_t;

/* Read the statistics counters into *out (host memory); blocking (waits for
 * the device).  Errors: HBHEAP_E_INVAL for a NULL argument, HBHEAP_E_HIP. */
int heap_stats(heap_t h, heap_stats_t* out);

/*
 * Single-thread replay of an op list on one device lane, in order (the
 * deterministic case that a sequential pool allocator reproduces exactly).
 * ops/out: device buffers of n int64.  ops[i] >= 0 allocates ops[i] bytes and
 * out[i] gets the block's byte offset in the data region or -1; ops[i] < 0
 * frees the block of op index -ops[i]-1 (a previous allocation) and out[i]
 * gets the free status (0 ok, 1 double, 2 invalid, 3 NULL).
 */
int heap_replay(heap_t h, const int64_t* ops, int64_t* out, size_t n, hipStream_t stream);

/* ---------------- harness: payload written into blocks (Methods) ---------
 * Block i holds exactly sizes[i] bytes of the little-endian words
 * w_j = fmix32(seed ^ fmix32(i) ^ j * 0x9E3779B9), fmix32 being the 32-bit
 * finaliser of MurmurHash3; the last word is truncated.  NULL blocks are
 * skipped, and so is any block not wholly inside h's data region (the check
 * counts it as one mismatch).  heap_pattern_check adds the number of
 * mismatching words to *mismatches (a device u64). */
int heap_pattern_write(heap_t h, void* const* ptrs, const size_t* sizes, size_t n, uint32_t seed,
                       hipStream_t stream);
int heap_pattern_check(heap_t h, void* const* ptrs, const size_t* sizes, size_t n, uint32_t seed,
                       unsigned long long* mismatches, hipStream_t stream);

/* ---------------- measurement kernels ----------------------------------- */

/* Device atomic-throughput probes over `buf` (device, >= buf_bytes):
 *   pattern 0: one 64-bit atomic add per wave, all on one address;
 *   pattern 1: one per wave on `lines` addresses 128 B apart (wave % lines);
 *   pattern 2: one 32-bit atomic add per lane on pseudo-random words of buf;
 *   pattern 3: one 64-bit compare-and-swap per wave on one address;
 *   pattern 4: one 64-bit atomic add per lane on one address;
 *   pattern 5: one 32-bit exchange per lane, lanes on consecutive words;
 *   pattern 6: one coherent (device-scope) 32-bit load and store per lane,
 *              lanes on consecutive words;
 *   pattern 7: the same with 64-bit words;
 *   pattern 8: a chain of 32-bit atomic adds per lane, lanes on consecutive
 *              words, each add's address depending on the value the lane's
 *              previous add returned (dependent round trips).
 * `threads` lanes each repeat `iters` times.  Operations issued: patterns 2
 * and 4..8: threads * iters; others: threads / 64 * iters. */
int hb_atomic_probe(int pattern, void* buf, size_t buf_bytes, size_t threads, uint32_t lines, uint32_t iters,
                    hipStream_t stream);

/* HBM stream copy of `bytes` (multiple of 16) from src to dst. */
int hb_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t stream);

/* Schedule fuzzing, for concurrency tests (the paper throttles allocating
 * threads with sleeps, Porting section; here sleeps are injected to widen
 * race windows instead).  Only the test build of the library
 * (libhbheap_fuzz.so, compiled with HBHEAP_FUZZ=1) has fuzz points: between
 * the atomic steps of reservations, takes, refills, publications, frees,
 * scans and segment hand-offs, a wave sleeps at one point in four for up to
 * most_sleeps - 1 periods of s_sleep 4, drawn from (seed, point, wave,
 * clock).  seed 0 turns it off.  Applies to every later launch of the
 * process; synchronises the device first.  The normal build returns
 * HBHEAP_E_UNSUP and has no fuzz points.  Errors: HBHEAP_E_HIP. */
int hb_fuzz_set(uint32_t seed, uint32_t most_sleeps);

/* Context figure (host code, no GPU): the host C library's malloc/free over
 * the device sweep's request streams.  For each of n_sizes sizes and each
 * of `iterations` rounds, `threads` host threads split `requests`
 * allocations of that size, wait for each other, then free them all;
 * seconds[size * iterations + round] receives the round's wall time (both
 * phases), *failed the number of NULL answers.  Errors: HBHEAP_E_INVAL
 * (NULL outputs, zero sizes/iterations/threads, threads > 1024),
 * HBHEAP_E_NOMEM. */
int hb_host_malloc_sweep(const uint64_t* sizes, uint32_t n_sizes, uint64_t requests, uint32_t iterations,
                         uint32_t threads, double* seconds, uint64_t* failed);

/* Baseline: the runtime's own per-thread device malloc / free.
 * hb_plain_set_heap sets the device malloc heap limit (call before use). */
int hb_plain_set_heap(size_t bytes);
int hb_plain_alloc(const size_t* sizes, void** ptrs, size_t n, hipStream_t stream);
int hb_plain_free(void* const* ptrs, size_t n, hipStream_t stream);
/* The payload words of heap_pattern_write / heap_pattern_check, for blocks
 * of the runtime's allocator (ptrs from hb_plain_alloc; device buffers):
 * writes them when mismatches is NULL, else checks them and adds the number
 * of mismatching words to *mismatches (a device u64).  NULL blocks are
 * skipped. */
int hb_plain_pattern(void* const* ptrs, const size_t* sizes, size_t n, uint32_t seed, unsigned long long* mismatches,
                     hipStream_t stream);

/* Library version string. */
const char* hbheap_version(void);

#ifdef __cplusplus
}
#endif
#endif
