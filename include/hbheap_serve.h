/*
 * hbheap_serve.h -- C ABI of the serving line: a host loop that takes
 * batches of allocation and free requests as they arrive, admits them
 * against the heap's free memory, and keeps up to K batches in flight on
 * their own streams, so that batches arriving while others run overlap on
 * the device.  The heap state stays resident on the device throughout.
 *
 * The allocation itself is the paper's method (Introduction: a heap the
 * host preallocates, served on the device by a heap algorithm); the loop
 * around it is the serving use of that heap.
 *
 * Requests of one run are numbered 0 .. R-1 in batch order.  ops[i] >= 0
 * asks for ops[i] bytes; ops[i] < 0 frees the block of request -ops[i]-1,
 * which must be an allocation of a batch at least `free_lag` batches
 * earlier, not freed before in the run.  Block addresses never travel to the
 * host: the device keeps a table of one address per request.
 *
 * Each request's work on the device: an allocation writes the seeded words
 *     w_j = fmix32(seed ^ fmix32(i) ^ j * 0x9E3779B9)
 * (i = request number; the first `size` bytes of that little-endian word
 * sequence) and reads them back; a free reads its block back, then frees
 * it.  The result of a request is (status, class, checksum), the checksum
 * being the 32-bit wrap-around sum of the words read back (a partial last
 * word zero-extended).  Results do not depend on timing or on the other
 * batches in flight: a run processed one batch at a time gives the same
 * results as the overlapped run.
 *
 * Admission (occupancy in chunks): a batch is launched only if
 *     chunks in use (upper bound) + worst case of the batch <= admit * N.
 * The worst case of a batch is the sum, over every (wave of 64 requests,
 * width segment, class) group of its allocations, of ceil(g / pages per
 * chunk): a group never takes more fresh chunks than that.  Chunks in use
 * are read from the pool counters by the last workgroup of each batch's
 * kernel and come back with its results (exact for that batch; the worst
 * cases of the batches in flight at its launch, and of those launched
 * since, are added).  Page variant: the same bound is
 * kept per class against the class's capacity (per shard, the chunks its
 * queue can hold the pages of), so an admitted allocation never fails.
 * When the bound does not admit the next batch and nothing is in flight,
 * the loop recounts exactly and, if that is not enough, trims the heap
 * (quiescent: fully free chunks return to the pools) and recounts.
 *
 * Conventions as in hbheap.h.  One run at a time per server; the heap must
 * not be used by other work while a run is in progress.
 */
#ifndef HBHEAP_SERVE_H
#define HBHEAP_SERVE_H

#include "hbheap.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hbheap_server* server_t;

typedef struct serve_config {
    uint32_t slots;          /* K: batches in flight, 1 .. 16 (streams)          */
    uint32_t max_batch;      /* largest batch, 1 .. 65536                        */
    uint64_t max_requests;   /* requests per run (device table: 8 B each)        */
    double   admit;          /* occupancy cap as a fraction of the chunks, (0,1] */
    uint32_t seed;           /* seed of the words written into blocks            */
    uint32_t free_lag;       /* >= 1: a free trails its allocation by that many
                                batches (its batch is complete when it launches) */
} serve_config_t;

/* Per-request status values. */
#define SERVE_OK          0   /* allocated, or freed                        */
#define SERVE_FREE_DOUBLE 1   /* free of a block already free               */
#define SERVE_FREE_INVAL  2   /* free of an address the heap did not hand out */
#define SERVE_FREE_NULL   3   /* free of a request whose allocation was NULL */
#define SERVE_ALLOC_NULL  4   /* allocation returned NULL                   */

typedef struct serve_stats {
    uint64_t batches, requests, allocs, frees;
    uint64_t trims;              /* quiescent trims the admission needed      */
    uint64_t admission_stalls;   /* batches that waited for admission         */
    uint64_t monitor_reads;      /* chunk-usage reads taken with batch results */
    uint64_t peak_bound;         /* largest chunks-in-use bound admitted      */
    uint64_t final_chunks;       /* chunks in use at the end (exact)          */
    double   wall_s;             /* first arrival .. last completion          */
} serve_stats_t;

/* Create a server over heap h, with K streams, pinned staging of 16 B per
 * request per slot, and the device table of max_requests addresses.  Chunk
 * variants (plain, virtualised array, virtualised list) and the page
 * variant are served; the page variant's admission also keeps per-class page
 * budgets.  The virtualised page variants are refused: their classes share
 * one page budget per shard, and a request can fail with chunks left in one
 * shard and budget left in another, which no bound on chunks in use rules
 * out.  Blocking.  Errors: HBHEAP_E_INVAL (also for a virtualised page
 * variant heap), HBHEAP_E_NOMEM, HBHEAP_E_HIP. */
int serve_create(heap_t h, const serve_config_t* cfg, server_t* out);

/* Release the server's streams and buffers (not the heap).  NULL is a no-op. */
int serve_destroy(server_t s);

/*
 * Run n_batches batches.  Host arrays: first (n_batches + 1 entries: batch b
 * = requests [first[b], first[b+1]), first[0] = 0), ops (first[n_batches]
 * entries), arrival_ns (n_batches, nondecreasing, relative to the start;
 * ignored when alone != 0).  alone = 0: real-time loop, batches launched
 * from their arrival on as slots and admission allow, up to K in flight;
 * alone = 1: one batch at a time, each waited for before the next.
 * Outputs (host, may be NULL): status, cls (class of the block, -1 for
 * none) and sum per request; latency_ns (arrival -> completion seen by the
 * host; alone: launch -> completion) and wait_ns (arrival -> launch) per
 * batch; stats.  The request list is validated before anything runs.
 * Blocking.  Errors: HBHEAP_E_INVAL (arguments, request list),
 * HBHEAP_E_NOMEM (a batch cannot be admitted even after a trim),
 * HBHEAP_E_HIP.
 */
int serve_run(server_t s, uint32_t n_batches, const uint64_t* first, const int64_t* ops, const uint64_t* arrival_ns,
              int alone, uint8_t* status, int8_t* cls, uint32_t* sum, uint64_t* latency_ns, uint64_t* wait_ns,
              serve_stats_t* stats);

/* Copy the device addresses of requests [first, first + n) into dst (device
 * buffer of n u64; 0 for frees and NULL allocations).  Stream-ordered. */
int serve_export(server_t s, uint64_t first, uint64_t n, uint64_t* dst, hipStream_t stream);

/* Chunks owned by size classes (taken from the pools), read from the pool
 * counters on `stream` and waited for.  Exact at quiescence. */
int heap_chunks_in_use(heap_t h, uint64_t* out, hipStream_t stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * count as heap_chunks_in_use, with no hipMalloc, hipFree or other
 * allocating call.  Its staging lives in a fixed device array of the
 * library (17 u64 per GPU, held until the process ends), not in memory
 * allocated per call.  out: device buffer of one u64, written in stream
 * order (asynchronous: nothing is waited for, so the call can be captured
 * into a graph).  Calls that overlap on one GPU share that array and race:
 * the caller orders them (one stream, or events).
 * Errors: HBHEAP_E_INVAL (h or out NULL), HBHEAP_E_RANGE (a heap with more
 * than 16 classes: never for heaps heap_create makes), HBHEAP_E_UNSUP
 * (device index beyond 63), HBHEAP_E_HIP.
 */
int heap_chunks_in_use_noalloc(heap_t h, uint64_t* out, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif
