/*
 * hbheap_growth.h -- C ABI of the growth line: many agents grow lists by
 * repeated reallocation inside persistent kernels, with the steps replayed
 * as one HIP graph, and an autotuner over heap geometry and queue options.
 *
 * What it exercises is the paper's use case (Introduction: threads of a
 * running kernel allocate without returning to the host; Methods: many
 * threads allocate at once) in its most dynamic form: each step, every
 * active agent allocates a block twice as large, copies its list into it,
 * appends new elements and frees the old block (the device allocator's
 * wave-level allocate and free).
 *
 * Agent a's list holds 32-bit words; word j of agent a is
 *     fmix32(seed ^ fmix32(a) ^ j * 0x9E3779B9)
 * (the same word as heap_pattern_write for request a), so after any step a
 * list of e elements is exactly the pattern of 4*e bytes and can be checked
 * with heap_pattern_check on the exported pointers and sizes.
 *
 * Schedule: step 0 allocates 16 B (4 elements) per agent; step s >= 1 doubles
 * the list of every agent with doublings[a] >= s.  Agents whose allocation
 * returns NULL keep their old list and are counted as failures.
 *
 * Conventions as in hbheap.h: 0 or a negative HBHEAP_E_* code; device
 * buffers are owned by the caller; stream calls are asynchronous.
 */
#ifndef HBHEAP_GROWTH_H
#define HBHEAP_GROWTH_H

#include "hbheap.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hbheap_growth* growth_t;

/*
 * Create a growth run over heap h for `agents` agents (1 .. 2^24) and
 * `steps` steps (1 .. 16; step s allocates 16 B * 2^s, so steps - 1 must
 * keep 16 B * 2^(steps-1) within the chunk size).  doublings: device buffer
 * of `agents` int32 (copied at creation; values are clamped to steps - 1).
 * seed: the list contents' seed.  The growth object owns a device table of
 * list pointers and element counts (12 B per agent); the lists themselves
 * are heap blocks.  Blocking.  Errors: HBHEAP_E_INVAL, HBHEAP_E_NOMEM,
 * HBHEAP_E_HIP.
 */
int growth_create(heap_t h, uint32_t agents, const int32_t* doublings, uint32_t steps, uint32_t seed,
                  growth_t* out);

/* Free the growth object's tables (not the lists: call growth_release
 * first, or let the heap keep them).  The caller guarantees nothing is in
 * flight.  NULL is a no-op. */
int growth_destroy(growth_t g);

/* Launch step `step` (< steps) as one persistent grid-stride kernel. */
int growth_step(growth_t g, uint32_t step, hipStream_t stream);

/*
 * Launch all steps as one HIP graph (kernel nodes in a chain, built and
 * instantiated on the first call; no memset nodes).  The graph holds the
 * heap's device handle as it was at that first call: flags changed later
 * with heap_set_flags are not seen by the graph.
 */
int growth_graph_launch(growth_t g, hipStream_t stream);

/* Free every agent's list (a grid-stride kernel), set the
 * tables to empty and the failure counter to zero. */
int growth_release(growth_t g, hipStream_t stream);

/*
 * Copy the tables out: ptrs (device, agents x u64: list address or 0) and
 * bytes (device, agents x u64: list bytes = 4 * elements, 0 for none);
 * either may be NULL.  failures (device, one u64, may be NULL): allocations
 * that returned NULL since the last release.
 */
int growth_export(growth_t g, uint64_t* ptrs, uint64_t* bytes, uint64_t* failures, hipStream_t stream);

/* Geometry of the persistent launch: blocks of 256 lanes. */
int growth_launch_shape(growth_t g, uint32_t* blocks, uint32_t* threads);

/* ---- autotuner ---- */

typedef struct growth_candidate {
    uint64_t chunk_bytes;   /* power of two in [4 KiB, 64 KiB]          */
    uint32_t variant;       /* any HBHEAP_VARIANT_*                     */
    uint32_t width;         /* aggregation width: 1, 2, 4 .. 64         */
    uint32_t flags;         /* creation flags: 0, or HBHEAP_FLAG_EAGER
                               with the chunk variant                   */
    uint32_t reserved;      /* 0                                        */
} growth_candidate_t;

/*
 * Time every candidate on the same schedule: for each one, create a heap of
 * heap_bytes with that geometry (default shards), a growth run, replay the
 * graph once untimed, then `reps` timed replays (HIP events around each
 * graph launch, a release after each), keep the median; destroy.  ms:
 * host array of n_cand floats (median graph time per candidate, or a
 * negative value when the candidate could not run or had failures).
 * *best: index of the fastest candidate that ran without failures (or -1).
 * Blocking; uses its own stream.  Errors: HBHEAP_E_INVAL.
 */
int growth_autotune(size_t heap_bytes, uint32_t agents, const int32_t* doublings, uint32_t steps, uint32_t seed,
                    const growth_candidate_t* cand, uint32_t n_cand, uint32_t reps, float* ms, int32_t* best);

#ifdef __cplusplus
}
#endif
#endif
