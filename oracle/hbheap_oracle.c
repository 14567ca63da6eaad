/*
 * hbheap_oracle.c -- plain sequential CPU oracle of the device heap allocator.
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the
 * benchmark's CPU-baseline leg; never by the product path.  Written from the
 * paper and the documented snapshot format; it shares no code with the HIP
 * library.
 *
 * The method (Introduction; Results, "Page allocator" and "Chunk
 * allocator"): a heap preallocated by the host is cut into chunks of one
 * fixed size C; a chunk, once handed to a size, is split into pages of that
 * size; sizes are powers of two and each size has its own queue.  In the
 * chunk variant the queue lists chunks that still have free pages and an
 * allocation takes a chunk from it, then a free page inside that chunk; in
 * the page variant the queue lists free pages directly.
 *
 * Readings (paper silent): smallest page 16 B; classes k = 0..K-1 with page
 * 16*2^k and K = log2(C) - 3; a request n maps to the smallest page >= n;
 * n == 0 or n > C is a NULL request; a chunk is returned to the pool of
 * unowned chunks only by trim() at quiescence; the page variant's queues
 * share a budget of bytes/8 of metadata, which caps the chunks one class
 * may own.
 *
 * Two tie-break policies produce legal outcomes:
 *   LOWEST -- the lowest chunk with a free page, then its lowest free page,
 *             else the lowest unowned chunk (the canonical outcome);
 *   FIFO   -- queue order as one device thread alone sees it: class queues
 *             and the pool are first-in first-out, a chunk that keeps free
 *             pages after an allocation goes to the back of its queue, a
 *             fresh chunk serves its page 0 and publishes the rest, the pool
 *             hands out its ids in stored order.
 */
#include "hbheap_oracle.h"

#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* geometry                                                            */
/* ------------------------------------------------------------------ */

static int ilog2_u64(uint64_t x) { int r = -1; while (x) { x >>= 1; ++r; } return r; }
static int is_pow2(uint64_t x) { return x && !(x & (x - 1)); }

int orc_geometry_ok(uint64_t bytes, uint64_t chunk_bytes)
{
    if (!is_pow2(chunk_bytes) || chunk_bytes < 4096 || chunk_bytes > 65536) return 0;
    if (bytes < chunk_bytes) return 0;
    return 1;
}

uint32_t orc_num_classes(uint64_t chunk_bytes) { return (uint32_t)(ilog2_u64(chunk_bytes) - 3); }

uint64_t orc_page_bytes(uint32_t k) { return (uint64_t)16 << k; }

uint64_t orc_pages_per_chunk(uint64_t chunk_bytes, uint32_t k) { return chunk_bytes / orc_page_bytes(k); }

/* Smallest class whose page holds n bytes: walk the page sizes upward. */
int orc_class_of(uint64_t n, uint64_t chunk_bytes)
{
    if (n == 0 || n > chunk_bytes) return -1;
    uint32_t k = 0;
    while (orc_page_bytes(k) < n) ++k;
    return (int)k;
}

void orc_classes(const uint64_t* sizes, uint64_t n, uint64_t chunk_bytes, int8_t* out)
{
    for (uint64_t i = 0; i < n; ++i) out[i] = (int8_t)orc_class_of(sizes[i], chunk_bytes);
}

/* Shards: runs of 2^log2_span consecutive chunks, as many as needed to
 * cover N; the span is the smallest power of two >= ceil(N / requested).
 * requested == 0: one shard per 256 chunks, doubling up to 64. */
void orc_shard_geometry(uint64_t n_chunks, uint32_t requested, uint32_t* shards, uint32_t* log2_span)
{
    uint64_t want = requested;
    if (want == 0) {
        want = 1;
        while (want < 64 && want * 2 * 256 <= n_chunks) want *= 2;
    }
    if (want > n_chunks) want = n_chunks;
    uint64_t per = (n_chunks + want - 1) / want;
    uint32_t l = 0;
    while ((1ull << l) < per) ++l;
    *log2_span = l;
    *shards = (uint32_t)((n_chunks + (1ull << l) - 1) >> l);
}

/* Page-variant queue budget: bytes/8 of 4-byte entries split evenly over the
 * K classes of each of the S shards, rounded down to a power of two (at
 * least one entry). */
uint64_t orc_page_ring_entries(uint64_t bytes, uint64_t chunk_bytes, uint32_t shards)
{
    uint64_t per = bytes / 8 / orc_num_classes(chunk_bytes) / 4 / shards;
    uint64_t p = 1;
    while (p * 2 <= per) p *= 2;
    return p;
}

/* Chunks one class may own in one shard (page variant). */
uint64_t orc_page_max_chunks(uint64_t bytes, uint64_t chunk_bytes, uint32_t k, uint32_t shards)
{
    return orc_page_ring_entries(bytes, chunk_bytes, shards) / orc_pages_per_chunk(chunk_bytes, k);
}

/* Virtualised array page variant ("Virtualised array and list allocators":
 * queue storage taken on demand).  The page variant's per-shard entry
 * budget (K queues of Q entries) becomes one store of segments of
 * 2^g entries, g = log2(Q) - 3 kept within [4, 10], shared by the shard's
 * queues.  A queue whose class owns P pages spans at most P positions,
 * i.e. at most P / 2^g + 2 segments, plus one being handed back: the
 * shard's classes may own (M - 3K) * 2^g pages together, M = K*Q / 2^g. */
uint32_t orc_va_log2_seg(uint64_t bytes, uint64_t chunk_bytes, uint32_t shards)
{
    uint64_t q = orc_page_ring_entries(bytes, chunk_bytes, shards);
    uint32_t lq = 0;
    while ((1ull << (lq + 1)) <= q) ++lq;
    int g = (int)lq - 3;
    if (g < 4) g = 4;
    if (g > 10) g = 10;
    return (uint32_t)g;
}
uint64_t orc_va_segments(uint64_t bytes, uint64_t chunk_bytes, uint32_t shards)
{
    return (orc_num_classes(chunk_bytes) * orc_page_ring_entries(bytes, chunk_bytes, shards)) >>
           orc_va_log2_seg(bytes, chunk_bytes, shards);
}
uint64_t orc_va_budget(uint64_t bytes, uint64_t chunk_bytes, uint32_t shards)
{
    const uint64_t m = orc_va_segments(bytes, chunk_bytes, shards);
    const uint64_t k3 = 3ull * orc_num_classes(chunk_bytes);
    return m > k3 ? (m - k3) << orc_va_log2_seg(bytes, chunk_bytes, shards) : 0;
}

/* Virtualised array chunk variant: a chunk is listed in at most one queue,
 * so the queues of a shard (span = 2^log2_span chunks) hold at most span
 * entries together.  Segments of 2^g slots, g = log2(span) - 3 kept within
 * [4, 10]; a queue spans at most ceil(span / 2^g) + 2 segments, plus one on
 * its way back: M = ceil(span / 2^g) + 3K per shard never runs out. */
uint32_t orc_va_chunk_log2_seg(uint64_t bytes, uint64_t chunk_bytes, uint32_t shards)
{
    uint32_t S = 1, ls = 0;
    orc_shard_geometry(bytes / chunk_bytes, shards, &S, &ls);
    int g = (int)ls - 3;
    if (g < 4) g = 4;
    if (g > 10) g = 10;
    return (uint32_t)g;
}
uint64_t orc_va_chunk_segments(uint64_t bytes, uint64_t chunk_bytes, uint32_t shards)
{
    uint32_t S = 1, ls = 0;
    orc_shard_geometry(bytes / chunk_bytes, shards, &S, &ls);
    const uint32_t g = orc_va_chunk_log2_seg(bytes, chunk_bytes, shards);
    return (((1ull << ls) + (1ull << g) - 1) >> g) + 3ull * orc_num_classes(chunk_bytes);
}

/* ------------------------------------------------------------------ */
/* small containers                                                    */
/* ------------------------------------------------------------------ */

/* hierarchical bitset: lowest set index in O(levels) */
typedef struct {
    int levels;
    uint64_t n;
    uint64_t* lv[8];
    uint64_t words[8];
} hset;

static void hset_init(hset* s, uint64_t n)
{
    memset(s, 0, sizeof(*s));
    s->n = n;
    uint64_t m = n;
    do {
        uint64_t w = (m + 63) / 64;
        s->words[s->levels] = w;
        s->lv[s->levels] = (uint64_t*)calloc(w ? w : 1, 8);
        s->levels++;
        m = w;
    } while (m > 1);
}
static void hset_free(hset* s) { for (int i = 0; i < s->levels; ++i) free(s->lv[i]); }
static void hset_set(hset* s, uint64_t i)
{
    for (int l = 0; l < s->levels; ++l) {
        uint64_t w = i >> 6, b = i & 63;
        int was = s->lv[l][w] != 0;
        s->lv[l][w] |= 1ull << b;
        if (was) break;
        i = w;
    }
}
static void hset_clear(hset* s, uint64_t i)
{
    for (int l = 0; l < s->levels; ++l) {
        uint64_t w = i >> 6, b = i & 63;
        s->lv[l][w] &= ~(1ull << b);
        if (s->lv[l][w]) break;
        i = w;
    }
}
static int64_t hset_lowest(const hset* s)
{
    int top = s->levels - 1;
    if (!s->lv[top][0]) return -1;
    uint64_t i = 0;
    for (int l = top; l >= 0; --l) {
        uint64_t w = s->lv[l][i];
        i = i * 64 + (uint64_t)__builtin_ctzll(w);
    }
    return (int64_t)i;
}

/* lowest set index >= from at level l (level 0 = the bits themselves) */
static int64_t hset_next_at(const hset* s, int l, uint64_t from)
{
    uint64_t nbits = l == 0 ? s->n : s->words[l - 1];
    if (from >= nbits) return -1;
    uint64_t w = from >> 6;
    uint64_t x = s->lv[l][w] & (~0ull << (from & 63));
    if (x) return (int64_t)(w * 64 + (uint64_t)__builtin_ctzll(x));
    if (l + 1 >= s->levels) return -1;
    int64_t nw = hset_next_at(s, l + 1, w + 1);
    if (nw < 0) return -1;
    return (int64_t)((uint64_t)nw * 64 + (uint64_t)__builtin_ctzll(s->lv[l][nw]));
}

/* growable FIFO of u64 */
typedef struct { uint64_t* a; uint64_t cap, head, len; } fifo;
static void fifo_init(fifo* q) { q->cap = 16; q->a = (uint64_t*)malloc(16 * 8); q->head = q->len = 0; }
static void fifo_free(fifo* q) { free(q->a); }
static void fifo_push(fifo* q, uint64_t v)
{
    if (q->len == q->cap) {
        uint64_t* b = (uint64_t*)malloc(q->cap * 2 * 8);
        for (uint64_t i = 0; i < q->len; ++i) b[i] = q->a[(q->head + i) % q->cap];
        free(q->a);
        q->a = b; q->head = 0; q->cap *= 2;
    }
    q->a[(q->head + q->len) % q->cap] = v;
    q->len++;
}
static uint64_t fifo_pop(fifo* q)
{
    uint64_t v = q->a[q->head];
    q->head = (q->head + 1) % q->cap;
    q->len--;
    return v;
}
static void fifo_clear(fifo* q) { q->head = q->len = 0; }
/* Drop the first occurrence of v, keeping the order of the rest. */
static void fifo_remove(fifo* q, uint64_t v)
{
    uint64_t i = 0;
    while (i < q->len && q->a[(q->head + i) % q->cap] != v) ++i;
    if (i == q->len) return;
    for (; i + 1 < q->len; ++i) q->a[(q->head + i) % q->cap] = q->a[(q->head + i + 1) % q->cap];
    q->len--;
}

/* ------------------------------------------------------------------ */
/* heap state                                                          */
/* ------------------------------------------------------------------ */

#define FREE_CLASS 0xFF

struct orc_heap {
    uint64_t bytes, C, N;
    uint32_t log2C, K, W, S, log2_span;
    int variant, policy;
    uint8_t*  cls;        /* class of each chunk, FREE_CLASS if unowned     */
    uint32_t* cnt;        /* free pages in each owned chunk                  */
    uint64_t* bits;       /* N*W words, bit set = page free                  */
    uint64_t  maxc[ORC_MAX_CLASSES];  /* chunks a class may own per shard    */
    uint64_t  va_budget;              /* va page: pages a shard's classes own */
    uint64_t* owned;      /* S*K: chunks owned per (shard, class)            */
    orc_acct  acct;
    /* LOWEST policy */
    hset free_set;                    /* unowned chunks                      */
    hset avail[ORC_MAX_CLASSES];      /* owned chunks with a free page       */
    /* FIFO policy: per shard a pool segment consumed in order, per (shard,
     * class) a queue of chunk ids (chunk variant) or page offsets (page) */
    uint32_t* pool;
    uint64_t* pool_size;
    uint64_t* pool_next;
    fifo* q;
    /* eager retirement (chunk variant): a chunk whose pages are all free
     * leaves its class at once; FIFO policy: each shard's pool is then a
     * queue, retired chunks joining it at the back */
    int eager;
    fifo* pq;
};

static uint64_t ppc_of(const orc_heap* h, uint32_t k) { return h->C >> (4 + k); }
static uint32_t shard_of(const orc_heap* h, uint64_t c) { return (uint32_t)(c >> h->log2_span); }
static uint64_t shard_first(const orc_heap* h, uint32_t j) { return (uint64_t)j << h->log2_span; }
static uint64_t shard_end(const orc_heap* h, uint32_t j)
{
    uint64_t e = ((uint64_t)j + 1) << h->log2_span;
    return e < h->N ? e : h->N;
}

orc_heap* orc_create_ex(uint64_t bytes, uint64_t chunk_bytes, int variant, int policy, uint32_t shards)
{
    if (!orc_geometry_ok(bytes, chunk_bytes)) return NULL;
    if (variant < ORC_VARIANT_CHUNK || variant > ORC_VARIANT_VL_CHUNK) return NULL;
    if (policy != ORC_POLICY_LOWEST && policy != ORC_POLICY_FIFO) return NULL;
    if (shards > 64 || (shards & (shards - 1))) return NULL;
    orc_heap* h = (orc_heap*)calloc(1, sizeof(orc_heap));
    h->bytes = bytes; h->C = chunk_bytes; h->N = bytes / chunk_bytes;
    h->log2C = (uint32_t)ilog2_u64(chunk_bytes);
    h->K = orc_num_classes(chunk_bytes);
    h->W = (uint32_t)(chunk_bytes / 16 / 64);
    h->variant = variant; h->policy = policy;
    orc_shard_geometry(h->N, shards, &h->S, &h->log2_span);
    h->cls = (uint8_t*)malloc(h->N);
    memset(h->cls, FREE_CLASS, h->N);
    h->cnt = (uint32_t*)calloc(h->N, 4);
    h->bits = (uint64_t*)calloc(h->N * h->W, 8);
    h->owned = (uint64_t*)calloc((uint64_t)h->S * h->K, 8);
    for (uint32_t k = 0; k < h->K; ++k)
        h->maxc[k] = variant == ORC_VARIANT_PAGE ? orc_page_max_chunks(bytes, chunk_bytes, k, h->S) : h->N;
    if (variant == ORC_VARIANT_VA_PAGE || variant == ORC_VARIANT_VL_PAGE) {
        h->va_budget = orc_va_budget(bytes, chunk_bytes, h->S);
        if (h->va_budget == 0) { free(h->cls); free(h->cnt); free(h->bits); free(h->owned); free(h); return NULL; }
    }
    h->acct.n_classes = h->K;
    h->acct.n_chunks = h->N;
    h->acct.free_chunks = h->N;
    if (policy == ORC_POLICY_LOWEST) {
        hset_init(&h->free_set, h->N);
        for (uint64_t c = 0; c < h->N; ++c) hset_set(&h->free_set, c);
        for (uint32_t k = 0; k < h->K; ++k) hset_init(&h->avail[k], h->N);
    } else {
        h->pool = (uint32_t*)malloc(h->N * 4);
        for (uint64_t c = 0; c < h->N; ++c) h->pool[c] = (uint32_t)c;
        h->pool_size = (uint64_t*)calloc(h->S, 8);
        h->pool_next = (uint64_t*)calloc(h->S, 8);
        for (uint32_t j = 0; j < h->S; ++j) h->pool_size[j] = shard_end(h, j) - shard_first(h, j);
        h->q = (fifo*)calloc((uint64_t)h->S * h->K, sizeof(fifo));
        for (uint64_t i = 0; i < (uint64_t)h->S * h->K; ++i) fifo_init(&h->q[i]);
    }
    return h;
}

orc_heap* orc_create(uint64_t bytes, uint64_t chunk_bytes, int variant, int policy)
{
    return orc_create_ex(bytes, chunk_bytes, variant, policy, 1);
}

uint32_t orc_shards(const orc_heap* h) { return h->S; }

void orc_destroy(orc_heap* h)
{
    if (!h) return;
    if (h->policy == ORC_POLICY_LOWEST) {
        hset_free(&h->free_set);
        for (uint32_t k = 0; k < h->K; ++k) hset_free(&h->avail[k]);
    } else {
        free(h->pool); free(h->pool_size); free(h->pool_next);
        for (uint64_t i = 0; i < (uint64_t)h->S * h->K; ++i) fifo_free(&h->q[i]);
        free(h->q);
    }
    if (h->pq) {
        for (uint32_t j = 0; j < h->S; ++j) fifo_free(&h->pq[j]);
        free(h->pq);
    }
    free(h->cls); free(h->cnt); free(h->bits); free(h->owned); free(h);
}

int orc_set_eager(orc_heap* h)
{
    if (h->variant != ORC_VARIANT_CHUNK || h->eager || h->acct.n_alloc_ok || h->acct.n_alloc_null) return -1;
    h->eager = 1;
    if (h->policy == ORC_POLICY_FIFO) {
        h->pq = (fifo*)calloc(h->S, sizeof(fifo));
        for (uint32_t j = 0; j < h->S; ++j) {
            fifo_init(&h->pq[j]);
            for (uint64_t c = shard_first(h, j); c < shard_end(h, j); ++c) fifo_push(&h->pq[j], c);
        }
    }
    return 0;
}

static int bit_get(const orc_heap* h, uint64_t c, uint64_t p) { return (int)((h->bits[c * h->W + (p >> 6)] >> (p & 63)) & 1); }
static void bit_set(orc_heap* h, uint64_t c, uint64_t p) { h->bits[c * h->W + (p >> 6)] |= 1ull << (p & 63); }
static void bit_clr(orc_heap* h, uint64_t c, uint64_t p) { h->bits[c * h->W + (p >> 6)] &= ~(1ull << (p & 63)); }

static int64_t lowest_free_page(const orc_heap* h, uint64_t c)
{
    for (uint32_t w = 0; w < h->W; ++w) {
        uint64_t x = h->bits[c * h->W + w];
        if (x) return (int64_t)(w * 64 + (uint64_t)__builtin_ctzll(x));
    }
    return -1;
}

static int64_t offset_of(const orc_heap* h, uint64_t c, uint32_t k, uint64_t p)
{
    return (int64_t)((c << h->log2C) + p * orc_page_bytes(k));
}

/* Hand a fresh chunk to class k: page 0 is served, the rest become free. */
static void claim_fresh(orc_heap* h, uint64_t c, uint32_t k)
{
    uint64_t ppc = ppc_of(h, k);
    h->cls[c] = (uint8_t)k;
    for (uint64_t p = 1; p < ppc; ++p) bit_set(h, c, p);
    h->cnt[c] = (uint32_t)(ppc - 1);
    h->owned[(uint64_t)shard_of(h, c) * h->K + k]++;
    h->acct.free_chunks--;
    h->acct.chunks[k]++;
    h->acct.free_pages[k] += ppc - 1;
    h->acct.live[k]++;
}

/* Queues of chunk ids (the chunk variants; storage does not change the
 * sequential behaviour) rather than of free pages. */
static int lists_chunks(int variant)
{
    return variant == ORC_VARIANT_CHUNK || variant == ORC_VARIANT_VA_CHUNK || variant == ORC_VARIANT_VL_CHUNK;
}
static int is_va(int variant) { return variant == ORC_VARIANT_VA_PAGE || variant == ORC_VARIANT_VA_CHUNK; }
static int is_vl(int variant) { return variant == ORC_VARIANT_VL_PAGE || variant == ORC_VARIANT_VL_CHUNK; }
static int segmented(int variant) { return is_va(variant) || is_vl(variant); }
static int shared_pages(int variant) { return variant == ORC_VARIANT_VA_PAGE || variant == ORC_VARIANT_VL_PAGE; }

static int can_grow(const orc_heap* h, uint32_t j, uint32_t k)
{
    if (shared_pages(h->variant)) {
        uint64_t pages = 0;
        for (uint32_t kk = 0; kk < h->K; ++kk) pages += h->owned[(uint64_t)j * h->K + kk] * ppc_of(h, kk);
        return pages + ppc_of(h, k) <= h->va_budget;
    }
    return h->owned[(uint64_t)j * h->K + k] < h->maxc[k];
}

static int64_t alloc_lowest(orc_heap* h, uint32_t k)
{
    int64_t c = hset_lowest(&h->avail[k]);
    if (c >= 0) {
        int64_t p = lowest_free_page(h, (uint64_t)c);
        bit_clr(h, (uint64_t)c, (uint64_t)p);
        if (--h->cnt[c] == 0) hset_clear(&h->avail[k], (uint64_t)c);
        h->acct.free_pages[k]--; h->acct.live[k]++;
        return offset_of(h, (uint64_t)c, k, (uint64_t)p);
    }
    /* lowest unowned chunk in a shard where the class may still grow */
    for (uint32_t j = 0; j < h->S; ++j) {
        if (!can_grow(h, j, k)) continue;
        c = hset_next_at(&h->free_set, 0, shard_first(h, j));
        if (c < 0) return -1;
        if ((uint64_t)c >= shard_end(h, j)) { j = shard_of(h, (uint64_t)c) - 1; continue; }
        hset_clear(&h->free_set, (uint64_t)c);
        claim_fresh(h, (uint64_t)c, k);
        if (h->cnt[c] > 0) hset_set(&h->avail[k], (uint64_t)c);
        return offset_of(h, (uint64_t)c, k, 0);
    }
    return -1;
}

/* One device lane alone: its home shard is shard 0; each shard is tried in
 * order, its queue first, then its pool. */
static int64_t alloc_fifo(orc_heap* h, uint32_t k)
{
    for (uint32_t j = 0; j < h->S; ++j) {
        fifo* q = &h->q[(uint64_t)j * h->K + k];
        if (q->len) {
            if (lists_chunks(h->variant)) {
                uint64_t c = fifo_pop(q);
                int64_t p = lowest_free_page(h, c);
                bit_clr(h, c, (uint64_t)p);
                if (--h->cnt[c] > 0) fifo_push(q, c);
                h->acct.free_pages[k]--; h->acct.live[k]++;
                return offset_of(h, c, k, (uint64_t)p);
            } else {
                uint64_t off = fifo_pop(q);
                uint64_t c = off >> h->log2C, p = (off & (h->C - 1)) / orc_page_bytes(k);
                bit_clr(h, c, p);
                h->cnt[c]--;
                h->acct.free_pages[k]--; h->acct.live[k]++;
                return (int64_t)off;
            }
        }
        uint64_t c;
        if (h->pq) {
            if (!can_grow(h, j, k) || !h->pq[j].len) continue;
            c = fifo_pop(&h->pq[j]);
        } else {
            if (!can_grow(h, j, k) || h->pool_next[j] >= h->pool_size[j]) continue;
            c = h->pool[shard_first(h, j) + h->pool_next[j]++];
        }
        claim_fresh(h, c, k);
        if (lists_chunks(h->variant)) {
            if (h->cnt[c] > 0) fifo_push(q, c);
        } else {
            for (uint64_t p = 1; p < ppc_of(h, k); ++p) fifo_push(q, (uint64_t)offset_of(h, c, k, p));
        }
        return offset_of(h, c, k, 0);
    }
    return -1;
}

int64_t orc_alloc(orc_heap* h, uint64_t n)
{
    int k = orc_class_of(n, h->C);
    int64_t r = -1;
    if (k >= 0) r = h->policy == ORC_POLICY_LOWEST ? alloc_lowest(h, (uint32_t)k) : alloc_fifo(h, (uint32_t)k);
    if (r < 0) h->acct.n_alloc_null++; else h->acct.n_alloc_ok++;
    return r;
}

/* Chunk c of class k, all of whose pages are free, becomes unowned (no
 * bits, no count); the caller moves it between the structures of its
 * policy. */
static void unown(orc_heap* h, uint64_t c, uint32_t k)
{
    for (uint32_t w = 0; w < h->W; ++w) h->bits[c * h->W + w] = 0;
    h->cnt[c] = 0;
    h->cls[c] = FREE_CLASS;
    h->owned[(uint64_t)shard_of(h, c) * h->K + k]--;
    h->acct.chunks[k]--;
    h->acct.free_pages[k] -= ppc_of(h, k);
    h->acct.free_chunks++;
}

int orc_free(orc_heap* h, int64_t off)
{
    if (off < 0) return ORC_FREE_NULL;
    uint64_t o = (uint64_t)off;
    if (o >= h->N * h->C) { h->acct.n_free_invalid++; return ORC_FREE_INVALID; }
    uint64_t c = o >> h->log2C;
    if (h->cls[c] == FREE_CLASS) { h->acct.n_free_invalid++; return ORC_FREE_INVALID; }
    uint32_t k = h->cls[c];
    uint64_t in = o & (h->C - 1);
    if (in % orc_page_bytes(k)) { h->acct.n_free_invalid++; return ORC_FREE_INVALID; }
    uint64_t p = in / orc_page_bytes(k);
    if (bit_get(h, c, p)) { h->acct.n_free_double++; return ORC_FREE_DOUBLE; }
    bit_set(h, c, p);
    uint32_t was = h->cnt[c]++;
    h->acct.free_pages[k]++; h->acct.live[k]--; h->acct.n_free_ok++;
    if (h->eager && h->cnt[c] == ppc_of(h, k)) {
        /* eager retirement: the chunk leaves its class (and its queue, if
         * it was listed) and joins its shard's pool */
        unown(h, c, k);
        if (h->policy == ORC_POLICY_LOWEST) {
            hset_clear(&h->avail[k], c);
            hset_set(&h->free_set, c);
        } else {
            if (was > 0) fifo_remove(&h->q[(uint64_t)shard_of(h, c) * h->K + k], c);
            fifo_push(&h->pq[shard_of(h, c)], c);
        }
        return ORC_FREE_OK;
    }
    if (h->policy == ORC_POLICY_LOWEST) {
        if (was == 0) hset_set(&h->avail[k], c);
    } else {
        fifo* q = &h->q[(uint64_t)shard_of(h, c) * h->K + k];
        if (lists_chunks(h->variant)) {
            if (was == 0) fifo_push(q, c);
        } else {
            fifo_push(q, o);
        }
    }
    return ORC_FREE_OK;
}

/* Quiescent trim: chunks whose pages are all free go back to the pool; the
 * pool segments and the queues are rebuilt in ascending order. */
void orc_trim(orc_heap* h)
{
    for (uint64_t c = 0; c < h->N; ++c) {
        if (h->cls[c] == FREE_CLASS) continue;
        uint32_t k = h->cls[c];
        if (h->cnt[c] != ppc_of(h, k)) continue;
        unown(h, c, k);
        if (h->policy == ORC_POLICY_LOWEST) {
            hset_clear(&h->avail[k], c);
            hset_set(&h->free_set, c);
        }
    }
    if (h->policy == ORC_POLICY_FIFO) {
        for (uint32_t j = 0; j < h->S; ++j) {
            h->pool_size[j] = 0; h->pool_next[j] = 0;
            if (h->pq) fifo_clear(&h->pq[j]);
            for (uint64_t c = shard_first(h, j); c < shard_end(h, j); ++c) {
                if (h->cls[c] != FREE_CLASS) continue;
                h->pool[shard_first(h, j) + h->pool_size[j]++] = (uint32_t)c;
                if (h->pq) fifo_push(&h->pq[j], c);
            }
        }
        for (uint64_t i = 0; i < (uint64_t)h->S * h->K; ++i) fifo_clear(&h->q[i]);
        for (uint64_t c = 0; c < h->N; ++c) {
            if (h->cls[c] == FREE_CLASS || h->cnt[c] == 0) continue;
            uint32_t k = h->cls[c];
            fifo* q = &h->q[(uint64_t)shard_of(h, c) * h->K + k];
            if (lists_chunks(h->variant)) {
                fifo_push(q, c);
            } else {
                for (uint64_t p = 0; p < ppc_of(h, k); ++p)
                    if (bit_get(h, c, p)) fifo_push(q, (uint64_t)offset_of(h, c, k, p));
            }
        }
    }
}

void orc_alloc_batch(orc_heap* h, const uint64_t* sizes, int64_t* offs, uint64_t n)
{
    for (uint64_t i = 0; i < n; ++i) offs[i] = orc_alloc(h, sizes[i]);
}

void orc_free_batch(orc_heap* h, const int64_t* offs, uint64_t n, int32_t* status)
{
    for (uint64_t i = 0; i < n; ++i) {
        int s = orc_free(h, offs[i]);
        if (status) status[i] = s;
    }
}

void orc_replay(orc_heap* h, const int64_t* op, uint64_t n, int64_t* out)
{
    for (uint64_t i = 0; i < n; ++i) {
        if (op[i] >= 0) out[i] = orc_alloc(h, (uint64_t)op[i]);
        else out[i] = orc_free(h, out[(uint64_t)(-op[i] - 1)]);
    }
}

void orc_accounting(const orc_heap* h, orc_acct* out) { *out = h->acct; }

/* ------------------------------------------------------------------ */
/* pattern: the 32-bit finaliser of MurmurHash3 (public domain)        */
/* ------------------------------------------------------------------ */

uint32_t orc_fmix32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x85ebca6bu;
    x ^= x >> 13;
    x *= 0xc2b2ae35u;
    x ^= x >> 16;
    return x;
}

uint32_t orc_pattern_word(uint32_t seed, uint32_t req, uint32_t i)
{
    return orc_fmix32(seed ^ orc_fmix32(req) ^ (i * 0x9E3779B9u));
}

void orc_pattern_fill(uint32_t seed, uint32_t req, uint8_t* dst, uint64_t nbytes)
{
    for (uint64_t b = 0; b < nbytes; ++b) {
        uint32_t w = orc_pattern_word(seed, req, (uint32_t)(b / 4));
        dst[b] = (uint8_t)(w >> (8 * (b % 4)));
    }
}

/* Checksum of a block holding the pattern: the 32-bit wrap-around sum of
 * its little-endian words, a partial last word taken with its missing high
 * bytes as zero. */
uint32_t orc_pattern_sum(uint32_t seed, uint32_t req, uint64_t nbytes)
{
    uint32_t s = 0;
    for (uint64_t j = 0; j * 4 < nbytes; ++j) {
        uint32_t w = orc_pattern_word(seed, req, (uint32_t)j);
        const uint64_t have = nbytes - j * 4;
        if (have < 4) w &= (1u << (8 * have)) - 1u;
        s += w;
    }
    return s;
}

void orc_pattern_sums(uint32_t seed, const uint64_t* reqs, const uint64_t* sizes, uint64_t n, uint32_t* out)
{
    for (uint64_t i = 0; i < n; ++i) out[i] = orc_pattern_sum(seed, (uint32_t)reqs[i], sizes[i]);
}

/* ------------------------------------------------------------------ */
/* invariant checker: blocks                                           */
/* ------------------------------------------------------------------ */

typedef struct { uint64_t lo, hi; } ival;
static int ival_cmp(const void* a, const void* b)
{
    const ival* x = (const ival*)a; const ival* y = (const ival*)b;
    return x->lo < y->lo ? -1 : x->lo > y->lo ? 1 : 0;
}

int orc_check_blocks(uint64_t data_bytes, uint64_t chunk_bytes, const uint64_t* sizes,
                     const int64_t* offs, uint64_t n, orc_blocks_report* rep)
{
    memset(rep, 0, sizeof(*rep));
    rep->n = n;
    ival* iv = (ival*)malloc((n ? n : 1) * sizeof(ival));
    uint64_t m = 0;
    for (uint64_t i = 0; i < n; ++i) {
        int k = orc_class_of(sizes[i], chunk_bytes);
        if (offs[i] < 0) {
            rep->n_null++;
            if (k >= 0) rep->n_null_valid++;
            continue;
        }
        rep->n_nonnull++;
        if (k < 0) { rep->n_bad_size_nonnull++; continue; }
        uint64_t s = orc_page_bytes((uint32_t)k), o = (uint64_t)offs[i];
        if (o + s > data_bytes || o >= data_bytes) { rep->n_oob++; continue; }
        if (o % s) rep->n_misaligned++;
        if (o / chunk_bytes != (o + s - 1) / chunk_bytes) rep->n_straddle++;
        rep->live[k]++;
        iv[m].lo = o; iv[m].hi = o + s; m++;
    }
    qsort(iv, m, sizeof(ival), ival_cmp);
    for (uint64_t i = 1; i < m; ++i)
        if (iv[i].lo < iv[i - 1].hi) rep->n_overlap++;
    free(iv);
    return (rep->n_bad_size_nonnull || rep->n_oob || rep->n_misaligned || rep->n_straddle || rep->n_overlap) ? 1 : 0;
}

/* ------------------------------------------------------------------ */
/* invariant checker: snapshot (layout version 4)                      */
/*                                                                     */
/* header (256 B, little-endian):                                      */
/*   0 u32 magic 0x48424850   4 u32 version 4     8 u64 data_bytes     */
/*  16 u32 n_chunks          20 u32 log2_chunk   24 u32 n_classes      */
/*  28 u32 variant           32 u32 words/chunk  36 u32 log2 ring cap  */
/*  40 u32 shards S          44 u32 log2 span    48 u64 off pools      */
/*  56 u64 off classes       64 u64 off chunk_class                    */
/*  72 u64 off chunk_cnt     80 u64 off bits     88 u64 off pool_ids   */
/*  96 u64 off slots        104 u64 total bytes                        */
/* shard j owns chunks [j << span, (j+1) << span) (last one shorter)   */
/* pool block j (128 B): u64 bump, u32 size, u32 first pool index      */
/* class block (j, k) at index j*K + k (512 B): u64 state              */
/*   (H<<32 | C+2^31), u32 head at +128, u32 tail at +256, u64 owned   */
/*   at +384                                                           */
/* chunk_class u8[N] (0xFF unowned), chunk_cnt u32[N], bits u64[W*N]   */
/* (word-major: word w of chunk c at index w*N + c),                   */
/* pool_ids u32[N], slots u32[S*K << log2 ring cap] (0xFFFFFFFF empty) */
/* ring (j, k) at slot index (j*K + k) << log2 ring cap; page-variant  */
/* slots hold the page's byte offset / 16; a page-variant class may    */
/* own at most (ring entries / pages per chunk) chunks of one shard.   */
/* virtualised array variants (2 pages, 3 chunks), header continued:   */
/* 112 u32 log2 seg g  116 u32 log2 dir  120 u32 log2 store            */
/* 124 u32 segments M per shard  128 u64 page budget per shard         */
/* 136 u64 off dirs  144 u64 off taken  152 u64 off stores             */
/* 160 u64 off store slots.  The slot region holds, per shard, M       */
/* segments of 2^g slots (shard j's segment m at slot index            */
/* (j*M + m) << g).  Queue (j, k) finds position p in the segment      */
/* named by its directory entry (p >> g) mod 2^dir, u64 at index       */
/* ((j*K + k) << dir) + that: (p >> g) << 32 | m, all ones if empty;   */
/* taken u32[S*M] counts each segment's consumed slots; store j: a     */
/* 512 B block (u64 state, u32 head +128, u32 tail +256, u64 pages     */
/* the shard's classes own +384) and a ring of 2^store u32 free ids.   */
/* ------------------------------------------------------------------ */

#define SNAP_MAGIC 0x48424850u
#define SLOT_EMPTY 0xFFFFFFFFu

static uint32_t rd32(const uint8_t* p) { uint32_t v; memcpy(&v, p, 4); return v; }
static uint64_t rd64(const uint8_t* p) { uint64_t v; memcpy(&v, p, 8); return v; }

typedef struct {
    uint64_t data_bytes, N;
    uint32_t log2C, K, variant, W, log2q, S, log2_span;
    const uint8_t *pool, *classes, *cls, *cnt, *bits, *pool_ids, *slots;
    /* virtualised array */
    uint32_t g, ldir, lstore, M;
    uint64_t budget;
    const uint8_t *vdir, *vtaken, *vstore, *vslots;
    /* eager retirement */
    uint32_t eager;
    const uint8_t* ct;
} snapview;

static int snap_open(const uint8_t* s, uint64_t len, snapview* v)
{
    if (len < 256 || rd32(s) != SNAP_MAGIC || rd32(s + 4) != 4) return 0;
    v->data_bytes = rd64(s + 8);
    v->N = rd32(s + 16); v->log2C = rd32(s + 20); v->K = rd32(s + 24);
    v->variant = rd32(s + 28); v->W = rd32(s + 32); v->log2q = rd32(s + 36);
    v->S = rd32(s + 40); v->log2_span = rd32(s + 44);
    uint64_t o_pool = rd64(s + 48), o_cl = rd64(s + 56), o_cls = rd64(s + 64), o_cnt = rd64(s + 72);
    uint64_t o_bits = rd64(s + 80), o_pid = rd64(s + 88), o_sl = rd64(s + 96), total = rd64(s + 104);
    if (total > len || v->K == 0 || v->K > ORC_MAX_CLASSES || v->log2C < 12 || v->log2C > 16) return 0;
    if (v->W != (1u << v->log2C) / 1024 || v->data_bytes != (v->N << v->log2C)) return 0;
    if (v->S == 0 || v->log2_span > 31 || ((uint64_t)v->S << v->log2_span) < v->N ||
        ((uint64_t)(v->S - 1) << v->log2_span) >= v->N) return 0;
    v->pool = s + o_pool; v->classes = s + o_cl; v->cls = s + o_cls; v->cnt = s + o_cnt;
    v->bits = s + o_bits; v->pool_ids = s + o_pid; v->slots = s + o_sl;
    if (v->variant > 5) return 0;
    const int var = (int)v->variant;
    if (!segmented(var) && o_sl + (((uint64_t)v->S * v->K) << v->log2q) * 4 > total) return 0;
    if (segmented(var)) {
        v->g = rd32(s + 112); v->ldir = rd32(s + 116); v->lstore = rd32(s + 120); v->M = rd32(s + 124);
        v->budget = rd64(s + 128);
        uint64_t o_dir = rd64(s + 136), o_tk = rd64(s + 144), o_st = rd64(s + 152), o_ss = rd64(s + 160);
        if (v->g < 4 || v->g > 10 || v->ldir > 24 || v->lstore > 24 || v->M == 0 || (1ull << v->lstore) < v->M)
            return 0;
        if (shared_pages(var) && ((uint64_t)v->M << v->g) > ((uint64_t)v->K << v->log2q)) return 0;
        /* chunk queues: a queue spans at most ceil(span / 2^g) + 2 segments */
        const uint64_t per_queue = ((1ull << v->log2_span) + (1ull << v->g) - 1) >> v->g;
        if (lists_chunks(var) && v->M != per_queue + 3ull * v->K) return 0;
        if (is_va(var) && (1ull << v->ldir) < (shared_pages(var) ? (uint64_t)v->M + 3 : per_queue + 3)) return 0;
        if (is_vl(var) && v->ldir != 0) return 0;
        if (o_sl + (((uint64_t)v->S * v->M) << v->g) * 4 > total) return 0;
        const uint64_t dir_words = is_vl(var) ? 2ull * v->S * v->M : ((uint64_t)v->S * v->K) << v->ldir;
        if (o_dir + dir_words * 8 > total || o_tk + (uint64_t)v->S * v->M * 4 > total ||
            o_st + (uint64_t)v->S * 512 > total || o_ss + ((uint64_t)v->S << v->lstore) * 4 > total)
            return 0;
        v->vdir = s + o_dir; v->vtaken = s + o_tk; v->vstore = s + o_st; v->vslots = s + o_ss;
    }
    v->eager = rd32(s + 168);
    v->ct = NULL;
    if (v->eager > 1) return 0;
    if (v->eager) {
        uint64_t o_ct = rd64(s + 176);
        if (var != 0 || v->log2q != v->log2_span + 1 || v->log2q > 28) return 0;
        if (o_ct + 8 * v->N > total || o_pid + 4 * ((uint64_t)v->S << v->log2_span) > o_sl) return 0;
        v->ct = s + o_ct;
    }
    return 1;
}

/* Eager retirement: free pages and token of chunk c. */
#define TOK_NONE 0xFFFFFFFFu
#define TOK_HELD 0xFFFFFFFEu
/* Eager retirement: the count half holds the free pages in bits 0..15 and,
 * in bit 16 + k, whether the chunk has a stale entry in the queue of class k. */
static uint32_t sv_count(const snapview* v, uint64_t c)
{
    return v->ct ? ((uint32_t)rd64(v->ct + c * 8) & 0xFFFFu) : rd32(v->cnt + c * 4);
}
static int sv_stale_flag(const snapview* v, uint64_t c, uint32_t k)
{
    return ((uint32_t)rd64(v->ct + c * 8) >> (16 + k)) & 1u;
}
static uint32_t sv_token(const snapview* v, uint64_t c) { return (uint32_t)(rd64(v->ct + c * 8) >> 32); }

/* Virtualised list: tag and link of segment m of shard j, and the segment
 * holding number sg of queue (j, k), found by walking from the queue's
 * front (UINT32_MAX when the walk breaks: wrong tag, missing link). */
static uint64_t vl_tag(const snapview* v, uint32_t j, uint32_t m) { return rd64(v->vdir + ((uint64_t)j * v->M + m) * 8); }
static uint64_t vl_link(const snapview* v, uint32_t j, uint32_t m)
{
    return rd64(v->vdir + ((uint64_t)v->S * v->M + (uint64_t)j * v->M + m) * 8);
}
static uint32_t vl_find(const snapview* v, uint32_t j, uint32_t k, uint32_t sg)
{
    const uint8_t* cb = v->classes + ((uint64_t)j * v->K + k) * 512;
    const uint64_t f = rd64(cb + 392);
    uint32_t cs = (uint32_t)(f >> 32), cm = (uint32_t)f;
    for (uint32_t guard = 0; guard <= v->M; ++guard) {
        if (cm >= v->M || vl_tag(v, j, cm) != (((uint64_t)k << 32) | cs)) return UINT32_MAX;
        if (cs == sg) return cm;
        const uint64_t nx = vl_link(v, j, cm);
        if (nx == ~0ull) return UINT32_MAX;
        cm = (uint32_t)nx;
        ++cs;
    }
    return UINT32_MAX;
}

/* Entry of queue (j, k) at ring position pos, or SLOT_EMPTY when the
 * position's storage cannot be found (segmented variants: counted as a bad
 * directory or list by the caller's own checks). */
static uint32_t sv_entry(const snapview* v, uint32_t j, uint32_t k, uint32_t pos)
{
    const uint64_t ring = (uint64_t)j * v->K + k;
    if (is_vl((int)v->variant)) {
        const uint32_t m = vl_find(v, j, k, pos >> v->g);
        if (m == UINT32_MAX) return SLOT_EMPTY;
        return rd32(v->slots + ((((uint64_t)j * v->M + m) << v->g) + (pos & ((1u << v->g) - 1u))) * 4);
    }
    if (!is_va((int)v->variant)) {
        const uint64_t Q = 1ull << v->log2q;
        return rd32(v->slots + ((ring << v->log2q) + (pos & (uint32_t)(Q - 1))) * 4);
    }
    const uint32_t sg = pos >> v->g;
    const uint64_t e = rd64(v->vdir + ((ring << v->ldir) + (sg & ((1u << v->ldir) - 1u))) * 8);
    if (e == ~0ull || (uint32_t)(e >> 32) != sg || (uint32_t)e >= v->M) return SLOT_EMPTY;
    return rd32(v->slots + ((((uint64_t)j * v->M + (uint32_t)e) << v->g) + (pos & ((1u << v->g) - 1u))) * 4);
}

/* bitmask word w of chunk c (word-major) */
static uint64_t sv_word(const snapview* v, uint64_t c, uint32_t w) { return rd64(v->bits + ((uint64_t)w * v->N + c) * 8); }

static uint64_t popc_chunk(const snapview* v, uint64_t c)
{
    uint64_t t = 0;
    for (uint32_t w = 0; w < v->W; ++w) t += (uint64_t)__builtin_popcountll(sv_word(v, c, w));
    return t;
}

/* Virtualised array storage at quiescence, shard by shard:
 *  - queue (j, k) with positions [head, tail) uses exactly the segments
 *    s = head >> g, ..., while s << g < tail (a segment is handed back when
 *    all its slots are consumed, installed when its first one is produced);
 *    each names a distinct segment id < M in directory entry s mod 2^dir,
 *    every other entry is empty;
 *  - a used segment's consumed count is its positions below head, a free
 *    one's zero; every slot that holds no position in [head, tail) is empty;
 *  - the store holds exactly the ids no queue uses, once each, with no hold;
 *  - page queues: the pages the shard's classes own equal its committed
 *    count, within the budget; chunk queues keep that count at zero. */
static void check_va(const snapview* v, const uint64_t* chunks_sk, orc_snap_report* rep)
{
    const uint64_t G = 1ull << v->g, D = 1ull << v->ldir, QS = 1ull << v->lstore;
    uint8_t* used = (uint8_t*)malloc(v->M);
    uint8_t* mark = (uint8_t*)malloc(((uint64_t)v->M << v->g) ? ((uint64_t)v->M << v->g) : 1);
    uint32_t* cons = (uint32_t*)malloc((uint64_t)v->M * 4);
    for (uint32_t j = 0; j < v->S; ++j) {
        memset(used, 0, v->M);
        memset(mark, 0, (uint64_t)v->M << v->g);
        memset(cons, 0, (uint64_t)v->M * 4);
        uint64_t pages = 0;
        for (uint32_t k = 0; k < v->K; ++k) {
            const uint64_t ring = (uint64_t)j * v->K + k;
            const uint8_t* cb = v->classes + ring * 512;
            const uint32_t head = rd32(cb + 128), tail = rd32(cb + 256);
            const uint64_t H = head, T = H + (uint32_t)(tail - head);
            if (v->variant == 2) pages += chunks_sk[ring] * ((1ull << v->log2C) >> (4 + k));
            uint8_t* want = (uint8_t*)calloc(D, 1);
            const uint64_t smask = (v->g < 32) ? ((1ull << (32 - v->g)) - 1) : 0;
            for (uint64_t sg = H >> v->g; (sg << v->g) < T; ++sg) {
                const uint64_t di = sg & (D - 1);
                if (want[di]) { rep->bad_vdir++; continue; } /* span beyond the directory */
                want[di] = 1;
                const uint64_t e = rd64(v->vdir + ((ring << v->ldir) + di) * 8);
                if (e == ~0ull || (uint32_t)(e >> 32) != (uint32_t)(sg & smask) || (uint32_t)e >= v->M ||
                    used[(uint32_t)e]) {
                    rep->bad_vdir++;
                    continue;
                }
                const uint32_t m = (uint32_t)e;
                used[m] = 1;
                const uint64_t s0 = sg << v->g;
                cons[m] = (uint32_t)(H > s0 ? (H < s0 + G ? H - s0 : G) : 0);
                for (uint64_t p = s0 > H ? s0 : H; p < s0 + G && p < T; ++p) mark[((uint64_t)m << v->g) + (p - s0)] = 1;
            }
            for (uint64_t di = 0; di < D; ++di)
                if (!want[di] && rd64(v->vdir + ((ring << v->ldir) + di) * 8) != ~0ull) rep->bad_vdir++;
            free(want);
        }
        for (uint32_t m = 0; m < v->M; ++m) {
            if (rd32(v->vtaken + ((uint64_t)j * v->M + m) * 4) != cons[m]) rep->bad_vtaken++;
            for (uint64_t o = 0; o < G; ++o) {
                const uint64_t si = ((uint64_t)m << v->g) + o;
                if (!mark[si] && rd32(v->slots + (((uint64_t)j * v->M << v->g) + si) * 4) != SLOT_EMPTY)
                    rep->bad_ring_entry++;
            }
        }
        const uint8_t* sb = v->vstore + (uint64_t)j * 512;
        const uint64_t st = rd64(sb);
        const uint32_t sh = rd32(sb + 128), stl = rd32(sb + 256);
        const uint32_t n = stl - sh;
        if ((uint32_t)(st >> 32) != 0 || (int64_t)(uint32_t)st - (int64_t)0x80000000u != (int64_t)n || n > QS) {
            rep->bad_vstore++;
        } else {
            const uint8_t* ss = v->vslots + ((uint64_t)j << v->lstore) * 4;
            uint64_t in_store = 0;
            for (uint32_t i = 0; i < QS; ++i) {
                const uint32_t id = rd32(ss + (uint64_t)((sh + i) & (uint32_t)(QS - 1)) * 4);
                if (i >= n) { if (id != SLOT_EMPTY) rep->bad_vstore++; continue; }
                if (id >= v->M || used[id]) { rep->bad_vstore++; continue; }
                used[id] = 2;
                in_store++;
            }
            for (uint32_t m = 0; m < v->M; ++m)
                if (!used[m]) rep->bad_vstore++; /* a segment neither in use nor in the store */
            (void)in_store;
        }
        const uint64_t committed = rd64(sb + 384);
        if (committed != pages || (v->variant == 2 && committed > v->budget)) rep->bad_committed++;
    }
    free(used);
    free(mark);
    free(cons);
}

/* Virtualised list storage at quiescence, shard by shard:
 *  - queue (j, k) is the chain of segments from its front word to its back
 *    word: consecutive numbers, each tagged (k, number), linked one to the
 *    next, the back with no link; every segment sits in at most one chain;
 *  - the front is the segment of head, or -- head on a segment boundary --
 *    the fully consumed segment before it when that is also the back (a
 *    back stays linked for the next producer); the back is the segment of
 *    the last position written (the front for a queue never written);
 *  - the front's consumed count is its positions below head, every other
 *    chained segment's and every free segment's zero; every slot that holds
 *    no position in [head, tail) is empty;
 *  - the store holds exactly the ids no chain uses, once each, with no hold;
 *  - page queues: the pages the shard's classes own equal its committed
 *    count, within the budget; chunk queues keep that count at zero. */
static void check_vl(const snapview* v, const uint64_t* chunks_sk, orc_snap_report* rep)
{
    const uint64_t G = 1ull << v->g, QS = 1ull << v->lstore;
    uint8_t* used = (uint8_t*)malloc(v->M);
    uint8_t* mark = (uint8_t*)malloc(((uint64_t)v->M << v->g) ? ((uint64_t)v->M << v->g) : 1);
    uint32_t* cons = (uint32_t*)malloc((uint64_t)v->M * 4);
    for (uint32_t j = 0; j < v->S; ++j) {
        memset(used, 0, v->M);
        memset(mark, 0, (uint64_t)v->M << v->g);
        memset(cons, 0, (uint64_t)v->M * 4);
        uint64_t pages = 0;
        for (uint32_t k = 0; k < v->K; ++k) {
            const uint64_t ring = (uint64_t)j * v->K + k;
            const uint8_t* cb = v->classes + ring * 512;
            const uint32_t head = rd32(cb + 128), tail = rd32(cb + 256);
            const uint64_t H = head, T = H + (uint32_t)(tail - head);
            if (v->variant == ORC_VARIANT_VL_PAGE) pages += chunks_sk[ring] * ((1ull << v->log2C) >> (4 + k));
            const uint64_t f = rd64(cb + 392), b = rd64(cb + 400);
            const uint32_t fs = (uint32_t)(f >> 32), bs = (uint32_t)(b >> 32), bm = (uint32_t)b;
            const uint32_t hs = (uint32_t)(H >> v->g);
            const int front_ok = fs == hs || (fs + 1 == hs && (H & (G - 1)) == 0 && fs == bs);
            const uint64_t last = T > 0 ? (T - 1) >> v->g : fs;
            const int back_ok = bs == (last > fs ? last : fs);
            if (!front_ok || !back_ok) rep->bad_vdir++;
            /* walk the chain */
            uint32_t cs = fs, cm = (uint32_t)f;
            int ok = 0;
            for (uint32_t guard = 0; guard <= v->M; ++guard) {
                if (cm >= v->M || used[cm] || vl_tag(v, j, cm) != (((uint64_t)k << 32) | cs)) break;
                used[cm] = 1;
                const uint64_t s0 = (uint64_t)cs << v->g;
                cons[cm] = cs == fs ? (uint32_t)(H > s0 ? (H < s0 + G ? H - s0 : G) : 0) : 0;
                for (uint64_t p = s0 > H ? s0 : H; p < s0 + G && p < T; ++p) mark[((uint64_t)cm << v->g) + (p - s0)] = 1;
                const uint64_t nx = vl_link(v, j, cm);
                if (cs == bs) {
                    ok = cm == bm && nx == ~0ull;
                    break;
                }
                if (nx == ~0ull) break;
                cm = (uint32_t)nx;
                ++cs;
            }
            if (!ok) rep->bad_vdir++;
        }
        for (uint32_t m = 0; m < v->M; ++m) {
            if (rd32(v->vtaken + ((uint64_t)j * v->M + m) * 4) != cons[m]) rep->bad_vtaken++;
            for (uint64_t o = 0; o < G; ++o) {
                const uint64_t si = ((uint64_t)m << v->g) + o;
                if (!mark[si] && rd32(v->slots + (((uint64_t)j * v->M << v->g) + si) * 4) != SLOT_EMPTY)
                    rep->bad_ring_entry++;
            }
        }
        const uint8_t* sb = v->vstore + (uint64_t)j * 512;
        const uint64_t st = rd64(sb);
        const uint32_t sh = rd32(sb + 128), stl = rd32(sb + 256);
        const uint32_t n = stl - sh;
        if ((uint32_t)(st >> 32) != 0 || (int64_t)(uint32_t)st - (int64_t)0x80000000u != (int64_t)n || n > QS) {
            rep->bad_vstore++;
        } else {
            const uint8_t* ss = v->vslots + ((uint64_t)j << v->lstore) * 4;
            for (uint32_t i = 0; i < QS; ++i) {
                const uint32_t id = rd32(ss + (uint64_t)((sh + i) & (uint32_t)(QS - 1)) * 4);
                if (i >= n) { if (id != SLOT_EMPTY) rep->bad_vstore++; continue; }
                if (id >= v->M || used[id]) { rep->bad_vstore++; continue; }
                used[id] = 2;
            }
            for (uint32_t m = 0; m < v->M; ++m)
                if (!used[m]) rep->bad_vstore++; /* a segment neither in a chain nor in the store */
        }
        const uint64_t committed = rd64(sb + 384);
        if (committed != pages || (v->variant == ORC_VARIANT_VL_PAGE && committed > v->budget)) rep->bad_committed++;
    }
    free(used);
    free(mark);
    free(cons);
}

int orc_check_snapshot(const uint8_t* snap, uint64_t len, orc_snap_report* rep)
{
    memset(rep, 0, sizeof(*rep));
    snapview v;
    if (!snap_open(snap, len, &v)) { rep->ok_header = 0; return 1; }
    rep->ok_header = 1;
    rep->n_classes = v.K;
    const uint64_t C = 1ull << v.log2C;
    const uint64_t Q = 1ull << v.log2q;
    uint64_t* chunks_sk = (uint64_t*)calloc((uint64_t)v.S * v.K, 8);
    uint64_t* free_s = (uint64_t*)calloc(v.S, 8);

    /* per chunk: class byte, stray bits beyond the class's pages, counts */
    rep->eager = v.eager;
    for (uint64_t c = 0; c < v.N; ++c) {
        uint8_t k = v.cls[c];
        uint32_t cn = sv_count(&v, c);
        uint32_t j = (uint32_t)(c >> v.log2_span);
        if (k == 0xFF) {
            rep->free_chunks++;
            free_s[j]++;
            if (cn != 0 || popc_chunk(&v, c) != 0) rep->bad_free_chunk++;
            if (v.eager && (rd32(v.cnt + c * 4) != 0 || sv_token(&v, c) != TOK_NONE)) rep->bad_free_chunk++;
            continue;
        }
        if (k >= v.K) { rep->bad_class_byte++; continue; }
        uint64_t ppc = C >> (4 + k);
        for (uint32_t w = 0; w < v.W; ++w) {
            uint64_t x = sv_word(&v, c, w);
            uint64_t lo = (uint64_t)w * 64;
            uint64_t valid = lo >= ppc ? 0 : (ppc - lo >= 64 ? ~0ull : ((1ull << (ppc - lo)) - 1));
            if (x & ~valid) rep->bad_stray_bits++;
        }
        uint64_t f = popc_chunk(&v, c);
        if (lists_chunks((int)v.variant) && cn != f) rep->bad_count++;
        if (v.eager) {
            /* at quiescence: no owned chunk is whole (it would have been
             * retired), none is held, and one without free pages has no
             * token (the listed ones are checked with the rings) */
            uint32_t tk = sv_token(&v, c);
            if (tk == TOK_HELD || (cn == 0 && tk != TOK_NONE) || (cn > 0 && tk == TOK_NONE) || rd32(v.cnt + c * 4) != 0)
                rep->bad_count++;
            if (cn >= ppc) rep->whole_owned++;
        }
        rep->chunks[k]++;
        chunks_sk[(uint64_t)j * v.K + k]++;
        rep->free_pages[k] += f;
        rep->live[k] += ppc - f;
    }

    /* pools: shard j's ids[first+bump .. first+size) are exactly its unowned chunks */
    uint8_t* seen = (uint8_t*)calloc(v.N ? v.N : 1, 1);
    for (uint32_t j = 0; j < v.S; ++j) {
        const uint8_t* pb = v.pool + 128ull * j;
        uint64_t bump = rd64(pb), psize = rd32(pb + 8), first = rd32(pb + 12);
        uint64_t lo = (uint64_t)j << v.log2_span, hi = lo + (1ull << v.log2_span);
        if (hi > v.N) hi = v.N;
        if (first != lo || psize > hi - lo) { rep->bad_pool++; continue; }
        if (v.eager) {
            /* pool ring: entries at positions [head, tail) (slot = position
             * mod 2^span) are exactly the shard's unowned chunks; no hold;
             * every other slot empty */
            const uint64_t span = 1ull << v.log2_span;
            uint32_t head = rd32(pb + 16), tail = rd32(pb + 20), used = tail - head;
            int64_t cnt = (int64_t)(uint32_t)bump - (int64_t)0x80000000u;
            if ((bump >> 32) != 0 || cnt != (int64_t)used || used > span || used != free_s[j]) { rep->bad_pool++; continue; }
            for (uint64_t i = 0; i < span; ++i) {
                uint32_t e = rd32(v.pool_ids + (first + ((head + i) & (span - 1))) * 4);
                if (i >= used) {
                    if (e != SLOT_EMPTY) rep->bad_pool++;
                    continue;
                }
                if (e < lo || e >= hi || v.cls[e] != 0xFF || seen[e]) { rep->bad_pool++; continue; }
                seen[e] = 1;
            }
            continue;
        }
        uint64_t start = bump < psize ? bump : psize;
        for (uint64_t i = start; i < psize; ++i) {
            uint32_t c = rd32(v.pool_ids + (first + i) * 4);
            if (c < lo || c >= hi || v.cls[c] != 0xFF || seen[c]) { rep->bad_pool++; continue; }
            seen[c] = 1;
        }
        if (psize - start != free_s[j]) rep->bad_pool++;
    }
    uint64_t sum = rep->free_chunks;
    for (uint32_t k = 0; k < v.K; ++k) sum += rep->chunks[k];
    if (sum != v.N) rep->bad_conservation++;

    /* rings (eager retirement: stale entries counted per chunk) */
    uint8_t* nstale = (uint8_t*)calloc(v.N ? v.N * v.K : 1, 1);
    for (uint32_t j = 0; j < v.S; ++j) {
        uint64_t lo = (uint64_t)j << v.log2_span, hi = lo + (1ull << v.log2_span);
        if (hi > v.N) hi = v.N;
        for (uint32_t k = 0; k < v.K; ++k) {
            const uint64_t ring = (uint64_t)j * v.K + k;
            const uint8_t* cb = v.classes + ring * 512;
            uint64_t state = rd64(cb), owned = rd64(cb + 384);
            uint32_t head = rd32(cb + 128), tail = rd32(cb + 256);
            uint32_t H = (uint32_t)(state >> 32);
            int64_t Cnt = (int64_t)(uint32_t)state - (int64_t)0x80000000u;
            uint32_t used = tail - head;
            const uint64_t cap = segmented((int)v.variant) ? ((uint64_t)v.M << v.g) : Q;
            if (H != 0 || Cnt != (int64_t)used || used > cap) { rep->bad_ring_ctl++; continue; }
            if (!lists_chunks((int)v.variant) && owned != chunks_sk[ring]) rep->bad_owned++;
            if (lists_chunks((int)v.variant) && owned != 0) rep->bad_owned++;
            if (v.variant == 1 && chunks_sk[ring] > (Q >> (v.log2C - 4 - k))) rep->bad_owned++;
            if (!segmented((int)v.variant)) {
                const uint8_t* sl = v.slots + (ring << v.log2q) * 4;
                for (uint64_t i = used; i < Q; ++i) {
                    uint32_t e = rd32(sl + ((uint64_t)((head + (uint32_t)i) & (uint32_t)(Q - 1))) * 4);
                    if (e != SLOT_EMPTY) rep->bad_ring_entry++;
                }
            }
            if (lists_chunks((int)v.variant)) {
                for (uint64_t c = lo; c < hi; ++c) seen[c] = 0;
                for (uint32_t i = 0; i < used; ++i) {
                    uint32_t c = sv_entry(&v, j, k, head + i);
                    if (v.eager && c >= lo && c < hi &&
                        sv_token(&v, c) != ((k << 28) | ((head + i) & 0x0FFFFFFFu))) {
                        /* eager retirement: an entry whose chunk's token names
                         * another listing is stale (dropped when taken) */
                        rep->stale_entries++;
                        if (nstale[(uint64_t)c * v.K + k] < 255) nstale[(uint64_t)c * v.K + k]++;
                        continue;
                    }
                    if (c < lo || c >= hi || v.cls[c] != k || sv_count(&v, c) == 0) { rep->bad_ring_entry++; continue; }
                    if (seen[c]) { rep->bad_ring_dup++; continue; }
                    seen[c] = 1;
                }
                for (uint64_t c = lo; c < hi; ++c)
                    if (v.cls[c] == k && sv_count(&v, c) > 0 && !seen[c]) rep->bad_ring_missing++;
            } else {
                /* page variant: entries are exactly the free pages of class k in shard j */
                uint64_t s = 16ull << k, ppc = C >> (4 + k);
                uint64_t npages = (hi - lo) * ppc;
                uint8_t* pseen = (uint8_t*)calloc(npages ? npages : 1, 1);
                for (uint32_t i = 0; i < used; ++i) {
                    uint64_t off = (uint64_t)sv_entry(&v, j, k, head + i) * 16;
                    uint64_t c = off >> v.log2C;
                    uint64_t in = off & (C - 1);
                    if (off >= v.data_bytes || c < lo || c >= hi || v.cls[c] != k || in % s) { rep->bad_ring_entry++; continue; }
                    uint64_t p = in / s;
                    if (!((sv_word(&v, c, (uint32_t)(p >> 6)) >> (p & 63)) & 1)) { rep->bad_ring_entry++; continue; }
                    uint64_t gi = (c - lo) * ppc + p;
                    if (pseen[gi]) { rep->bad_ring_dup++; continue; }
                    pseen[gi] = 1;
                }
                for (uint64_t c = lo; c < hi; ++c) {
                    if (v.cls[c] != k) continue;
                    for (uint64_t p = 0; p < ppc; ++p)
                        if (((sv_word(&v, c, (uint32_t)(p >> 6)) >> (p & 63)) & 1) && !pseen[(c - lo) * ppc + p])
                            rep->bad_ring_missing++;
                }
                free(pseen);
            }
        }
    }
    /* eager retirement: at most one stale entry per chunk in each queue,
     * and the chunk's bit for that class says whether it has one */
    if (v.eager)
        for (uint64_t c = 0; c < v.N; ++c) {
            if ((uint32_t)rd64(v.ct + c * 8) >> (16 + v.K)) rep->bad_count++;
            for (uint32_t k = 0; k < v.K; ++k) {
                uint8_t n = nstale[c * v.K + k];
                if (n > 1) rep->bad_ring_dup++;
                else if (sv_stale_flag(&v, c, k) != (n == 1)) rep->bad_count++;
            }
        }
    free(nstale);
    if (is_va((int)v.variant)) check_va(&v, chunks_sk, rep);
    if (is_vl((int)v.variant)) check_vl(&v, chunks_sk, rep);
    free(seen);
    free(chunks_sk);
    free(free_s);
    uint64_t bad = rep->bad_class_byte + rep->bad_free_chunk + rep->bad_stray_bits + rep->bad_count + rep->bad_pool +
                   rep->bad_ring_ctl + rep->bad_ring_entry + rep->bad_ring_missing + rep->bad_ring_dup +
                   rep->bad_conservation + rep->bad_owned + rep->bad_vdir + rep->bad_vtaken + rep->bad_vstore +
                   rep->bad_committed;
    return bad ? 1 : 0;
}

uint64_t orc_check_blocks_in_snapshot(const uint8_t* snap, uint64_t len, const uint64_t* sizes,
                                      const int64_t* offs, uint64_t n)
{
    snapview v;
    if (!snap_open(snap, len, &v)) return n ? n : 1;
    const uint64_t C = 1ull << v.log2C;
    uint64_t bad = 0;
    for (uint64_t i = 0; i < n; ++i) {
        if (offs[i] < 0) continue;
        int k = orc_class_of(sizes[i], C);
        uint64_t o = (uint64_t)offs[i];
        if (k < 0 || o >= v.data_bytes) { bad++; continue; }
        uint64_t c = o >> v.log2C, p = (o & (C - 1)) >> (4 + k);
        if (v.cls[c] != (uint8_t)k) { bad++; continue; }
        if ((sv_word(&v, c, (uint32_t)(p >> 6)) >> (p & 63)) & 1) bad++;
    }
    return bad;
}
