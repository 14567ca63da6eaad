/*
 * hbheap_model.c -- step-level model of the concurrent heap algorithm,
 * explored over every interleaving.  TEST INFRASTRUCTURE ONLY (see
 * hbheap_oracle.h): used by tests, never by the product path; it shares no
 * code with the HIP library and restates the algorithm on its own.
 *
 * What is modelled (one shard, one size class, a tiny heap):
 *   - the class queue: a ring of slots with head, tail and a state word
 *     holding H (operations in flight that may still publish) and the count
 *     of published entries; slots are taken by exchange against EMPTY and
 *     filled by compare-and-swap from EMPTY (a taker waits while its slot is
 *     empty, a filler while it is still full);
 *   - per chunk: owner flag, free count (chunk variant) and free-page bits;
 *   - the pool of unowned chunks, consumed by a bump counter; page variant:
 *     the per-class owned-chunk counter and cap;
 *   - "leaders": one per wave, each running a list of aggregated operations
 *     (allocate g pages, free its own pages, free pages handed to it), one
 *     atomic memory step at a time; lanes of one leader act in lane order;
 *   - variant 2, eager retirement of the chunk variant: per chunk a token
 *     (the queue position it is listed at, held, or none) changed together
 *     with its free count, a stale bit per chunk, queue entries taken by
 *     position modulo Q and dropped when no token names them, chunks whose
 *     pages are all free retired to a pool ring (a grouped tail add, puts
 *     and one publish), and refills taken from that ring.
 * Waits are transitions that are disabled until their condition holds, so a
 * deadlock is a state with unfinished leaders and no enabled transition.
 *
 * Checked in every reachable state:
 *   - tokens: a chunk with a positive free count is held exactly once -- in
 *     a slot, by the leader that took it, by a free that raised its count
 *     from zero, or by the refill that is publishing it (chunk variant); a
 *     free page is held exactly once in the same sense (page variant);
 *   - free count <= free bits (chunk variant);
 *   - exact out-of-memory: a leader gives up only when the pool is empty
 *     (or the class cap is reached) and every free page of the class still
 *     reachable is owed to a free that has not finished (so the request can
 *     be ordered before it); with no concurrent frees: nothing is left.
 * Checked in every final state: no hold in flight, count = tail - head,
 * every slot outside [head, tail) empty, every token back in the ring,
 * granted pages distinct and marked allocated, pages conserved.  Variant 2
 * adds: the pool ring holds exactly the unowned chunks; a chunk with free
 * pages is listed at a position in [head, tail) whose slot holds it; at most
 * one stale entry per chunk, and its stale bit set exactly then.
 * Freeze mode stops one leader forever after each of its steps and records
 * where the others can no longer finish (the algorithm's blocking points).
 * Mutations plant known mistakes so the tests can show each check fires.
 */
#include "hbheap_oracle.h"

#include <stdlib.h>
#include <string.h>

#define M_MAXN 4
#define M_MAXP 8
#define M_MAXQ 32
#define M_MAXL 3
#define M_MAXG 4
#define M_MAXOPS 3
#define M_EMPTY 0xFF

typedef orc_model_op model_op;
typedef orc_model_params model_params;
typedef orc_model_result model_result;

enum { OP_NONE = ORC_OP_NONE, OP_ALLOC = ORC_OP_ALLOC, OP_FREE_OWN = ORC_OP_FREE_OWN, OP_FREE_GIVEN = ORC_OP_FREE_GIVEN };
enum {
    MUT_NONE = 0, MUT_NO_HOLD = 1, MUT_REQUEUE_ALWAYS = 2, MUT_FREE_ENQ_ALWAYS = 3,
    MUT_NO_REFUND = 4, MUT_RELEASE_NO_PUB = 5, MUT_PUBLISH_EARLY = 6,
    MUT_DRY_ALWAYS = 7, /* page alloc: first pass without a hold even when it refills */
    MUT_SCAN_NO_POS = 8, /* the out-of-memory look ignores a gap between head and tail */
    MUT_EAGER_EXACT_POS = 9, /* eager: a taker accepts only its exact position (no lap swaps) */
    MUT_EAGER_NO_STALE_FLAG = 11 /* eager: retire leaving a stale entry even with one outstanding */
};
#define TOK_NONE 0xFF
#define TOK_HELD 0xFE

/* ---------------- state ---------------- */

typedef struct {
    uint8_t op, pc, need, served, got, want, h0, i, t0, nrq, took, publish, exhausted, m, gm, bump0;
    uint8_t lastgot;
    uint8_t early;             /* chunk alloc: requeue and release before claiming */
    uint8_t dry;               /* page alloc: the pool looked dry at start */
    uint8_t held;              /* page alloc: this pass holds the queue   */
    uint8_t pass;              /* page alloc: passes made by this op      */
    uint8_t c[M_MAXG];         /* chunk (chunk var.) or page (page var.) per lane */
    int8_t v[M_MAXG];          /* free count read per helper              */
    uint8_t t[M_MAXG];         /* pages this helper serves                */
    uint8_t keep[M_MAXG];      /* helper keeps a token to requeue         */
    uint8_t tok[M_MAXG];       /* helper currently holds a token          */
    uint8_t left[M_MAXG];      /* pages still to claim per helper         */
    uint8_t pick;              /* claim: bits picked by the current lane  */
    uint8_t enq[M_MAXG];       /* free: lane must enqueue                 */
    uint8_t fpend[M_MAXG];     /* free: lane's token not yet in a slot    */
    uint8_t fpub;              /* free: lanes whose entries await publish */
    uint8_t lo_chunk;          /* refill: leftover chunk, M_EMPTY if none */
    uint8_t lo_tok;            /* refill: holds the leftover's token(s)   */
    uint8_t lo_u, lo_n;        /* refill (page var.): leftover page range */
    uint8_t granted[M_MAXOPS][M_MAXG]; /* pages granted by alloc ops      */
    uint8_t ngranted[M_MAXOPS];
    uint8_t failed[M_MAXOPS];  /* requests that got NULL                   */
    /* eager retirement */
    uint8_t dropped;           /* a stale entry was dropped this pass      */
    uint8_t lpos[M_MAXG];      /* queue position a lane lists its chunk at */
    uint8_t ppend[M_MAXG];     /* lane has an entry still to put           */
    uint8_t xtok[M_MAXG], xn[M_MAXG], xst[M_MAXG]; /* free: the retire CAS's expected word */
    uint8_t rq[M_MAXG];        /* chunk a lane retires (M_EMPTY: none)     */
    uint8_t nret, rpos, ret_pc;
    uint8_t pgot, ph0;         /* refill from the pool ring                */
    uint8_t pch[M_MAXG];       /* chunks taken from the pool ring          */
} leader_t;

typedef struct {
    int16_t cnt_pub;           /* published count (C)                      */
    uint8_t H, head, tail, bump, owned;
    uint8_t slot[M_MAXQ];
    uint8_t own[M_MAXN];
    int8_t cnt[M_MAXN];
    uint8_t bits[M_MAXN];
    uint8_t given[M_MAXL][M_MAXG]; /* pages handed to leaders by prefill  */
    uint8_t ngiven[M_MAXL];
    /* eager retirement: per chunk token (TOK_NONE, TOK_HELD or the queue
     * position it is listed at); the pool ring of unowned chunks */
    uint8_t tok[M_MAXN];
    uint8_t stale[M_MAXN];     /* the chunk has a stale entry in the queue */
    uint8_t pslot[M_MAXN];
    uint8_t phead, ptail;
    int8_t pcnt;
    leader_t L[M_MAXL];
} mstate;

typedef struct {
    const model_params* p;
    int Q, N, P, PQ;
    model_result* r;
    /* visited set: open addressing over stored states */
    mstate* tab;
    uint8_t* used;
    uint64_t cap;
    int frozen;                /* freeze: leader never scheduled again, -1 none */
    uint8_t pre[M_MAXN * M_MAXP];      /* prefill pages                   */
    uint8_t pre_given[M_MAXN * M_MAXP];/* handed to a leader that frees it */
    int npre;
} ctx;

static uint64_t hash_state(const mstate* s)
{
    const uint8_t* b = (const uint8_t*)s;
    uint64_t h = 1469598103934665603ull;
    for (size_t i = 0; i < sizeof(mstate); ++i) { h ^= b[i]; h *= 1099511628211ull; }
    return h ^ (h >> 29);
}

/* returns 1 if newly inserted, 0 if seen, -1 if full */
static int visit(ctx* x, const mstate* s)
{
    uint64_t h = hash_state(s) & (x->cap - 1);
    for (uint64_t probe = 0; probe < x->cap; ++probe) {
        uint64_t i = (h + probe) & (x->cap - 1);
        if (!x->used[i]) {
            if ((int64_t)x->r->states >= x->p->max_states) return -1;
            x->used[i] = 1;
            x->tab[i] = *s;
            x->r->states++;
            return 1;
        }
        if (!memcmp(&x->tab[i], s, sizeof(mstate))) return 0;
    }
    return -1;
}

static int popc8(uint8_t v) { return __builtin_popcount(v); }
static uint8_t full_mask(int P) { return (uint8_t)((1u << P) - 1u); }

static void violation(ctx* x, int code, int64_t* which)
{
    x->r->violations++;
    if (which) (*which)++;
    if (!x->r->first_violation) x->r->first_violation = code;
}

/* ---------------- invariants ---------------- */

/* Does an unfinished free still hold entry v (chunk or page) before putting
 * it into a slot? */
static int held_by_free(const ctx* x, const mstate* s, uint8_t v)
{
    for (int l = 0; l < x->p->n_leaders; ++l) {
        const leader_t* L = &s->L[l];
        if (L->pc < 40 || L->pc >= 50) continue;
        for (int i = 0; i < M_MAXG; ++i)
            if (L->fpend[i] && L->c[i] == v) return 1;
    }
    return 0;
}

/* Page variant: page v belongs to an allocation already -- it sits in a
 * slot whose position the allocation reserved (head moved past it), or the
 * allocation took it out of its slot and has not yet cleared its bit. */
static int held_by_alloc(const ctx* x, const mstate* s, uint8_t v)
{
    for (int l = 0; l < x->p->n_leaders; ++l) {
        const leader_t* L = &s->L[l];
        if (L->pc < 20 || L->pc >= 40) continue;
        for (int i = 0; i < M_MAXG; ++i)
            if (L->tok[i] && L->c[i] == v) return 1;
        if (L->pc == 24)
            for (int q = L->i; q < L->got; ++q)
                if (s->slot[(uint8_t)(L->h0 + q) % x->Q] == v) return 1;
    }
    return 0;
}

static void check_tokens(ctx* x, const mstate* s)
{
    int N = x->N, P = x->P;
    if (x->p->variant == 0) {
        int tokens[M_MAXN] = {0};
        for (int q = 0; q < x->Q; ++q)
            if (s->slot[q] != M_EMPTY && s->slot[q] < N) tokens[s->slot[q]]++;
        for (int l = 0; l < x->p->n_leaders; ++l) {
            const leader_t* L = &s->L[l];
            for (int i = 0; i < M_MAXG; ++i) {
                if (L->tok[i] && L->c[i] < N) tokens[L->c[i]]++;
                if (L->fpend[i] && L->c[i] < N) tokens[L->c[i]]++;
            }
            if (L->lo_tok && L->lo_chunk < N) tokens[L->lo_chunk]++;
        }
        for (int c = 0; c < N; ++c) {
            int want = s->cnt[c] > 0 ? 1 : 0;
            if (tokens[c] != want) { violation(x, 10 + c, &x->r->token_violations); return; }
            if (s->cnt[c] > popc8(s->bits[c])) { violation(x, 20 + c, &x->r->token_violations); return; }
            if (!s->own[c] && (s->cnt[c] || s->bits[c])) { violation(x, 30 + c, &x->r->token_violations); return; }
        }
    } else {
        int tokens[M_MAXN * M_MAXP];
        memset(tokens, 0, sizeof(tokens));
        for (int q = 0; q < x->Q; ++q)
            if (s->slot[q] != M_EMPTY && s->slot[q] < N * P) tokens[s->slot[q]]++;
        for (int l = 0; l < x->p->n_leaders; ++l) {
            const leader_t* L = &s->L[l];
            for (int i = 0; i < M_MAXG; ++i) {
                if (L->tok[i] && L->c[i] < N * P) tokens[L->c[i]]++;
                if (L->fpend[i] && L->c[i] < N * P) tokens[L->c[i]]++;
            }
            if (L->lo_tok && L->lo_chunk < N)
                for (int j = L->lo_u; j < L->lo_u + L->lo_n; ++j) tokens[L->lo_chunk * P + j]++;
        }
        for (int c = 0; c < N; ++c)
            for (int pg = 0; pg < P; ++pg) {
                int want = (s->bits[c] >> pg) & 1;
                if (tokens[c * P + pg] != want) { violation(x, 40 + c * P + pg, &x->r->token_violations); return; }
            }
    }
}

/* At a give-up decision (taken with no hold in flight and a published
 * count <= 0): the pool is empty (or the class capped), and every free chunk
 * (chunk variant) or page (page variant) of the class that no unfinished
 * free still holds is covered by an entry that an unfinished free has put
 * but not yet published.  Entries are interchangeable, so such a request can
 * be ordered before those frees take effect; in runs without concurrent
 * frees this is exactly "nothing of the class is left". */
/* What the out-of-memory look waits for: a hold (an operation that may
 * still publish), or a gap between head and tail.  The gap covers takers
 * that over-asked without a hold and have not yet given the excess back:
 * while they have not, the count can read zero although a free published
 * entries meanwhile; those entries still lie between head and tail.  (Head
 * is read before tail: both only grow, so an equal pair means no published
 * entry was left untaken at the moment head was read.) */
static int in_flight(const ctx* x, const mstate* s)
{
    if (s->H != 0) return 1;
    return x->p->mutation != MUT_SCAN_NO_POS && s->head != s->tail;
}

static void check_oom(ctx* x, const mstate* s)
{
    int N = x->N, P = x->P;
    int pool_left = s->bump < N;
    int can_grow = pool_left && (x->p->variant == 0 || s->owned < x->p->maxc);
    if (can_grow) { violation(x, 60, &x->r->oom_violations); return; }
    int visible = 0, pending = 0;
    for (int l = 0; l < x->p->n_leaders; ++l) {
        const leader_t* L = &s->L[l];
        if (L->pc >= 40 && L->pc < 50) pending += popc8(L->fpub);
    }
    for (int c = 0; c < N; ++c) {
        if (!s->own[c]) continue;
        if (x->p->variant == 0) {
            if (s->cnt[c] > 0 && !held_by_free(x, s, (uint8_t)c)) visible++;
        } else {
            for (int pg = 0; pg < P; ++pg)
                if (((s->bits[c] >> pg) & 1) && !held_by_free(x, s, (uint8_t)(c * P + pg)) &&
                    !held_by_alloc(x, s, (uint8_t)(c * P + pg)))
                    visible++;
        }
    }
    if (visible > pending) violation(x, x->p->variant == 0 ? 61 : 62, &x->r->oom_violations);
}


/* ---------------- eager retirement (variant 2) invariants ---------------- */

/* Is leader l in the middle of a free (its current op frees pages)? */
static int in_free(const ctx* x, const mstate* s, int l)
{
    const leader_t* L = &s->L[l];
    if (L->pc == 0 || L->pc == 99 || L->op >= x->p->n_ops[l]) return 0;
    return x->p->ops[l][L->op].kind != OP_ALLOC;
}

/* Every reachable state: free count (less what holders will take off it)
 * within the free bits; an unowned chunk
 * has no bits, count or token; a held token is held by exactly one
 * allocator lane; a chunk with free pages has a token unless a free that
 * owns it is still listing it or a retirement of it is under way; a whole
 * owned chunk is whole only while a free or an allocator is about to
 * retire it. */
static void check_tokens_eager(ctx* x, const mstate* s)
{
    for (int c = 0; c < x->N; ++c) {
        /* a holder takes its pages off the count only when it puts the
         * token back, possibly after clearing their bits */
        int pending = 0;
        for (int l = 0; l < x->p->n_leaders; ++l) {
            const leader_t* L = &s->L[l];
            if (L->pc < 100 || L->pc >= 140) continue;
            for (int i = 0; i < M_MAXG; ++i)
                if (L->tok[i] && L->c[i] == c) pending += L->t[i];
        }
        if (s->cnt[c] < 0 || s->cnt[c] - pending > popc8(s->bits[c])) { violation(x, 80 + c, &x->r->token_violations); return; }
        if (!s->own[c] && (s->cnt[c] || s->bits[c] || s->tok[c] != TOK_NONE)) {
            violation(x, 84 + c, &x->r->token_violations);
            return;
        }
        int holders = 0, listing = 0;
        for (int l = 0; l < x->p->n_leaders; ++l) {
            const leader_t* L = &s->L[l];
            for (int i = 0; i < M_MAXG; ++i) {
                if (L->pc >= 100 && L->pc < 140 && L->tok[i] && L->c[i] == c) holders++;
                if (in_free(x, s, l) && L->c[i] == c && (L->fpend[i] || L->enq[i] == 2)) listing++;
            }
        }
        if ((s->tok[c] == TOK_HELD) != (holders == 1) || holders > 1) { violation(x, 88 + c, &x->r->token_violations); return; }
        if (s->own[c] && s->cnt[c] > 0 && s->tok[c] == TOK_NONE && !listing) {
            violation(x, 92 + c, &x->r->token_violations);
            return;
        }
    }
}

/* A give-up (no hold in flight, no published entry, pool ring empty) with
 * no free under way: no owned chunk may still have a free page. */
static void check_oom_eager(ctx* x, const mstate* s)
{
    if (s->pcnt > 0) { violation(x, 63, &x->r->oom_violations); return; }
    for (int l = 0; l < x->p->n_leaders; ++l)
        if (in_free(x, s, l)) return;
    for (int c = 0; c < x->N; ++c)
        if (s->own[c] && s->cnt[c] > 0) { violation(x, 64, &x->r->oom_violations); return; }
}

/* Final state: the queue and the pool ring are consistent; every owned
 * chunk has count = free bits; one with free pages is
 * listed at a position in [head, tail) whose slot holds it; one without has
 * no token; the pool ring holds exactly the unowned chunks. */
static void check_final_eager(ctx* x, const mstate* s)
{
    const int N = x->N, Q = x->Q, PQ = x->PQ;
    uint8_t used = (uint8_t)(s->tail - s->head);
    if (s->H != 0 || s->cnt_pub != used || used > Q) { violation(x, 100, &x->r->final_violations); return; }
    for (int i = 0; i < Q; ++i) {
        int in = i < used;
        uint8_t e = s->slot[(uint8_t)(s->head + i) % Q];
        if (in != (e != M_EMPTY)) { violation(x, 101, &x->r->final_violations); return; }
    }
    uint8_t pused = (uint8_t)(s->ptail - s->phead);
    if (s->pcnt != pused || pused > PQ) { violation(x, 102, &x->r->final_violations); return; }
    int inpool[M_MAXN] = {0};
    for (int i = 0; i < PQ; ++i) {
        uint8_t e = s->pslot[(uint8_t)(s->phead + i) % PQ];
        if ((i < pused) != (e != M_EMPTY)) { violation(x, 103, &x->r->final_violations); return; }
        if (i < pused) {
            if (e >= N || s->own[e] || inpool[e]) { violation(x, 104, &x->r->final_violations); return; }
            inpool[e] = 1;
        }
    }
    /* at most one stale entry per chunk, and the flag says whether it has one */
    for (int c = 0; c < N; ++c) {
        int nst = 0;
        for (int i = 0; i < used; ++i) {
            uint8_t p = (uint8_t)(s->head + i);
            if (s->slot[p % Q] == c && !(s->own[c] && s->cnt[c] > 0 && s->tok[c] == p)) nst++;
        }
        if (nst > 1 || s->stale[c] != (nst == 1)) { violation(x, 109, &x->r->final_violations); return; }
    }
    for (int c = 0; c < N; ++c) {
        if (!s->own[c]) {
            if (!inpool[c]) { violation(x, 105, &x->r->final_violations); return; }
            continue;
        }
        /* a whole chunk may stay listed (a stale entry of its queue blocked
         * its retirement) */
        if (s->cnt[c] != popc8(s->bits[c])) { violation(x, 106, &x->r->final_violations); return; }
        if (s->cnt[c] == 0) {
            if (s->tok[c] != TOK_NONE) { violation(x, 107, &x->r->final_violations); return; }
            continue;
        }
        uint8_t p = s->tok[c];
        if (p >= TOK_HELD || (uint8_t)(p - s->head) >= used || s->slot[p % Q] != c) {
            violation(x, 108, &x->r->final_violations);
            return;
        }
    }
}

static void check_final(ctx* x, const mstate* s)
{
    if (x->p->variant == 2) {
        check_final_eager(x, s);
        if (x->r->final_violations) return;
    }
    int N = x->N, P = x->P, Q = x->Q;
    uint8_t used = (uint8_t)(s->tail - s->head);
    if (s->H != 0 || s->cnt_pub != used || used > Q) { violation(x, 70, &x->r->final_violations); return; }
    for (int i = used; i < Q; ++i)
        if (s->slot[(uint8_t)(s->head + i) % Q] != M_EMPTY) { violation(x, 71, &x->r->final_violations); return; }
    for (int i = 0; i < used; ++i)
        if (s->slot[(uint8_t)(s->head + i) % Q] == M_EMPTY) { violation(x, 72, &x->r->final_violations); return; }
    /* granted pages still held by their leader: distinct and allocated */
    uint8_t seen[M_MAXN * M_MAXP];
    memset(seen, 0, sizeof(seen));
    int live = 0;
    for (int l = 0; l < x->p->n_leaders; ++l) {
        const leader_t* L = &s->L[l];
        for (int o = 0; o < M_MAXOPS; ++o)
            for (int g = 0; g < L->ngranted[o]; ++g) {
                uint8_t pg = L->granted[o][g];
                if (pg == M_EMPTY) continue;
                if (pg >= N * P || seen[pg]) { violation(x, 73, &x->r->grant_violations); return; }
                seen[pg] = 1;
                live++;
                if ((s->bits[pg / P] >> (pg % P)) & 1) { violation(x, 74, &x->r->grant_violations); return; }
                if (!s->own[pg / P]) { violation(x, 75, &x->r->grant_violations); return; }
            }
    }
    /* prefill pages nobody freed are still allocated */
    for (int i = 0; i < x->npre; ++i) {
        if (x->pre_given[i]) continue;
        if (seen[x->pre[i]]) { violation(x, 76, &x->r->grant_violations); return; }
        seen[x->pre[i]] = 1;
        live++;
    }
    /* conservation: allocated pages = owned chunk pages - free bits */
    int freeb = 0, owned = 0;
    for (int c = 0; c < N; ++c) {
        if (s->own[c]) { owned++; freeb += popc8(s->bits[c]); }
        if (x->p->variant != 1 && s->cnt[c] != popc8(s->bits[c])) { violation(x, 77, &x->r->final_violations); return; }
    }
    if (x->p->variant != 2 && owned != (s->bump < N ? s->bump : N)) { violation(x, 78, &x->r->final_violations); return; }
    if (owned * P - freeb != live) { violation(x, 79, &x->r->final_violations); return; }
    if (x->p->variant == 2) check_tokens_eager(x, s);
    else check_tokens(x, s);
}

/* ---------------- transitions ---------------- */

/* Program counters (per leader):
 *  0 start next op / done when op == n_ops
 *  alloc, chunk variant:
 *   1 reserve  2 refund  3 head  4 take slot(i)  5 read count(i)  6 count add(i)
 *   7 read bits(i)  8 clear bits(i)  9 tail add  10 put slot(i)  11 refill pool
 *  12 refill init  13 refill tail  14 refill put  15 release  16 oom decide
 *  alloc, page variant:
 *  21 reserve  22 refund  23 head  24 take slot(i)  25 clear bit(i)
 *  26 owned reserve (CAS)  27 pool  28 owned give-back  29 refill init  30 refill tail
 *  31 refill put(i)  32 release  33 oom decide
 *  free (both):
 *  40 set bit(i)  41 count add(i)  42 tail add  43 put slot(i)  44 publish
 *  99 done
 */

static int op_count(const ctx* x, int l) { return x->p->n_ops[l]; }

static void start_op(ctx* x, mstate* s, int l)
{
    leader_t* L = &s->L[l];
    if (L->op >= op_count(x, l)) { L->pc = 99; return; }
    const model_op* o = &x->p->ops[l][L->op];
    memset(L->c, M_EMPTY, sizeof(L->c));
    memset(L->tok, 0, sizeof(L->tok));
    memset(L->fpend, 0, sizeof(L->fpend));
    memset(L->enq, 0, sizeof(L->enq));
    L->fpub = 0;
    L->lo_chunk = M_EMPTY;
    L->lo_tok = 0;
    L->i = 0;
    memset(L->rq, M_EMPTY, sizeof(L->rq));
    memset(L->ppend, 0, sizeof(L->ppend));
    L->nret = 0;
    if (o->kind == OP_ALLOC) {
        L->need = (uint8_t)o->a;
        L->served = 0;
        L->ngranted[L->op] = (uint8_t)o->a;
        memset(L->granted[L->op], M_EMPTY, M_MAXG);
        L->pc = x->p->variant == 0 ? 1 : (x->p->variant == 2 ? 100 : 20);
    } else {
        /* the pages to free, one per lane */
        int n = 0;
        if (o->kind == OP_FREE_OWN) {
            int src = o->a;
            for (int g = 0; g < L->ngranted[src]; ++g) L->c[n++] = L->granted[src][g];
            L->ngranted[src] = 0; /* no longer held */
        } else {
            for (int g = 0; g < s->ngiven[l]; ++g) L->c[n++] = s->given[l][g];
        }
        L->need = (uint8_t)n;
        L->pc = 40;
    }
}

static void finish_op(ctx* x, mstate* s, int l)
{
    leader_t* L = &s->L[l];
    L->op++;
    start_op(x, s, l);
}

/* chunk variant helpers */
/* chunks to reserve: ceil(need / ppc) (the wave has at least that many lanes) */
static int want_chunks(const ctx* x, const leader_t* L) { return (L->need + x->P - 1) / x->P; }

/* Execute leader l's next step on s; returns 0 if the step is disabled. */
static int step(ctx* x, mstate* s, int l)
{
    leader_t* L = &s->L[l];
    const int N = x->N, P = x->P, Q = x->Q;
    const int mut = x->p->mutation;
    switch (L->pc) {
    case 0:
        start_op(x, s, l);
        return 1;
    /* ---------------- chunk variant alloc ---------------- */
    case 1: {
        L->want = (uint8_t)want_chunks(x, L);
        int c_old = s->cnt_pub;
        s->cnt_pub -= L->want;
        if (mut != MUT_NO_HOLD) s->H++;
        int got = c_old <= 0 ? 0 : (c_old < L->want ? c_old : L->want);
        L->got = (uint8_t)got;
        L->took = 0;
        L->pc = (got < L->want && mut != MUT_NO_REFUND) ? 2 : 3;
        return 1;
    }
    case 2:
        s->cnt_pub += L->want - L->got;
        L->pc = 3;
        return 1;
    case 3:
        if (L->got) { L->h0 = s->head; s->head = (uint8_t)(s->head + L->got); L->i = 0; L->pc = 4; }
        else { L->nrq = 0; L->pc = 11; }
        return 1;
    case 4: {
        uint8_t* sl = &s->slot[(uint8_t)(L->h0 + L->i) % Q];
        if (*sl == M_EMPTY) return 0;
        L->c[L->i] = *sl;
        *sl = M_EMPTY;
        L->tok[L->i] = 1;
        L->pc = 5;
        return 1;
    }
    case 5: {
        L->v[L->i] = s->cnt[L->c[L->i]];
        if (++L->i < L->got) { L->pc = 4; return 1; }
        /* distribute need over helpers in order */
        int pre = 0;
        for (int i = 0; i < L->got; ++i) {
            int vc = L->v[i] > 0 ? (L->v[i] < L->need ? L->v[i] : L->need) : 0;
            int t = pre < L->need ? ((L->need - pre) < vc ? (L->need - pre) : vc) : 0;
            L->t[i] = (uint8_t)t;
            L->left[i] = (uint8_t)t;
            L->keep[i] = 0;
            pre += vc;
        }
        L->i = 0;
        L->pc = 6;
        return 1;
    }
    case 6: {
        int i = L->i;
        if (L->t[i]) {
            int old = s->cnt[L->c[i]];
            s->cnt[L->c[i]] = (int8_t)(old - L->t[i]);
            L->keep[i] = (uint8_t)((old - L->t[i] > 0) || mut == MUT_REQUEUE_ALWAYS);
        } else {
            L->keep[i] = (uint8_t)(L->v[i] > 0);
        }
        if (!L->keep[i]) L->tok[i] = 0;
        if (++L->i < L->got) return 1;
        L->i = 0;
        /* a pass that will not refill (every reservation served, or the
         * queue gave all it was asked for) puts its kept chunks back and
         * releases the queue first, then claims its pages' bits */
        int sum_t = 0;
        for (int q = 0; q < L->got; ++q) sum_t += L->t[q];
        L->early = (uint8_t)(x->p->early_requeue && !(L->got < L->want && L->need > sum_t));
        L->pc = L->early ? 9 : 7;
        return 1;
    }
    case 7: {
        /* skip helpers with nothing to claim */
        while (L->i < L->got && L->left[L->i] == 0) L->i++;
        if (L->i >= L->got) { L->i = 0; L->pc = L->early ? 18 : 9; return 1; }
        uint8_t x8 = s->bits[L->c[L->i]];
        uint8_t pick = 0;
        for (int b = 0, n = 0; b < P && n < L->left[L->i]; ++b)
            if ((x8 >> b) & 1) { pick |= (uint8_t)(1u << b); n++; }
        if (!pick) return 0; /* wait until the bits become visible */
        L->pick = pick;
        L->pc = 8;
        return 1;
    }
    case 8: {
        uint8_t* w = &s->bits[L->c[L->i]];
        uint8_t won = *w & L->pick;
        *w = (uint8_t)(*w & ~L->pick);
        for (int b = 0; b < P; ++b)
            if ((won >> b) & 1) {
                L->granted[L->op][L->served + L->took] = (uint8_t)(L->c[L->i] * P + b);
                L->took++;
                L->left[L->i]--;
            }
        L->pc = 7;
        return 1;
    }
    case 9: {
        int n = 0;
        for (int i = 0; i < L->got; ++i) n += L->keep[i];
        L->nrq = (uint8_t)n;
        L->need = (uint8_t)(L->need - L->took);
        L->served = (uint8_t)(L->served + L->took);
        if (n) { L->t0 = s->tail; s->tail = (uint8_t)(s->tail + n); L->i = 0; L->pc = 10; return 1; }
        L->publish = 0;
        L->pc = L->early ? 17 : 11;
        return 1;
    }
    case 10: {
        /* put the kept chunks, in helper order, at t0.. */
        int r = 0, i = 0;
        for (i = 0; i < L->got; ++i) {
            if (!L->keep[i]) continue;
            if (L->tok[i]) break;
            r++;
        }
        if (i >= L->got) { L->publish = L->nrq; L->pc = L->early ? 17 : 11; return 1; }
        uint8_t* sl = &s->slot[(uint8_t)(L->t0 + r) % Q];
        if (*sl != M_EMPTY) return 0;
        *sl = L->c[i];
        L->tok[i] = 0;
        return 1;
    }
    case 11: {
        /* refill when the queue was short */
        if (L->pc == 11 && L->got == 0) L->publish = 0;
        if (L->got < L->want && L->need > 0) {
            int m = (L->need + P - 1) / P;
            int b = s->bump;
            if (b < N) s->bump = (uint8_t)(s->bump + m); /* an exhausted pool is only read */
            int gm = b >= N ? 0 : (N - b < m ? N - b : m);
            L->m = (uint8_t)m;
            L->gm = (uint8_t)gm;
            L->bump0 = (uint8_t)b;
            L->exhausted = (uint8_t)(gm < m);
            L->pc = 12;
        } else {
            L->exhausted = 0;
            L->pc = 15;
        }
        return 1;
    }
    case 12: {
        /* class bytes, pages of fully used chunks, leftover init */
        int gm = L->gm;
        int cap = gm * P;
        int r = cap < L->need ? cap : L->need;
        for (int j = 0; j < gm; ++j) s->own[L->bump0 + j] = 1;
        for (int q = 0; q < r; ++q)
            L->granted[L->op][L->served + q] = (uint8_t)((L->bump0 + q / P) * P + q % P);
        if (cap > L->need) {
            int last = L->bump0 + gm - 1;
            int u = L->need - (gm - 1) * P;
            L->lo_chunk = (uint8_t)last;
            if (mut != MUT_PUBLISH_EARLY) {
                s->bits[last] = (uint8_t)(full_mask(P) & ~((1u << u) - 1u));
                s->cnt[last] = (int8_t)(P - u);
            }
            L->lo_u = (uint8_t)u;
            L->lo_tok = 1;
            L->pc = 13;
        } else {
            L->pc = 15;
        }
        L->need = (uint8_t)(L->need - r);
        L->served = (uint8_t)(L->served + r);
        return 1;
    }
    case 13:
        L->t0 = s->tail;
        s->tail = (uint8_t)(s->tail + 1);
        L->pc = 14;
        return 1;
    case 14: {
        uint8_t* sl = &s->slot[L->t0 % Q];
        if (*sl != M_EMPTY) return 0;
        *sl = L->lo_chunk;
        L->lo_tok = 0;
        if (mut == MUT_PUBLISH_EARLY) {
            /* the mistake: bits and count written after the entry is visible */
            s->bits[L->lo_chunk] = (uint8_t)(full_mask(P) & ~((1u << L->lo_u) - 1u));
        }
        L->publish = (uint8_t)(L->publish + 1);
        L->pc = 15;
        return 1;
    }
    case 15:
        s->cnt_pub += (mut == MUT_RELEASE_NO_PUB) ? 0 : L->publish;
        if (mut != MUT_NO_HOLD) s->H--;
        if (mut == MUT_PUBLISH_EARLY && L->lo_chunk != M_EMPTY && s->cnt[L->lo_chunk] == 0 && s->bits[L->lo_chunk])
            s->cnt[L->lo_chunk] = (int8_t)(P - L->lo_u);
        L->lo_chunk = M_EMPTY;
        if (L->need > 0 && L->got < L->want && L->exhausted) { L->pc = 16; return 1; }
        if (L->got > 0 && L->took == 0 && L->need > 0) { L->pc = 16; return 1; }
        if (L->need > 0) { L->pc = 1; return 1; }
        finish_op(x, s, l);
        return 1;
    case 17:
        /* early release: publish the kept chunks, drop the hold, then claim */
        s->cnt_pub += (mut == MUT_RELEASE_NO_PUB) ? 0 : L->publish;
        if (mut != MUT_NO_HOLD) s->H--;
        L->i = 0;
        L->pc = 7;
        return 1;
    case 18:
        /* early pass: the claims are done */
        L->need = (uint8_t)(L->need - L->took);
        L->served = (uint8_t)(L->served + L->took);
        L->early = 0;
        if (L->got > 0 && L->took == 0 && L->need > 0) { L->pc = 16; return 1; }
        if (L->need > 0) { L->pc = 1; return 1; }
        finish_op(x, s, l);
        return 1;
    case 16: {
        /* look again: entries or room -> another pass; otherwise wait while
         * anything is in flight, then give up */
        if (s->cnt_pub > 0 || s->bump < N) { L->pc = 1; return 1; }
        if (in_flight(x, s)) return 0;
        check_oom(x, s);
        L->failed[L->op] = L->need;
        finish_op(x, s, l);
        return 1;
    }
    /* ---------------- page variant alloc ---------------- */
    case 20:
        /* read the pool before the request (the device loads it beside the
         * request size): a dry pool lets the first pass take published
         * entries without holding the queue, since it cannot refill */
        L->pass = 0;
        L->dry = (uint8_t)((x->p->dry_hint && s->bump >= N) || x->p->first_nohold || mut == MUT_DRY_ALWAYS);
        if (L->dry && x->r->dry_starts < 0xFFFFFFFFu) x->r->dry_starts++;
        L->held = (uint8_t)!L->dry;
        L->pc = 21;
        return 1;
    case 21: {
        L->want = L->need;
        int c_old = s->cnt_pub;
        s->cnt_pub -= L->want;
        if (mut != MUT_NO_HOLD && L->held) s->H++;
        int got = c_old <= 0 ? 0 : (c_old < L->want ? c_old : L->want);
        L->got = (uint8_t)got;
        L->pc = (got < L->want && mut != MUT_NO_REFUND) ? 22 : 23;
        return 1;
    }
    case 22:
        s->cnt_pub += L->want - L->got;
        L->pc = 23;
        return 1;
    case 23:
        if (L->got) { L->h0 = s->head; s->head = (uint8_t)(s->head + L->got); L->i = 0; L->pc = 24; }
        else { L->pc = 26; }
        return 1;
    case 24: {
        /* takers read their slots; the bits are cleared afterwards */
        uint8_t* sl = &s->slot[(uint8_t)(L->h0 + L->i) % Q];
        if (*sl == M_EMPTY) return 0;
        L->c[L->i] = *sl;
        *sl = M_EMPTY;
        L->tok[L->i] = 1;
        if (++L->i < L->got) return 1;
        L->i = 0;
        L->pc = 25;
        return 1;
    }
    case 25: {
        /* clear the bits of the taken pages, one lane per step (the device
         * combines lanes of one word into a single atomicAnd) */
        uint8_t pg = L->c[L->i];
        uint8_t bit = (uint8_t)(1u << (pg % P));
        if (!(s->bits[pg / P] & bit)) violation(x, 80, &x->r->token_violations);
        s->bits[pg / P] = (uint8_t)(s->bits[pg / P] & ~bit);
        L->tok[L->i] = 0;
        L->granted[L->op][L->served + L->i] = pg;
        if (++L->i < L->got) return 1;
        L->need = (uint8_t)(L->need - L->got);
        L->served = (uint8_t)(L->served + L->got);
        L->pc = 26;
        return 1;
    }
    case 26:
        L->publish = 0;
        L->exhausted = 0;
        if (L->need == 0) { L->pc = 32; return 1; }
        if (!L->held && mut != MUT_DRY_ALWAYS) { L->exhausted = 1; L->pc = 32; return 1; }
        /* the wave's first pass made for all its groups at once refills
         * nothing: what is still needed is asked for again by a held pass at
         * once where the pool did not look dry, after a look where it did */
        if (x->p->fast_first && L->pass == 0) { L->exhausted = L->dry; L->pc = 32; return 1; }
        L->m = (uint8_t)((L->need + P - 1) / P);
        if (s->bump >= N) { L->gm = 0; L->exhausted = 1; L->pc = 32; return 1; }
        {
            /* reserve room under the cap with compare-and-swap: never above it */
            int o = s->owned;
            int allow = o >= x->p->maxc ? 0 : (x->p->maxc - o < L->m ? x->p->maxc - o : L->m);
            s->owned = (uint8_t)(s->owned + allow);
            L->t0 = (uint8_t)allow;
        }
        L->pc = 27;
        return 1;
    case 27: {
        int allow = L->t0, gm = 0;
        if (allow) {
            int b = s->bump;
            if (b < N) s->bump = (uint8_t)(s->bump + allow);
            gm = b >= N ? 0 : (N - b < allow ? N - b : allow);
            L->bump0 = (uint8_t)b;
        }
        L->gm = (uint8_t)gm;
        L->exhausted = (uint8_t)(gm < L->m);
        L->pc = gm < allow ? 28 : 29;
        return 1;
    }
    case 28:
        /* the pool ran dry: give back the room not used */
        s->owned = (uint8_t)(s->owned - (L->t0 - L->gm));
        L->pc = 29;
        return 1;
    case 29: {
        int gm = L->gm, cap = gm * P;
        int r = cap < L->need ? cap : L->need;
        for (int j = 0; j < gm; ++j) s->own[L->bump0 + j] = 1;
        for (int q = 0; q < r; ++q)
            L->granted[L->op][L->served + q] = (uint8_t)((L->bump0 + q / P) * P + q % P);
        if (cap > L->need) {
            int last = L->bump0 + gm - 1;
            int u = L->need - (gm - 1) * P;
            s->bits[last] = (uint8_t)(full_mask(P) & ~((1u << u) - 1u));
            L->lo_chunk = (uint8_t)last;
            L->lo_u = (uint8_t)u;
            L->lo_n = (uint8_t)(P - u);
            L->lo_tok = 1;
            L->pc = 30;
        } else {
            L->pc = 32;
        }
        L->need = (uint8_t)(L->need - r);
        L->served = (uint8_t)(L->served + r);
        return 1;
    }
    case 30:
        L->t0 = s->tail;
        s->tail = (uint8_t)(s->tail + L->lo_n);
        L->publish = 0;
        L->pc = 31;
        return 1;
    case 31: {
        /* leftover pages go to consecutive slots; the refill holds the rest */
        uint8_t* sl = &s->slot[L->t0 % Q];
        if (*sl != M_EMPTY) return 0;
        *sl = (uint8_t)(L->lo_chunk * P + L->lo_u);
        L->lo_u = (uint8_t)(L->lo_u + 1);
        L->lo_n = (uint8_t)(L->lo_n - 1);
        L->t0 = (uint8_t)(L->t0 + 1);
        L->publish = (uint8_t)(L->publish + 1);
        if (L->lo_n == 0) {
            L->lo_tok = 0;
            L->pc = 32;
        }
        return 1;
    }
    case 32:
        s->cnt_pub += (mut == MUT_RELEASE_NO_PUB) ? 0 : L->publish;
        if (mut != MUT_NO_HOLD && L->held) s->H--;
        L->held = 1; /* later passes hold the queue */
        L->pass = 1;
        L->lo_chunk = M_EMPTY;
        if (L->need > 0 && L->exhausted) { L->pc = 33; return 1; }
        if (L->need > 0) { L->pc = 21; return 1; }
        finish_op(x, s, l);
        return 1;
    case 33: {
        if (s->cnt_pub > 0 || (s->bump < N && s->owned < x->p->maxc)) { L->pc = 21; return 1; }
        if (in_flight(x, s)) return 0;
        check_oom(x, s);
        L->failed[L->op] = L->need;
        finish_op(x, s, l);
        return 1;
    }
    /* ---------------- free (both variants) ---------------- */
    case 40: {
        if (L->i >= L->need) { L->i = 0; L->pc = x->p->variant == 0 ? 41 : (x->p->variant == 2 ? 141 : 42); return 1; }
        uint8_t pg = L->c[L->i];
        if (pg == M_EMPTY) { L->i++; return 1; } /* NULL: nothing to free */
        uint8_t bit = (uint8_t)(1u << (pg % P));
        if (s->bits[pg / P] & bit) {
            /* double free: ignored */
            L->c[L->i] = M_EMPTY;
        } else {
            s->bits[pg / P] |= bit;
            if (x->p->variant == 1) { L->enq[L->i] = 1; L->fpend[L->i] = 1; }
        }
        L->i++;
        return 1;
    }
    case 41: {
        if (L->i >= L->need) { L->i = 0; L->pc = 42; return 1; }
        uint8_t pg = L->c[L->i];
        if (pg != M_EMPTY) {
            int c = pg / P;
            int old = s->cnt[c]++;
            if (old == 0 || mut == MUT_FREE_ENQ_ALWAYS) {
                L->enq[L->i] = 1;
                L->fpend[L->i] = 1;
                L->c[L->i] = (uint8_t)c; /* the entry is the chunk */
            }
        }
        L->i++;
        return 1;
    }
    case 42: {
        int n = 0;
        for (int i = 0; i < L->need; ++i) n += L->enq[i];
        L->nrq = (uint8_t)n;
        if (!n) { finish_op(x, s, l); return 1; }
        L->t0 = s->tail;
        s->tail = (uint8_t)(s->tail + n);
        L->i = 0;
        L->pc = 43;
        return 1;
    }
    case 43: {
        int r = 0, i;
        for (i = 0; i < L->need; ++i) {
            if (!L->enq[i]) continue;
            if (L->fpend[i]) break;
            r++;
        }
        if (i >= L->need) { L->pc = 44; return 1; }
        uint8_t* sl = &s->slot[(uint8_t)(L->t0 + r) % Q];
        if (*sl != M_EMPTY) return 0;
        *sl = L->c[i];
        L->fpend[i] = 0;
        L->fpub |= (uint8_t)(1u << i);
        return 1;
    }
    case 44:
        s->cnt_pub += L->nrq;
        L->fpub = 0;
        finish_op(x, s, l);
        return 1;
    /* ---------------- eager retirement (variant 2): alloc ----------------
     * 100 reserve  101 refund  102 head  103 take slot(i)  104 claim token(i)
     * 105 tail for kept  106 put token back / retire(i)  107 put slot(i)
     * 108 release token(i)  109 tail(i)  110 put token back(i)  131 put slot(i)
     * 132 publish(i)  111 early release  112 pick bits(i)  113 clear bits(i)
     * 118 early pass done  115 refill?  116 pool reserve  117 pool refund
     * 119 pool head  120 take pool slot(i)  121 refill init  122 tail
     * 125 token of the leftover  126 put slot  123 release  124 oom decide */
    case 100: {
        L->want = (uint8_t)want_chunks(x, L);
        int c_old = s->cnt_pub;
        s->cnt_pub -= L->want;
        s->H++;
        int got = c_old <= 0 ? 0 : (c_old < L->want ? c_old : L->want);
        L->got = (uint8_t)got;
        L->took = 0;
        L->dropped = 0;
        L->publish = 0;
        L->nrq = 0;
        L->pc = got < L->want ? 101 : 102;
        return 1;
    }
    case 101:
        s->cnt_pub += L->want - L->got;
        L->pc = 102;
        return 1;
    case 102:
        if (L->got) { L->h0 = s->head; s->head = (uint8_t)(s->head + L->got); L->i = 0; L->pc = 103; }
        else { L->early = 0; L->pc = 115; }
        return 1;
    case 103: {
        uint8_t* sl = &s->slot[(uint8_t)(L->h0 + L->i) % Q];
        if (*sl == M_EMPTY) return 0;
        L->c[L->i] = *sl;
        *sl = M_EMPTY;
        L->pc = 104;
        return 1;
    }
    case 104: {
        /* the token, if it names this position modulo Q, becomes held */
        int i = L->i;
        uint8_t c = L->c[i], tk = s->tok[c], pos = (uint8_t)(L->h0 + i);
        int match = tk < TOK_HELD && (mut == MUT_EAGER_EXACT_POS ? tk == pos : (tk % Q) == (pos % Q));
        if (match) { s->tok[c] = TOK_HELD; L->v[i] = s->cnt[c]; L->tok[i] = 1; }
        else { L->v[i] = 0; L->tok[i] = 0; L->dropped = 1; s->stale[c] = 0; }
        if (++L->i < L->got) { L->pc = 103; return 1; }
        int pre = 0, sum_t = 0;
        for (int q = 0; q < L->got; ++q) {
            int vc = L->v[q] > 0 ? (L->v[q] < L->need ? L->v[q] : L->need) : 0;
            int t = pre < L->need ? ((L->need - pre) < vc ? (L->need - pre) : vc) : 0;
            L->t[q] = (uint8_t)t;
            L->left[q] = (uint8_t)t;
            L->keep[q] = (uint8_t)(L->v[q] > 0 && (t == 0 || L->v[q] > t));
            pre += vc;
            sum_t += t;
        }
        L->early = (uint8_t)!(L->got < L->want && L->need > sum_t);
        L->i = 0;
        L->pc = L->early ? 105 : 112;
        return 1;
    }
    case 105: {
        int n = 0;
        for (int q = 0; q < L->got; ++q)
            if (L->keep[q]) L->lpos[q] = (uint8_t)(s->tail + n++);
        L->nrq = (uint8_t)n;
        s->tail = (uint8_t)(s->tail + n);
        L->i = 0;
        L->pc = 106;
        return 1;
    }
    case 106: {
        int q = L->i;
        while (q < L->got && !(L->keep[q] && L->tok[q])) q++;
        if (q >= L->got) { L->i = 0; L->pc = 108; return 1; }
        uint8_t c = L->c[q];
        int n = s->cnt[c] - L->t[q];
        L->tok[q] = 0;
        L->ppend[q] = 1;
        L->i = (uint8_t)q;
        if (n >= P && (!s->stale[c] || mut == MUT_EAGER_NO_STALE_FLAG)) {
            s->tok[c] = TOK_NONE; s->cnt[c] = 0; s->stale[c] = 1;
            L->rq[q] = c; L->ret_pc = 107; L->pc = 160;
        } else {
            s->tok[c] = L->lpos[q]; s->cnt[c] = (int8_t)n;
            L->pc = 107;
        }
        return 1;
    }
    case 107: {
        uint8_t* sl = &s->slot[L->lpos[L->i] % Q];
        if (*sl != M_EMPTY) return 0;
        *sl = L->c[L->i];
        L->ppend[L->i] = 0;
        L->i++;
        L->pc = 106;
        return 1;
    }
    case 108: {
        int q = L->i;
        while (q < L->got && !(!L->keep[q] && L->tok[q])) q++;
        if (q >= L->got) { L->pc = 111; return 1; }
        uint8_t c = L->c[q];
        if (s->tok[c] == TOK_HELD && s->cnt[c] == L->t[q]) {
            s->cnt[c] = 0; s->tok[c] = TOK_NONE;
            L->tok[q] = 0;
            L->i = (uint8_t)(q + 1);
            return 1;
        }
        L->i = (uint8_t)q;  /* frees came in while it was held: list it after all */
        L->pc = 109;
        return 1;
    }
    case 109:
        L->lpos[L->i] = s->tail;
        s->tail = (uint8_t)(s->tail + 1);
        L->pc = 110;
        return 1;
    case 110: {
        int q = L->i;
        uint8_t c = L->c[q];
        int n = s->cnt[c] - L->t[q];
        L->tok[q] = 0;
        L->ppend[q] = 1;
        if (n >= P && (!s->stale[c] || mut == MUT_EAGER_NO_STALE_FLAG)) {
            s->tok[c] = TOK_NONE; s->cnt[c] = 0; s->stale[c] = 1;
            L->rq[q] = c; L->ret_pc = 131; L->pc = 160;
        } else {
            s->tok[c] = L->lpos[q]; s->cnt[c] = (int8_t)n;
            L->pc = 131;
        }
        return 1;
    }
    case 131: {
        uint8_t* sl = &s->slot[L->lpos[L->i] % Q];
        if (*sl != M_EMPTY) return 0;
        *sl = L->c[L->i];
        L->ppend[L->i] = 0;
        L->pc = 132;
        return 1;
    }
    case 132:
        s->cnt_pub += 1;
        L->i++;
        L->pc = 108;
        return 1;
    case 111:
        if (L->early) {
            s->cnt_pub += L->nrq;
            s->H--;
            L->i = 0;
            L->pc = 112;
        } else {
            L->pc = 115;
        }
        return 1;
    case 112: {
        while (L->i < L->got && L->left[L->i] == 0) L->i++;
        if (L->i >= L->got) { L->i = 0; L->pc = L->early ? 118 : 105; return 1; }
        uint8_t x8 = s->bits[L->c[L->i]];
        uint8_t pick = 0;
        for (int b = 0, n = 0; b < P && n < L->left[L->i]; ++b)
            if ((x8 >> b) & 1) { pick |= (uint8_t)(1u << b); n++; }
        if (!pick) return 0;
        L->pick = pick;
        L->pc = 113;
        return 1;
    }
    case 113: {
        uint8_t* w = &s->bits[L->c[L->i]];
        uint8_t won = *w & L->pick;
        *w = (uint8_t)(*w & ~L->pick);
        for (int b = 0; b < P; ++b)
            if ((won >> b) & 1) {
                L->granted[L->op][L->served + L->took] = (uint8_t)(L->c[L->i] * P + b);
                L->took++;
                L->left[L->i]--;
            }
        L->pc = 112;
        return 1;
    }
    case 118:
        L->need = (uint8_t)(L->need - L->took);
        L->served = (uint8_t)(L->served + L->took);
        L->early = 0;
        if (L->got > 0 && L->took == 0 && !L->dropped && L->need > 0) { L->pc = 124; return 1; }
        if (L->need > 0) { L->pc = 100; return 1; }
        finish_op(x, s, l);
        return 1;
    case 115:
        L->need = (uint8_t)(L->need - L->took);
        L->served = (uint8_t)(L->served + L->took);
        L->publish = L->nrq;
        L->exhausted = 0;
        if (L->got < L->want && L->need > 0) {
            L->m = (uint8_t)((L->need + P - 1) / P);
            L->pc = 116;
        } else {
            L->pc = 123;
        }
        return 1;
    case 116: {
        int c_old = s->pcnt;
        if (c_old <= 0) { L->gm = 0; L->exhausted = 1; L->pc = 123; return 1; }
        s->pcnt = (int8_t)(s->pcnt - L->m);
        L->gm = (uint8_t)(c_old < L->m ? c_old : L->m);
        L->exhausted = (uint8_t)(L->gm < L->m);
        L->pc = L->gm < L->m ? 117 : 119;
        return 1;
    }
    case 117:
        s->pcnt = (int8_t)(s->pcnt + L->m - L->gm);
        L->pc = 119;
        return 1;
    case 119:
        L->ph0 = s->phead;
        s->phead = (uint8_t)(s->phead + L->gm);
        L->i = 0;
        L->pc = 120;
        return 1;
    case 120: {
        if (L->i >= L->gm) { L->pc = 121; return 1; }
        uint8_t* sl = &s->pslot[(uint8_t)(L->ph0 + L->i) % x->PQ];
        if (*sl == M_EMPTY) return 0;
        L->pch[L->i] = *sl;
        *sl = M_EMPTY;
        L->i++;
        return 1;
    }
    case 121: {
        int gm = L->gm, cap = gm * P;
        int r = cap < L->need ? cap : L->need;
        for (int j = 0; j < gm; ++j) s->own[L->pch[j]] = 1;
        for (int q = 0; q < r; ++q)
            L->granted[L->op][L->served + q] = (uint8_t)(L->pch[q / P] * P + q % P);
        if (cap > L->need) {
            uint8_t last = L->pch[gm - 1];
            int u = L->need - (gm - 1) * P;
            L->lo_chunk = last;
            L->lo_u = (uint8_t)u;
            s->bits[last] = (uint8_t)(full_mask(P) & ~((1u << u) - 1u));
            L->lo_tok = 1;
            L->pc = 122;
        } else {
            L->pc = 123;
        }
        L->need = (uint8_t)(L->need - r);
        L->served = (uint8_t)(L->served + r);
        return 1;
    }
    case 122:
        L->t0 = s->tail;
        s->tail = (uint8_t)(s->tail + 1);
        L->pc = 125;
        return 1;
    case 125:
        s->tok[L->lo_chunk] = L->t0;
        s->cnt[L->lo_chunk] = (int8_t)(P - L->lo_u);
        L->pc = 126;
        return 1;
    case 126: {
        uint8_t* sl = &s->slot[L->t0 % Q];
        if (*sl != M_EMPTY) return 0;
        *sl = L->lo_chunk;
        L->lo_tok = 0;
        L->publish = (uint8_t)(L->publish + 1);
        L->pc = 123;
        return 1;
    }
    case 123:
        s->cnt_pub += L->publish;
        s->H--;
        L->lo_chunk = M_EMPTY;
        if (L->need > 0 && L->got < L->want && L->exhausted) { L->pc = 124; return 1; }
        if (L->got > 0 && L->took == 0 && !L->dropped && L->need > 0) { L->pc = 124; return 1; }
        if (L->need > 0) { L->pc = 100; return 1; }
        finish_op(x, s, l);
        return 1;
    case 124:
        if (s->cnt_pub > 0 || s->pcnt > 0) { L->pc = 100; return 1; }
        if (in_flight(x, s)) return 0;
        check_oom_eager(x, s);
        L->failed[L->op] = L->need;
        finish_op(x, s, l);
        return 1;
    /* ---------------- eager retirement (variant 2): free ----------------
     * 40 set bit(i)  141 count add(i)  142 retire CAS(i)  143 tail for owners
     * 144 list or retire(i)  145 put slot(i)  146 publish */
    case 141: {
        if (L->i >= L->need) { L->i = 0; L->pc = 142; return 1; }
        uint8_t pg = L->c[L->i];
        L->enq[L->i] = 0;
        if (pg != M_EMPTY) {
            uint8_t c = (uint8_t)(pg / P);
            int old = s->cnt[c], n = old + 1;
            uint8_t otok = s->tok[c];
            s->cnt[c] = (int8_t)n;
            L->c[L->i] = c;
            L->xst[L->i] = s->stale[c];
            if (otok == TOK_NONE && old == 0) {
                if (n >= P) { L->enq[L->i] = 2; L->xtok[L->i] = TOK_NONE; L->xn[L->i] = (uint8_t)n; }
                else { L->enq[L->i] = 1; L->fpend[L->i] = 1; }
            } else if (otok < TOK_HELD && n >= P && (!s->stale[c] || mut == MUT_EAGER_NO_STALE_FLAG)) {
                L->enq[L->i] = 2; L->xtok[L->i] = otok; L->xn[L->i] = (uint8_t)n;
            }
        }
        L->i++;
        return 1;
    }
    case 142: {
        int q = L->i;
        while (q < L->need && L->enq[q] != 2) q++;
        if (q >= L->need) {
            L->i = 0;
            int n = 0;
            for (int j = 0; j < L->need; ++j) n += L->rq[j] != M_EMPTY;
            if (n) { L->ret_pc = 143; L->pc = 160; } else { L->pc = 143; }
            return 1;
        }
        uint8_t c = L->c[q];
        if (s->tok[c] == L->xtok[q] && s->cnt[c] == L->xn[q] && (s->stale[c] == L->xst[q] || mut == MUT_EAGER_NO_STALE_FLAG)) {
            /* retiring a listed chunk leaves its entry stale */
            if (L->xtok[q] != TOK_NONE) s->stale[c] = 1;
            s->tok[c] = TOK_NONE; s->cnt[c] = 0; L->rq[q] = c;
        }
        L->enq[q] = 0;
        L->i = (uint8_t)(q + 1);
        return 1;
    }
    case 143: {
        int n = 0;
        for (int q = 0; q < L->need; ++q)
            if (L->enq[q] == 1) L->lpos[q] = (uint8_t)(s->tail + n++);
        L->nrq = (uint8_t)n;
        if (!n) { finish_op(x, s, l); return 1; }
        s->tail = (uint8_t)(s->tail + n);
        L->i = 0;
        L->pc = 144;
        return 1;
    }
    case 144: {
        int q = L->i;
        while (q < L->need && !(L->enq[q] == 1 && L->fpend[q])) q++;
        if (q >= L->need) { L->pc = 146; return 1; }
        uint8_t c = L->c[q];
        L->i = (uint8_t)q;
        if (s->cnt[c] >= P && (!s->stale[c] || mut == MUT_EAGER_NO_STALE_FLAG)) {
            s->tok[c] = TOK_NONE; s->cnt[c] = 0; s->stale[c] = 1;
            L->rq[q] = c; L->ret_pc = 145; L->pc = 160;
        } else {
            s->tok[c] = L->lpos[q];
            L->pc = 145;
        }
        return 1;
    }
    case 145: {
        uint8_t* sl = &s->slot[L->lpos[L->i] % Q];
        if (*sl != M_EMPTY) return 0;
        *sl = L->c[L->i];
        L->fpend[L->i] = 0;
        L->fpub |= (uint8_t)(1u << L->i);
        L->i++;
        L->pc = 144;
        return 1;
    }
    case 146:
        s->cnt_pub += L->nrq;
        L->fpub = 0;
        finish_op(x, s, l);
        return 1;
    /* ---------------- eager retirement: the chunks in rq[] go to the pool
     * 160 reset (bits, class)  161 pool tail  162 put pool slot(i)  163 publish */
    case 160: {
        int n = 0;
        for (int q = 0; q < M_MAXG; ++q)
            if (L->rq[q] != M_EMPTY) { s->bits[L->rq[q]] = 0; s->own[L->rq[q]] = 0; n++; }
        L->nret = (uint8_t)n;
        L->pc = n ? 161 : L->ret_pc;
        return 1;
    }
    case 161:
        L->rpos = s->ptail;
        s->ptail = (uint8_t)(s->ptail + L->nret);
        L->pgot = 0;
        L->pc = 162;
        return 1;
    case 162: {
        int q = 0;
        while (q < M_MAXG && L->rq[q] == M_EMPTY) q++;
        if (q >= M_MAXG) { L->pc = 163; return 1; }
        uint8_t* sl = &s->pslot[(uint8_t)(L->rpos + L->pgot) % x->PQ];
        if (*sl != M_EMPTY) return 0;
        *sl = L->rq[q];
        L->rq[q] = M_EMPTY;
        L->pgot++;
        return 1;
    }
    case 163:
        s->pcnt = (int8_t)(s->pcnt + L->nret);
        L->nret = 0;
        L->pc = L->ret_pc;
        return 1;
    default:
        return 0;
    }
}

/* ---------------- exploration ---------------- */

static int all_done(const ctx* x, const mstate* s, int except)
{
    for (int l = 0; l < x->p->n_leaders; ++l)
        if (l != except && s->L[l].pc != 99) return 0;
    return 1;
}

/* Depth-first search with an explicit stack of states. */
typedef struct {
    mstate* a;
    uint64_t n, cap;
} stack_t;

static void push(stack_t* st, const mstate* s)
{
    if (st->n == st->cap) {
        st->cap = st->cap ? st->cap * 2 : 1024;
        st->a = (mstate*)realloc(st->a, st->cap * sizeof(mstate));
    }
    st->a[st->n++] = *s;
}

static void explore(ctx* x, const mstate* init)
{
    stack_t st = {0};
    if (visit(x, init) == 1) push(&st, init);
    while (st.n) {
        mstate s = st.a[--st.n];
        int moved = 0;
        for (int l = 0; l < x->p->n_leaders; ++l) {
            if (l == x->frozen || s.L[l].pc == 99) continue;
            mstate t = s;
            if (!step(x, &t, l)) continue;
            moved = 1;
            if (x->frozen < 0) { if (x->p->variant == 2) check_tokens_eager(x, &t); else check_tokens(x, &t); }
            int v = visit(x, &t);
            if (v < 0) { x->r->truncated = 1; continue; }
            if (v == 1) push(&st, &t);
        }
        if (!moved) {
            if (all_done(x, &s, x->frozen)) {
                if (x->frozen < 0) {
                    x->r->terminals++;
                    check_final(x, &s);
                    for (int l = 0; l < x->p->n_leaders; ++l)
                        for (int o = 0; o < M_MAXOPS; ++o)
                            if (s.L[l].failed[o]) { x->r->null_outcomes++; l = x->p->n_leaders; break; }
                }
            } else if (x->frozen < 0) {
                x->r->deadlocks++;
                violation(x, 90, NULL);
            } else {
                x->r->blocked_freezes++;
                x->r->blocking_pcs |= 1u << (s.L[x->frozen].pc % 32);
                x->r->blocking_set[s.L[x->frozen].pc >> 6] |= 1ull << (s.L[x->frozen].pc & 63);
            }
        }
    }
    free(st.a);
}

static void ctx_tables(ctx* x, uint64_t cap)
{
    x->cap = cap;
    x->tab = (mstate*)malloc(cap * sizeof(mstate));
    x->used = (uint8_t*)calloc(cap, 1);
}

static void ctx_reset(ctx* x) { memset(x->used, 0, x->cap); }

/* Build the initial state: prefill pages allocated one by one by a lone
 * leader (sequential run of the same algorithm), handed out as given pages. */
static int build_init(ctx* x, mstate* s)
{
    memset(s, 0, sizeof(*s));
    memset(s->slot, M_EMPTY, sizeof(s->slot));
    memset(s->given, M_EMPTY, sizeof(s->given));
    /* eager retirement: no tokens; the pool ring holds every chunk */
    memset(s->tok, TOK_NONE, sizeof(s->tok));
    memset(s->pslot, M_EMPTY, sizeof(s->pslot));
    for (int c = 0; c < x->N; ++c) s->pslot[c] = (uint8_t)c;
    s->ptail = (uint8_t)x->N;
    s->pcnt = (int8_t)x->N;
    for (int l = 0; l < M_MAXL; ++l) s->L[l].pc = 0;
    int pages[M_MAXN * M_MAXP];
    int np = 0;
    if (x->p->prefill > 0) {
        /* a sequential allocator run: fresh chunks in order, ring for leftovers */
        model_params solo = *x->p;
        solo.n_leaders = 1;
        solo.n_ops[0] = 1;
        solo.ops[0][0].kind = OP_ALLOC;
        solo.ops[0][0].a = 1;
        solo.mutation = MUT_NONE;
        ctx y = *x;
        y.p = &solo;
        for (int i = 0; i < x->p->prefill; ++i) {
            s->L[0] = (leader_t){0};
            s->L[0].pc = 0;
            int guard = 0;
            while (s->L[0].pc != 99 && guard++ < 10000)
                if (!step(&y, s, 0)) return 0;
            if (s->L[0].granted[0][0] == M_EMPTY || s->L[0].failed[0]) return 0;
            pages[np++] = s->L[0].granted[0][0];
        }
        memset(&s->L[0], 0, sizeof(leader_t));
    }
    /* hand prefill pages to leaders with FREE_GIVEN ops: a = first, b = count */
    x->npre = np;
    for (int i = 0; i < np; ++i) { x->pre[i] = (uint8_t)pages[i]; x->pre_given[i] = 0; }
    for (int l = 0; l < x->p->n_leaders; ++l) {
        s->L[l].pc = 0;
        for (int o = 0; o < x->p->n_ops[l]; ++o) {
            const model_op* op = &x->p->ops[l][o];
            if (op->kind != OP_FREE_GIVEN) continue;
            for (int g = 0; g < op->b && g < M_MAXG; ++g)
                if (op->a + g < np) {
                    s->given[l][s->ngiven[l]++] = (uint8_t)pages[op->a + g];
                    x->pre_given[op->a + g] = 1;
                }
        }
    }
    return 1;
}

int orc_model_run(const orc_model_params* p, orc_model_result* r)
{
    memset(r, 0, sizeof(*r));
    if (p->n_chunks < 1 || p->n_chunks > M_MAXN || p->ppc < 1 || p->ppc > M_MAXP || p->n_leaders < 1 ||
        p->n_leaders > M_MAXL)
        return -1;
    ctx x;
    memset(&x, 0, sizeof(x));
    x.p = p;
    x.r = r;
    x.N = p->n_chunks;
    x.P = p->ppc;
    /* eager retirement: twice the chunks, room for stale entries */
    int entries = p->variant == 0 ? p->n_chunks : (p->variant == 2 ? 2 * p->n_chunks : p->n_chunks * p->ppc);
    x.Q = 1;
    while (x.Q < entries) x.Q *= 2;
    if (x.Q > M_MAXQ) return -1;
    x.PQ = 1;
    while (x.PQ < p->n_chunks) x.PQ *= 2;
    if (p->variant < 0 || p->variant > 2) return -1;
    x.frozen = -1;
    mstate init;
    if (!build_init(&x, &init)) return -2;
    uint64_t cap = 1;
    while (cap < (uint64_t)p->max_states * 2) cap *= 2;
    ctx_tables(&x, cap);
    explore(&x, &init);
    if (p->freeze) {
        /* freeze each leader after each reachable prefix of its own steps:
         * re-explore with the leader never scheduled from chosen states */
        model_result saved = *r;
        for (int l = 0; l < p->n_leaders; ++l) {
            /* collect the reachable states (from the table) and freeze there */
            const int max_roots = 2048;
            mstate* roots = (mstate*)malloc(sizeof(mstate) * max_roots);
            int nroots = 0;
            uint64_t stride = x.r->states / max_roots + 1, seen_n = 0;
            for (uint64_t i = 0; i < x.cap && nroots < max_roots; ++i)
                if (x.used[i] && x.tab[i].L[l].pc != 99 && (seen_n++ % stride) == 0) roots[nroots++] = x.tab[i];
            ctx y = x;
            model_result fr;
            memset(&fr, 0, sizeof(fr));
            y.r = &fr;
            model_params pf = *p;
            pf.max_states = 1 << 16;
            y.p = &pf;
            ctx_tables(&y, 1 << 17);
            y.frozen = l;
            for (int i = 0; i < nroots; ++i) {
                ctx_reset(&y);
                fr.states = 0;
                explore(&y, &roots[i]);
            }
            saved.blocked_freezes += fr.blocked_freezes;
            saved.blocking_pcs |= fr.blocking_pcs;
            for (int q = 0; q < 4; ++q) saved.blocking_set[q] |= fr.blocking_set[q];
            free(y.tab);
            free(y.used);
            free(roots);
        }
        *r = saved;
    }
    free(x.tab);
    free(x.used);
    return 0;
}
