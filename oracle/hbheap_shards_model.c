/*
 * hbheap_shards_model.c -- step-level model of the page variant across
 * several shards, explored over every interleaving.  TEST INFRASTRUCTURE
 * ONLY (see hbheap_oracle.h): used by tests, never by the product path; it
 * shares no code with the HIP library and restates the algorithm on its own.
 *
 * What is modelled: S shards, each with a pool of unowned chunks consumed by
 * a bump counter, a page queue (ring of slots, head, tail, and a state word
 * holding H -- passes that hold the queue and may still publish -- and the
 * published count C) and per-chunk free-page bits; "leaders", one per wave,
 * each running one operation:
 *   - allocate g pages from home shard h (the wave's aggregated group):
 *       serve(h): a first pass that takes published entries without a hold
 *       (C -= need, any excess given back), then passes that look (pool,
 *       room, then state), hold the queue, take, and refill from the shard's
 *       own pool (the refill takes ceil(need / ppc) chunks, serves the group
 *       and publishes the last chunk's other pages: bits, tail add, one slot
 *       per page, then one release that publishes the count and drops the
 *       hold);
 *       with a room cap (the most chunks the class may own in a shard), the
 *       refill first adds the chunks it wants to the shard's room counter,
 *       gives back at once whatever passed the cap, and gives back again
 *       what the pool could not supply;
 *       while pages are missing: scan every shard, reading per shard its
 *       pool bump, room counter, state word, head and tail in that order
 *       (the room counter's place in it is free: a reading at or above the
 *       cap stays true until the pool runs dry); serve the first
 *       shard (from home on) that shows entries or chunks; answer NULL only
 *       when the scan finds every shard with an empty pool, no hold, no
 *       published entry and head = tail; otherwise scan again;
 *   - free pages it was handed: per page, set its bit, reserve a tail
 *       position, fill the slot (wait while the previous lap's entry is still
 *       there), publish (C += 1).
 * Waits are transitions that are disabled until their condition holds.
 *
 * Checked:
 *   - at every NULL answer (the exactness the scan claims): no chunk is left
 *     in any pool, no refill in flight holds pages it has not published, and
 *     every entry between a shard's head and tail lies at or beyond the tail
 *     the scan read for that shard (published after the scan looked there:
 *     by a free) or is still owed to a free that has not finished; with no
 *     frees running this is "nothing is left";
 *   - in every final state: no hold, C = tail - head on every shard, slots
 *     full exactly on [head, tail), the room counter equal to the chunks the
 *     class owns and these within the cap, every page exactly once either granted
 *     (bit clear), or free (bit set) in one slot of its own shard's queue,
 *     or in an unowned chunk (bits clear); granted pages distinct;
 *   - deadlock freedom.
 * Mutations plant known mistakes so the tests can show each check fires.
 */
#include "hbheap_oracle.h"

#include <stdlib.h>
#include <string.h>

#define SM_S 3      /* shards          */
#define SM_C 2      /* chunks per shard */
#define SM_P 4      /* pages per chunk */
#define SM_Q 16     /* ring slots      */
#define SM_L 3      /* leaders         */
#define SM_EMPTY 0xFF

enum {
    SMUT_NONE = 0, SMUT_STATE_FIRST = 1, SMUT_NO_POSITIONS = 2, SMUT_NO_HOLD_CHECK = 3, SMUT_HOME_ONLY = 4,
    SMUT_ROOM_NO_CAP = 5,       /* the refill keeps all it added, past the cap    */
    SMUT_ROOM_KEEP_EXCESS = 6,  /* what passed the cap is never given back        */
    SMUT_ROOM_BACK_ALL = 7,     /* the give-back returns the granted part as well */
};

typedef struct {
    uint8_t bump;           /* chunks taken from the pool                 */
    uint8_t owned;          /* room counter (with a cap)                  */
    int8_t C;               /* published count                             */
    uint8_t H;              /* holds                                       */
    uint8_t head, tail;     /* positions, monotone modulo 256              */
    uint8_t slot[SM_Q];
} shard_t;

/* leader program counters */
enum {
    PC_DONE = 0,
    /* allocation */
    PC_START,       /* read the home pool hint (dry)                       */
    PC_LOOK_POOL,   /* look: pool of shard j                               */
    PC_LOOK_ROOM,   /* look: room counter of shard j (with a cap)          */
    PC_LOOK_STATE,  /* look: state word of shard j                         */
    PC_RESERVE,     /* take_published (no hold) or reserve with a hold     */
    PC_REFUND,      /* give back what the reservation could not cover      */
    PC_HEAD,        /* head add                                            */
    PC_TAKE,        /* take slot h0 + i                                    */
    PC_CLEAR,       /* clear the bits of the pages taken                   */
    PC_POOL,        /* refill: take chunks from the pool (with a cap: the
                       pool look; the take is PC_TAKE_POOL)                */
    PC_ROOM,        /* refill: add the chunks wanted to the room counter   */
    PC_ROOM_BACK,   /* refill: give back what passed the cap               */
    PC_TAKE_POOL,   /* refill: bump the pool by what the room allowed      */
    PC_ROOM_REFUND, /* refill: give back room the pool could not supply    */
    PC_BITS,        /* refill: set the leftover pages' bits                */
    PC_TAIL,        /* refill: tail add                                    */
    PC_PUT,         /* refill: fill slot t0 + k                            */
    PC_RELEASE,     /* publish and drop the hold                           */
    PC_SCAN,        /* scan: read (shard sr, phase)                        */
    /* free */
    PC_F_OR, PC_F_TAIL, PC_F_PUT, PC_F_PUB
};

typedef struct {
    uint8_t pc, kind;
    uint8_t home, j, need, got, h0, i, held, look, dry, check_first, served_before;
    uint8_t rc, rserve, L, t0, k, exhausted;   /* refill chunk (global), pages served, leftover */
    uint8_t m, allow, gm, pb;  /* chunks wanted, allowed by the room, taken; first */
    uint8_t rd_room;        /* scan: the room counter read below the cap   */
    uint8_t taken[SM_P * 2], ntaken;
    uint8_t granted[SM_P * 2], ngranted, failed;
    uint8_t sr, sph, rd_pool, rd_H, rd_head, avail_r, busy;
    int8_t rd_C;
    uint8_t scan_tail[SM_S];
    uint8_t scanned;        /* shards the last complete scan read (bit j)  */
    /* free */
    uint8_t fpages[SM_P * 2], nf, fi, fpos;
    uint8_t in_serve;       /* serve() entered on shard j (0: in the scan loop) */
} sleader_t;

typedef struct {
    shard_t sh[SM_S];
    uint8_t bits[SM_S * SM_C];
    sleader_t L[SM_L];
} sstate;

typedef struct {
    const orc_shards_params* p;
    orc_shards_result* r;
    int S, Cn, P, Q, room;
    sstate* tab;
    uint8_t* used;
    uint64_t cap;
} sctx;

static uint64_t s_hash(const sstate* s)
{
    const uint8_t* b = (const uint8_t*)s;
    uint64_t h = 1469598103934665603ull;
    for (size_t i = 0; i < sizeof(sstate); ++i) { h ^= b[i]; h *= 1099511628211ull; }
    return h ^ (h >> 29);
}

static int s_visit(sctx* x, const sstate* s)
{
    uint64_t h = s_hash(s) & (x->cap - 1);
    for (uint64_t probe = 0; probe < x->cap; ++probe) {
        uint64_t i = (h + probe) & (x->cap - 1);
        if (!x->used[i]) {
            if ((int64_t)x->r->states >= x->p->max_states) return -1;
            x->used[i] = 1;
            x->tab[i] = *s;
            x->r->states++;
            return 1;
        }
        if (!memcmp(&x->tab[i], s, sizeof(sstate))) return 0;
    }
    return -1;
}

static void s_violation(sctx* x, int code, int64_t* which)
{
    x->r->violations++;
    if (which) (*which)++;
    if (!x->r->first_violation) x->r->first_violation = code;
}

/* page id = (shard * Cn + chunk) * P + page */
static int page_shard(const sctx* x, int v) { return v / (x->Cn * x->P); }
static int page_chunk(const sctx* x, int v) { return v / x->P; }           /* global chunk */
static int in_range(uint8_t pos, uint8_t lo, uint8_t hi) { return (uint8_t)(pos - lo) < (uint8_t)(hi - lo); }

/* is page v still owed by a free that has not finished (its bit set, its
 * slot not yet published)? */
static int owed_by_free(const sctx* x, const sstate* s, int v)
{
    for (int l = 0; l < x->p->n_leaders; ++l) {
        const sleader_t* L = &s->L[l];
        if (L->kind != ORC_SOP_FREE || L->pc == PC_DONE) continue;
        for (int q = L->fi; q < L->nf; ++q)
            if (L->fpages[q] == v) return 1;
    }
    return 0;
}

/* The exactness a NULL answer of leader me claims (see the file comment). */
static void check_null(sctx* x, const sstate* s, int me)
{
    const sleader_t* M = &s->L[me];
    int avail = 0;
    for (int j = 0; j < x->S; ++j) {
        const shard_t* sh = &s->sh[j];
        if (sh->bump < x->Cn) {
            /* chunks still in the pool, as far as the cap lets the class take
             * them (the class owns exactly the chunks bumped out of the pool) */
            int chunks = x->Cn - sh->bump;
            if (x->room) {
                const int r = x->room - sh->bump;
                if (r < chunks) chunks = r > 0 ? r : 0;
            }
            avail += chunks * x->P;
        }
        for (uint8_t pos = sh->head; pos != sh->tail; ++pos) {
            const uint8_t v = sh->slot[pos % x->Q];
            if (v == SM_EMPTY) continue;
            /* published after the scan read this shard's tail */
            if (((M->scanned >> j) & 1) && !in_range(pos, sh->head, M->scan_tail[j])) continue;
            if (owed_by_free(x, s, v)) continue;
            avail++;
        }
    }
    for (int l = 0; l < x->p->n_leaders; ++l) {
        const sleader_t* L = &s->L[l];
        if (l == me || L->kind != ORC_SOP_ALLOC || L->rc == SM_EMPTY) continue;
        avail += L->L - L->k; /* leftover pages of a refill not yet in slots */
    }
    if (avail) s_violation(x, 100 + me, &x->r->oom_violations);
}

static void check_final(sctx* x, const sstate* s)
{
    int seen[SM_S * SM_C * SM_P];
    memset(seen, 0, sizeof(seen));
    for (int j = 0; j < x->S; ++j) {
        const shard_t* sh = &s->sh[j];
        if (sh->H || sh->C != (int8_t)(uint8_t)(sh->tail - sh->head)) { s_violation(x, 200 + j, &x->r->final_violations); return; }
        if (x->room && (sh->owned != sh->bump || sh->bump > x->room)) {
            s_violation(x, 260 + j, &x->r->final_violations);
            return;
        }
        for (int q = 0; q < x->Q; ++q) {
            int inside = 0;
            for (uint8_t pos = sh->head; pos != sh->tail; ++pos)
                if (pos % x->Q == q) inside = 1;
            const uint8_t v = sh->slot[q];
            if (inside != (v != SM_EMPTY)) { s_violation(x, 210 + j, &x->r->final_violations); return; }
            if (v != SM_EMPTY) {
                if (page_shard(x, v) != j || !((s->bits[page_chunk(x, v)] >> (v % x->P)) & 1)) {
                    s_violation(x, 220 + j, &x->r->final_violations);
                    return;
                }
                seen[v]++;
            }
        }
    }
    for (int l = 0; l < x->p->n_leaders; ++l) {
        const sleader_t* L = &s->L[l];
        for (int q = 0; q < L->ngranted; ++q) {
            const int v = L->granted[q];
            if ((s->bits[page_chunk(x, v)] >> (v % x->P)) & 1) { s_violation(x, 230, &x->r->grant_violations); return; }
            seen[v]++;
        }
    }
    for (int j = 0; j < x->S; ++j)
        for (int c = 0; c < x->Cn; ++c) {
            const int gc = j * x->Cn + c;
            for (int pg = 0; pg < x->P; ++pg) {
                const int v = gc * x->P + pg;
                const int bit = (s->bits[gc] >> pg) & 1;
                if (c >= s->sh[j].bump) { /* unowned: in the pool */
                    if (bit || seen[v]) { s_violation(x, 240, &x->r->final_violations); return; }
                    continue;
                }
                /* owned: granted now (once), free in one slot, or allocated
                 * before and never freed (prefill pages nobody frees) */
                const int pre_alloc = (x->p->prealloc[j] >> (c * x->P + pg)) & 1;
                int freed = 0;
                for (int l = 0; l < x->p->n_leaders; ++l)
                    for (int q = 0; q < s->L[l].nf; ++q)
                        if (s->L[l].kind == ORC_SOP_FREE && s->L[l].fpages[q] == v) freed = 1;
                const int want = (pre_alloc && !freed) ? 0 : 1;
                if (seen[v] != want) { s_violation(x, 250, &x->r->final_violations); return; }
            }
        }
}

/* The refill took gm chunks from shard L->j's pool, the first at pool
 * position b: serve the group's pages from them in order, and leave the last
 * chunk's other pages to publish. */
static void refill_serve(const sctx* x, sleader_t* L, int b, int gm)
{
    const int cap = gm * x->P;
    const int rr = cap < L->need ? cap : L->need;
    for (int q = 0; q < rr; ++q) {
        const int c = L->j * x->Cn + b + q / x->P;
        L->granted[L->ngranted++] = (uint8_t)(c * x->P + q % x->P);
    }
    L->exhausted = gm < L->m;
    if (cap > L->need) {
        L->rc = (uint8_t)(L->j * x->Cn + b + gm - 1);
        L->rserve = (uint8_t)(L->need - (gm - 1) * x->P);
        L->L = (uint8_t)(x->P - L->rserve);
        L->k = 0;
        L->pc = PC_BITS;
    } else {
        L->L = 0;
        L->rc = SM_EMPTY;
        L->pc = PC_RELEASE;
    }
    L->need = (uint8_t)(L->need - rr);
}

/* leader l takes one step; returns 0 if disabled */
static int step(sctx* x, sstate* s, int l)
{
    sleader_t* L = &s->L[l];
    const int mut = x->p->mutation;
    switch (L->pc) {
    case PC_DONE:
        return 0;
    case PC_START: {
        shard_t* sh = &s->sh[L->home];
        L->dry = sh->bump >= x->Cn;
        L->j = L->home;
        /* serve(home, dry, check_first = 0) */
        L->in_serve = 1;
        L->look = 0;
        L->held = 0;
        L->check_first = 0;
        L->pc = PC_RESERVE;
        return 1;
    }
    case PC_LOOK_POOL:
        L->rd_pool = s->sh[L->j].bump >= x->Cn; /* 1: dry */
        L->pc = x->room && !L->rd_pool ? PC_LOOK_ROOM : PC_LOOK_STATE;
        return 1;
    case PC_LOOK_ROOM:
        if (s->sh[L->j].owned >= x->room) L->rd_pool = 1; /* no room: as good as dry */
        L->pc = PC_LOOK_STATE;
        return 1;
    case PC_LOOK_STATE: {
        const int some = !L->rd_pool || s->sh[L->j].C > 0;
        if (!some) { L->in_serve = 0; L->pc = PC_SCAN; L->sr = 0; L->sph = 0; L->avail_r = SM_EMPTY; L->busy = 0; L->scanned = 0; return 1; }
        L->pc = PC_RESERVE;
        return 1;
    }
    case PC_RESERVE: {
        shard_t* sh = &s->sh[L->j];
        const int c = sh->C;
        L->got = c <= 0 ? 0 : (c < L->need ? (uint8_t)c : L->need);
        sh->C = (int8_t)(sh->C - L->need);
        if (L->held) sh->H++;
        L->pc = L->got < L->need ? PC_REFUND : PC_HEAD;
        return 1;
    }
    case PC_REFUND:
        s->sh[L->j].C = (int8_t)(s->sh[L->j].C + (L->need - L->got));
        L->pc = PC_HEAD;
        return 1;
    case PC_HEAD:
        if (L->got) {
            L->h0 = s->sh[L->j].head;
            s->sh[L->j].head = (uint8_t)(s->sh[L->j].head + L->got);
            L->i = 0;
            L->pc = PC_TAKE;
        } else {
            L->pc = PC_CLEAR;
        }
        return 1;
    case PC_TAKE: {
        uint8_t* sl = &s->sh[L->j].slot[(uint8_t)(L->h0 + L->i) % x->Q];
        if (*sl == SM_EMPTY) return 0; /* producer late: wait */
        L->taken[L->ntaken++] = *sl;
        *sl = SM_EMPTY;
        if (++L->i == L->got) L->pc = PC_CLEAR;
        return 1;
    }
    case PC_CLEAR: {
        for (int q = 0; q < L->ntaken; ++q) {
            const int v = L->taken[q];
            s->bits[page_chunk(x, v)] &= (uint8_t)~(1u << (v % x->P));
            L->granted[L->ngranted++] = (uint8_t)v;
        }
        L->ntaken = 0;
        L->need = (uint8_t)(L->need - L->got);
        L->exhausted = !L->held && L->dry && L->j == L->home && L->check_first == 0;
        if (L->need > 0 && L->held) { L->pc = PC_POOL; return 1; }
        L->L = 0;
        L->pc = PC_RELEASE; /* drops the hold only if the pass held */
        return 1;
    }
    case PC_POOL: {
        shard_t* sh = &s->sh[L->j];
        L->m = (uint8_t)((L->need + x->P - 1) / x->P);
        if (sh->bump >= x->Cn) { /* dry: nothing reserved, nothing taken */
            L->L = 0;
            L->exhausted = 1;
            L->pc = PC_RELEASE;
            return 1;
        }
        if (x->room) { /* the look above; the room and the take are steps of their own */
            L->pc = PC_ROOM;
            return 1;
        }
        const int b = sh->bump, gm = x->Cn - b < L->m ? x->Cn - b : L->m;
        sh->bump = (uint8_t)(b + gm);
        refill_serve(x, L, b, gm);
        return 1;
    }
    case PC_ROOM: {
        /* add first; what passed the cap goes back in the next step */
        shard_t* sh = &s->sh[L->j];
        const int o = sh->owned;
        sh->owned = (uint8_t)(o + L->m);
        int allow = o + L->m <= x->room ? L->m : (o < x->room ? x->room - o : 0);
        if (mut == SMUT_ROOM_NO_CAP) allow = L->m;
        L->allow = (uint8_t)allow;
        L->pc = allow < L->m ? PC_ROOM_BACK : PC_TAKE_POOL;
        return 1;
    }
    case PC_ROOM_BACK: {
        shard_t* sh = &s->sh[L->j];
        if (mut == SMUT_ROOM_BACK_ALL) sh->owned = (uint8_t)(sh->owned - L->m);
        else if (mut != SMUT_ROOM_KEEP_EXCESS) sh->owned = (uint8_t)(sh->owned - (L->m - L->allow));
        if (!L->allow) { /* no room: no take */
            L->L = 0;
            L->exhausted = 1;
            L->pc = PC_RELEASE;
            return 1;
        }
        L->pc = PC_TAKE_POOL;
        return 1;
    }
    case PC_TAKE_POOL: {
        shard_t* sh = &s->sh[L->j];
        const int b = sh->bump;
        const int gm = b >= x->Cn ? 0 : (x->Cn - b < L->allow ? x->Cn - b : L->allow);
        sh->bump = (uint8_t)(b + gm);
        L->gm = (uint8_t)gm;
        L->pb = (uint8_t)b;
        if (gm < L->allow) { L->pc = PC_ROOM_REFUND; return 1; }
        refill_serve(x, L, b, gm);
        return 1;
    }
    case PC_ROOM_REFUND: {
        /* the pool ran dry under the reservation: give back the rest */
        shard_t* sh = &s->sh[L->j];
        sh->owned = (uint8_t)(sh->owned - (L->allow - L->gm));
        refill_serve(x, L, L->pb, L->gm);
        return 1;
    }
    case PC_BITS:
        for (int pg = L->rserve; pg < x->P; ++pg) s->bits[L->rc] |= (uint8_t)(1u << pg);
        L->pc = PC_TAIL;
        return 1;
    case PC_TAIL:
        L->t0 = s->sh[L->j].tail;
        s->sh[L->j].tail = (uint8_t)(s->sh[L->j].tail + L->L);
        L->pc = PC_PUT;
        return 1;
    case PC_PUT: {
        uint8_t* sl = &s->sh[L->j].slot[(uint8_t)(L->t0 + L->k) % x->Q];
        if (*sl != SM_EMPTY) return 0; /* previous lap not consumed: wait */
        *sl = (uint8_t)(L->rc * x->P + L->rserve + L->k);
        if (++L->k == L->L) { L->rc = SM_EMPTY; L->pc = PC_RELEASE; }
        return 1;
    }
    case PC_RELEASE: {
        shard_t* sh = &s->sh[L->j];
        if (L->held) {
            sh->C = (int8_t)(sh->C + L->L);
            sh->H--;
        }
        L->L = 0;
        L->k = 0;
        if (L->need == 0) { L->pc = PC_DONE; return 1; }
        if (L->exhausted) { L->in_serve = 0; L->pc = PC_SCAN; L->sr = 0; L->sph = 0; L->avail_r = SM_EMPTY; L->busy = 0; L->scanned = 0; return 1; }
        /* the serve loop's next pass: look, then hold */
        L->held = 1;
        L->pc = PC_LOOK_POOL;
        return 1;
    }
    case PC_SCAN: {
        /* shard sr positions after home; phases read pool, room counter (with
         * a cap), state, head, tail (the planted mistake reads the state word
         * before the pool) */
        const int S = mut == SMUT_HOME_ONLY ? 1 : x->S;
        const int j = (L->home + L->sr) % x->S;
        const shard_t* sh = &s->sh[j];
        int phase = L->sph;
        if (mut == SMUT_STATE_FIRST && (phase == 0 || phase == 2)) phase = 2 - phase;
        switch (phase) {
        case 0: L->rd_pool = sh->bump >= x->Cn; break;
        case 1: L->rd_room = sh->owned < x->room; break;
        case 2: L->rd_H = sh->H; L->rd_C = sh->C; break;
        case 3: L->rd_head = sh->head; break;
        case 4: {
            const uint8_t tl = sh->tail;
            L->scan_tail[j] = tl;
            L->scanned |= (uint8_t)(1u << j);
            int hold = L->rd_H != 0 && mut != SMUT_NO_HOLD_CHECK;
            if (L->rd_head != tl && mut != SMUT_NO_POSITIONS) hold = 1;
            if (hold) L->busy = 1;
            const int grow = !L->rd_pool && (!x->room || L->rd_room);
            if ((L->rd_C > 0 || grow) && L->avail_r == SM_EMPTY) L->avail_r = L->sr;
            break;
        }
        }
        if (++L->sph == 1 && !x->room) L->sph = 2; /* no cap: no room read */
        if (L->sph < 5) return 1;
        L->sph = 0;
        if (++L->sr < S) return 1;
        /* the scan is complete */
        if (L->avail_r != SM_EMPTY) {
            L->j = (uint8_t)((L->home + L->avail_r) % x->S);
            L->in_serve = 1;
            L->held = 0;
            L->check_first = 1;
            L->served_before = L->need;
            L->pc = PC_RESERVE;
            return 1;
        }
        if (!L->busy) {
            check_null(x, s, l);
            L->failed = L->need;
            L->need = 0;
            L->pc = PC_DONE;
            return 1;
        }
        /* holds or entries in flight: look again */
        L->sr = 0;
        L->avail_r = SM_EMPTY;
        L->busy = 0;
        L->scanned = 0;
        return 1;
    }
    case PC_F_OR: {
        const int v = L->fpages[L->fi];
        s->bits[page_chunk(x, v)] |= (uint8_t)(1u << (v % x->P));
        L->pc = PC_F_TAIL;
        return 1;
    }
    case PC_F_TAIL: {
        shard_t* sh = &s->sh[page_shard(x, L->fpages[L->fi])];
        L->fpos = sh->tail;
        sh->tail++;
        L->pc = PC_F_PUT;
        return 1;
    }
    case PC_F_PUT: {
        shard_t* sh = &s->sh[page_shard(x, L->fpages[L->fi])];
        uint8_t* sl = &sh->slot[L->fpos % x->Q];
        if (*sl != SM_EMPTY) return 0;
        *sl = L->fpages[L->fi];
        L->pc = PC_F_PUB;
        return 1;
    }
    case PC_F_PUB: {
        shard_t* sh = &s->sh[page_shard(x, L->fpages[L->fi])];
        sh->C++;
        if (++L->fi == L->nf) L->pc = PC_DONE;
        else L->pc = PC_F_OR;
        return 1;
    }
    }
    return 0;
}

static void dfs(sctx* x, const sstate* s)
{
    int any = 0, all_done = 1;
    for (int l = 0; l < x->p->n_leaders; ++l) {
        if (s->L[l].pc == PC_DONE) continue;
        all_done = 0;
        sstate n = *s;
        if (!step(x, &n, l)) continue;
        any = 1;
        const int v = s_visit(x, &n);
        if (v < 0) { x->r->truncated = 1; return; }
        if (v == 1) dfs(x, &n);
        if (x->r->truncated) return;
    }
    if (all_done) {
        x->r->terminals++;
        check_final(x, s);
        for (int l = 0; l < x->p->n_leaders; ++l)
            if (s->L[l].failed) { x->r->null_outcomes++; break; }
    } else if (!any) {
        x->r->deadlocks++;
        s_violation(x, 300, NULL);
    }
}

int orc_shards_model_run(const orc_shards_params* p, orc_shards_result* r)
{
    memset(r, 0, sizeof(*r));
    if (p->n_shards < 1 || p->n_shards > SM_S || p->chunks < 1 || p->chunks > SM_C || p->ppc < 1 || p->ppc > SM_P ||
        p->n_leaders < 1 || p->n_leaders > SM_L || p->room < 0 || p->room > SM_C)
        return -1;
    sctx x;
    memset(&x, 0, sizeof(x));
    x.p = p;
    x.r = r;
    x.S = p->n_shards;
    x.Cn = p->chunks;
    x.P = p->ppc;
    x.Q = SM_Q;
    x.room = p->room;
    sstate s0;
    memset(&s0, 0, sizeof(s0));
    /* prefill: shard j's first taken[j] chunks are owned by the class; their
     * pages allocated per prealloc[j] (bit c*P + p), all others free and
     * published in ascending order */
    for (int j = 0; j < x.S; ++j) {
        shard_t* sh = &s0.sh[j];
        memset(sh->slot, SM_EMPTY, sizeof(sh->slot));
        if (p->taken[j] > x.Cn || (x.room && p->taken[j] > x.room)) return -2;
        sh->bump = (uint8_t)p->taken[j];
        sh->owned = (uint8_t)p->taken[j];
        for (int c = 0; c < p->taken[j]; ++c)
            for (int pg = 0; pg < x.P; ++pg) {
                if ((p->prealloc[j] >> (c * x.P + pg)) & 1) continue;
                const int v = (j * x.Cn + c) * x.P + pg;
                s0.bits[j * x.Cn + c] |= (uint8_t)(1u << pg);
                if (sh->tail >= x.Q) return -3;
                sh->slot[sh->tail++] = (uint8_t)v;
                sh->C++;
            }
    }
    for (int l = 0; l < SM_L; ++l) s0.L[l].rc = SM_EMPTY;
    for (int l = 0; l < p->n_leaders; ++l) {
        sleader_t* L = &s0.L[l];
        const orc_shards_op* op = &p->ops[l];
        L->kind = (uint8_t)op->kind;
        if (op->kind == ORC_SOP_ALLOC) {
            if (op->a < 1 || op->a > 2 * x.P || op->b < 0 || op->b >= x.S) return -4;
            L->need = (uint8_t)op->a;
            L->home = (uint8_t)op->b;
            L->pc = PC_START;
        } else if (op->kind == ORC_SOP_FREE) {
            /* free the prefill-allocated pages [a, a + b) of the global
             * page numbering */
            if (op->b < 1 || op->b > SM_P * 2) return -5;
            for (int q = 0; q < op->b; ++q) {
                const int v = op->a + q;
                const int j = v / (x.Cn * x.P), c = (v / x.P) % x.Cn, pg = v % x.P;
                if (j >= x.S || c >= p->taken[j] || !((p->prealloc[j] >> (c * x.P + pg)) & 1)) return -6;
                L->fpages[L->nf++] = (uint8_t)v;
            }
            L->pc = PC_F_OR;
        } else {
            return -7;
        }
    }
    x.cap = 1ull << 22;
    while (x.cap < (uint64_t)p->max_states * 2) x.cap <<= 1;
    x.tab = (sstate*)malloc(x.cap * sizeof(sstate));
    x.used = (uint8_t*)calloc(x.cap, 1);
    if (!x.tab || !x.used) { free(x.tab); free(x.used); return -8; }
    s_visit(&x, &s0);
    dfs(&x, &s0);
    free(x.tab);
    free(x.used);
    return 0;
}
