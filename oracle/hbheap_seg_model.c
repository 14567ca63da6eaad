/*
 * hbheap_seg_model.c -- step-level model of the virtualised queues: a queue
 * whose ring positions live in segments of G slots taken on demand from a
 * store the queues of a shard share, explored over every interleaving.
 * TEST INFRASTRUCTURE ONLY (see hbheap_oracle.h): used by tests, never by
 * the product path; it shares no code with the HIP library and restates the
 * protocol on its own.
 *
 * Two forms (the paper's virtualised array and virtualised list queues,
 * Results):
 *   - array: position p lies in segment number s = p / G, found in the
 *     queue's directory entry s mod D, which holds (s, segment id) while the
 *     segment is in use; the producer of a segment's first slot takes a
 *     segment from the store and installs it with a compare-and-swap from
 *     the empty entry, everyone else waits for the entry to show s;
 *   - list: the queue keeps a front and a back word (number, id); segment
 *     ids carry a tag (queue, number) and a link to the next segment; the
 *     producer of a segment's first slot takes a segment from the store,
 *     tags it and clears its link as soon as it knows its position (the back
 *     may still be behind s - 1), then, once the back is segment s - 1,
 *     links it after the back and moves the back to it; consumers walk from the front
 *     along links, trusting a link only while the segment it was read from
 *     still carries the tag the walk expects.
 * In both, the consumer of a segment's last slot is its closer: once the
 * segment's consumed count shows all G slots taken, it retires the segment:
 * array -- reset the count, empty the directory entry, return the id to the
 * store; list -- unlink fully consumed segments from the front (a
 * compare-and-swap on the front word picks one retirer, which resets the
 * count and link and returns the id), also run by the producer that linked a
 * successor.  The store is itself a ring of free ids (count, head, tail).
 * Producers reserve a tail position, fill the slot (compare-and-swap from
 * empty, waiting while the previous lap's entry is still there) and publish
 * the count; consumers reserve a published entry (waiting while none),
 * advance the head, exchange the slot out and add to the segment's count.
 * Waits are transitions that are disabled until their condition holds.
 *
 * Checked: every value produced is taken exactly once and never read from a
 * slot of a segment other than its position's; every segment id is in
 * exactly one place (the store, a directory entry or the list, or the hands
 * of one leader moving it); final states: the store holds exactly the ids
 * not in use, the queue's segments are exactly those its live positions
 * need, counts and positions agree; no deadlock.  Mutations plant known
 * mistakes so the tests can show each check fires.
 */
#include "hbheap_oracle.h"

#include <stdlib.h>
#include <string.h>

#define GM_Q 2        /* queues                      */
#define GM_M 4        /* segments in the store       */
#define GM_G 2        /* slots per segment           */
#define GM_D 2        /* directory entries per queue */
#define GM_L 3        /* leaders                     */
#define GM_OPS 6      /* operations per leader       */
#define GM_E 0xFF

enum { GMUT_NONE = 0, GMUT_CLOSE_EARLY = 1, GMUT_INSTALL_BLIND = 2, GMUT_KEEP_COUNT = 3, GMUT_RETIRE_UNCOUNTED = 4,
       GMUT_LINK_EARLY = 5 /* list: a prepared segment linked after whatever the back is */ };

typedef struct {
    int8_t C;                  /* published entries                          */
    uint8_t head, tail;        /* positions                                  */
    uint8_t dir[GM_D];         /* array: segment number << 4 | id, or GM_E    */
    uint8_t front_s, front_m;  /* list: number and id of the front segment   */
    uint8_t back_s, back_m;    /* list: number and id of the back segment    */
} queue_t;

typedef struct {
    uint8_t pc, op, q, pos, seg, val, c, hand, walk_s, walk_m, w0s, w0m, nx, rf_s, rf_m, rc, prod;
    uint8_t ngot;
} gleader_t;

typedef struct {
    queue_t q[GM_Q];
    uint8_t slot[GM_M][GM_G];  /* segment slots: a value or GM_E             */
    uint8_t taken[GM_M];       /* consumed count per segment                 */
    uint8_t tag_q[GM_M], tag_s[GM_M]; /* list: tag (queue, number), GM_E none */
    uint8_t next[GM_M];        /* list: link, GM_E none                      */
    /* the store: a ring of free ids */
    int8_t sC;
    uint8_t shead, stail;
    uint8_t sslot[GM_M];
    gleader_t L[GM_L];
    uint8_t produced[32];      /* per value: 1 produced and not yet taken, 2 taken */
    uint8_t vpos[32], vq[32];  /* the position and queue a value was written at */
} gstate;

typedef struct {
    const orc_seg_params* p;
    orc_seg_result* r;
    int G, D, M, list;
    gstate* tab;
    uint8_t* used;
    uint64_t cap;
} gctx;

/* program counters */
enum {
    G_DONE = 0, G_NEXT,
    /* producer */
    G_P_TAIL, G_P_LOOK, G_P_STORE_RES, G_P_STORE_HEAD, G_P_STORE_TAKE, G_P_INSTALL,
    G_P_TAG, G_P_CLEARLINK, G_P_LINK, G_P_BACK, G_P_PUT, G_P_PUB,
    /* consumer */
    G_C_RES, G_C_HEAD, G_C_LOOK, G_C_FRONT, G_C_WALK, G_C_WALK_TAG, G_C_RETRY, G_C_TAKE, G_C_COUNT, G_C_CLOSE_WAIT,
    G_C_RESET, G_C_DIR, G_S_PUT_TAIL, G_S_PUT, G_S_PUT_PUB,
    /* list retire loop */
    G_R_FRONT, G_R_COUNT, G_R_LINK, G_R_CAS, G_R_RESET, G_R_UNLINK
};

static uint64_t g_hash(const gstate* s)
{
    const uint8_t* b = (const uint8_t*)s;
    uint64_t h = 1469598103934665603ull;
    for (size_t i = 0; i < sizeof(gstate); ++i) { h ^= b[i]; h *= 1099511628211ull; }
    return h ^ (h >> 29);
}

static int g_visit(gctx* x, const gstate* s)
{
    uint64_t h = g_hash(s) & (x->cap - 1);
    for (uint64_t probe = 0; probe < x->cap; ++probe) {
        uint64_t i = (h + probe) & (x->cap - 1);
        if (!x->used[i]) {
            if ((int64_t)x->r->states >= x->p->max_states) return -1;
            x->used[i] = 1;
            x->tab[i] = *s;
            x->r->states++;
            return 1;
        }
        if (!memcmp(&x->tab[i], s, sizeof(gstate))) return 0;
    }
    return -1;
}

static void g_violation(gctx* x, int code, int64_t* which)
{
    x->r->violations++;
    if (which) (*which)++;
    if (!x->r->first_violation) x->r->first_violation = code;
}

static uint8_t dent(uint8_t s, uint8_t m) { return (uint8_t)((s << 4) | m); }

/* each segment id in exactly one place */
static void check_segments(gctx* x, const gstate* s)
{
    int where[GM_M] = {0};
    /* every store slot holding an id (a taker empties its slot when it takes
     * the id, so a reserved but untaken slot still counts) */
    for (int i = 0; i < x->M; ++i)
        if (s->sslot[i] != GM_E) where[s->sslot[i]]++;
    for (int q = 0; q < x->p->n_queues; ++q) {
        const queue_t* Q = &s->q[q];
        if (!x->list) {
            for (int d = 0; d < x->D; ++d)
                if (Q->dir[d] != GM_E) where[Q->dir[d] & 15]++;
        } else {
            /* the chain from the front along the links (the back is on it,
             * or -- between a retirement of the old back and the linker's
             * move of the back -- just behind the front) */
            uint8_t m = Q->front_m;
            int hop = 0;
            for (; hop <= x->M && m != GM_E; ++hop) {
                where[m]++;
                m = s->next[m];
            }
            if (hop > x->M) { g_violation(x, 40, &x->r->segment_violations); return; }
        }
    }
    for (int l = 0; l < x->p->n_leaders; ++l)
        if (s->L[l].hand != GM_E) where[s->L[l].hand]++;
    for (int m = 0; m < x->M; ++m)
        if (where[m] != 1) { g_violation(x, 50 + m, &x->r->segment_violations); return; }
}

static void check_final(gctx* x, const gstate* s)
{
    for (int v = 0; v < 32; ++v)
        if (s->produced[v] == 1 && x->p->consume_all) { g_violation(x, 60, &x->r->final_violations); return; }
    for (int q = 0; q < x->p->n_queues; ++q) {
        const queue_t* Q = &s->q[q];
        if (Q->C != (int8_t)(uint8_t)(Q->tail - Q->head)) { g_violation(x, 70 + q, &x->r->final_violations); return; }
        if (x->list) {
            /* the chain front .. back carries the tags (q, front_s) ..
             * (q, back_s), ends without a link, and covers every live
             * position */
            uint8_t m = Q->front_m;
            for (int sg = Q->front_s;; ++sg) {
                if (s->tag_q[m] != q || s->tag_s[m] != sg) { g_violation(x, 85 + q, &x->r->final_violations); return; }
                if (sg == Q->back_s) break;
                m = s->next[m];
                if (m == GM_E) { g_violation(x, 87 + q, &x->r->final_violations); return; }
            }
            if (s->next[Q->back_m] != GM_E || Q->front_s * x->G > Q->head || (Q->back_s + 1) * x->G < Q->tail) {
                g_violation(x, 89, &x->r->final_violations);
                return;
            }
        }
        if (!x->list) {
            /* directory: exactly the segments from head's to tail - 1's */
            uint8_t want[GM_D];
            memset(want, GM_E, sizeof(want));
            const int hs = Q->head / x->G;
            for (int sg = hs; sg * x->G < Q->tail; ++sg) want[sg % x->D] = (uint8_t)sg;
            for (int d = 0; d < x->D; ++d) {
                const int has = Q->dir[d] != GM_E;
                if (has != (want[d] != GM_E) || (has && (Q->dir[d] >> 4) != want[d])) {
                    g_violation(x, 80 + q, &x->r->final_violations);
                    return;
                }
            }
        }
    }
    check_segments(x, s);
}

/* one step of leader l; 0 if disabled */
static int gstep(gctx* x, gstate* s, int l)
{
    const orc_seg_params* p = x->p;
    const int mut = p->mutation;
    const int G = x->G;
    gleader_t* L = &s->L[l];
    switch (L->pc) {
    case G_DONE:
        return 0;
    case G_NEXT: {
        if (L->op >= p->n_ops[l]) { L->pc = G_DONE; return 1; }
        const orc_seg_op* op = &p->ops[l][L->op];
        L->q = (uint8_t)op->queue;
        if (op->kind == ORC_GOP_PUT) { L->val = (uint8_t)op->value; L->pc = G_P_TAIL; }
        else L->pc = G_C_RES;
        return 1;
    }
    /* ---- producer ---- */
    case G_P_TAIL:
        L->pos = s->q[L->q].tail++;
        L->pc = G_P_LOOK;
        return 1;
    case G_P_LOOK: {
        queue_t* Q = &s->q[L->q];
        const uint8_t sg = L->pos / G, off = L->pos % G;
        if (!x->list) {
            const uint8_t d = Q->dir[sg % x->D];
            if (d != GM_E && (d >> 4) == sg) { L->seg = d & 15; L->pc = G_P_PUT; return 1; }
            if (off == 0 && (d == GM_E || mut == GMUT_INSTALL_BLIND)) { L->pc = G_P_STORE_RES; return 1; }
            return 0; /* wait for the installer */
        }
        if (Q->back_s == sg) { L->seg = Q->back_m; L->pc = G_P_PUT; return 1; }
        if (off == 0 && (int8_t)(sg - Q->back_s) >= 1) {
            /* the producer of a segment's first slot takes and tags its
             * segment first (even while earlier segments are not linked
             * yet), then links it once the back is segment sg - 1 */
            if (L->hand == GM_E) { L->pc = G_P_STORE_RES; return 1; }
            if ((uint8_t)(Q->back_s + 1) == sg || mut == GMUT_LINK_EARLY) {
                L->rf_m = Q->back_m;
                L->pc = G_P_LINK;
                return 1;
            }
            return 0; /* wait for the back */
        }
        if ((int8_t)(Q->back_s - sg) > 0) {
            /* a late producer of an older segment: walk from the front */
            L->prod = 1;
            L->pc = G_C_FRONT;
            return 1;
        }
        return 0;
    }
    case G_P_STORE_RES: {
        /* reserve a free id: count -= 1, waiting while none is published */
        if (s->sC <= 0) return 0;
        s->sC--;
        L->pc = G_P_STORE_HEAD;
        return 1;
    }
    case G_P_STORE_HEAD:
        L->c = s->shead++;            /* store position */
        L->pc = G_P_STORE_TAKE;
        return 1;
    case G_P_STORE_TAKE: {
        uint8_t* sl = &s->sslot[L->c % x->M];
        if (*sl == GM_E) return 0;
        L->hand = *sl;
        *sl = GM_E;
        L->pc = x->list ? G_P_TAG : G_P_INSTALL;
        return 1;
    }
    case G_P_INSTALL: {
        queue_t* Q = &s->q[L->q];
        const uint8_t sg = L->pos / G;
        uint8_t* d = &Q->dir[sg % x->D];
        if (*d != GM_E && mut != GMUT_INSTALL_BLIND) { g_violation(x, 10, &x->r->segment_violations); return 1; }
        *d = dent(sg, L->hand);
        L->seg = L->hand;
        L->hand = GM_E;
        L->pc = G_P_PUT;
        return 1;
    }
    case G_P_TAG:
        s->tag_q[L->hand] = L->q;
        s->tag_s[L->hand] = L->pos / G;
        L->pc = G_P_CLEARLINK;
        return 1;
    case G_P_CLEARLINK:
        s->next[L->hand] = GM_E;
        L->pc = G_P_LOOK; /* linked once the back is the segment before */
        return 1;
    case G_P_LINK:
        /* link after the back this producer read (only it moves the back
         * from segment s - 1 to s) */
        if (s->next[L->rf_m] != GM_E) g_violation(x, 11, &x->r->segment_violations);
        s->next[L->rf_m] = L->hand;
        L->seg = L->hand;
        L->hand = GM_E;     /* on the chain from now on */
        L->pc = G_P_BACK;
        return 1;
    case G_P_BACK: {
        queue_t* Q = &s->q[L->q];
        Q->back_s = L->pos / G;
        Q->back_m = L->seg;
        /* the linker may complete the retire conditions of the old front */
        L->rc = 1; /* after the retire loop: put the value */
        L->pc = G_R_FRONT;
        return 1;
    }
    case G_P_PUT: {
        uint8_t* sl = &s->slot[L->seg][L->pos % G];
        if (*sl != GM_E) return 0;
        *sl = L->val;
        s->produced[L->val] = 1;
        s->vpos[L->val] = L->pos;
        s->vq[L->val] = L->q;
        L->pc = G_P_PUB;
        return 1;
    }
    case G_P_PUB:
        s->q[L->q].C++;
        L->op++;
        L->pc = G_NEXT;
        return 1;
    /* ---- consumer ---- */
    case G_C_RES: {
        queue_t* Q = &s->q[L->q];
        if (Q->C <= 0) return 0;   /* wait for a published entry */
        Q->C--;
        L->pc = G_C_HEAD;
        return 1;
    }
    case G_C_HEAD:
        L->pos = s->q[L->q].head++;
        L->prod = 0;
        L->pc = x->list ? G_C_FRONT : G_C_LOOK;
        return 1;
    case G_C_LOOK: {
        const uint8_t sg = L->pos / G;
        const uint8_t d = s->q[L->q].dir[sg % x->D];
        if (d == GM_E || (d >> 4) != sg) return 0;
        L->seg = d & 15;
        L->pc = G_C_TAKE;
        return 1;
    }
    case G_C_FRONT:
        L->walk_s = L->w0s = s->q[L->q].front_s;
        L->walk_m = L->w0m = s->q[L->q].front_m;
        L->pc = G_C_WALK;
        return 1;
    case G_C_WALK: {
        const uint8_t sg = L->pos / G;
        if (L->walk_s == sg) {
            L->seg = L->walk_m;
            L->pc = L->prod ? G_P_PUT : G_C_TAKE;
            return 1;
        }
        if ((int8_t)(sg - L->walk_s) < 0) { L->pc = G_C_RETRY; return 1; }
        L->nx = s->next[L->walk_m];
        L->pc = G_C_WALK_TAG;
        return 1;
    }
    case G_C_WALK_TAG: {
        /* the link read is trusted only if the segment it was read from
         * still carries the tag the walk expects */
        const int tag_ok = s->tag_q[L->walk_m] == L->q && s->tag_s[L->walk_m] == L->walk_s;
        if (L->nx != GM_E && tag_ok) {
            L->walk_m = L->nx;
            L->walk_s++;
            L->pc = G_C_WALK;
        } else {
            L->pc = G_C_RETRY;
        }
        return 1;
    }
    case G_C_RETRY:
        /* wait, then walk again from the front, once it has moved */
        if (s->q[L->q].front_s == L->w0s && s->q[L->q].front_m == L->w0m) return 0;
        L->pc = G_C_FRONT;
        return 1;
    case G_C_TAKE: {
        uint8_t* sl = &s->slot[L->seg][L->pos % G];
        if (*sl == GM_E) return 0; /* producer late */
        const uint8_t v = *sl;
        *sl = GM_E;
        if (v >= 32 || s->produced[v] != 1) { g_violation(x, 20, &x->r->value_violations); return 1; }
        /* the value must be the one written at this position of this queue */
        if (s->vpos[v] != L->pos || s->vq[v] != L->q) g_violation(x, 21, &x->r->value_violations);
        s->produced[v] = 2;
        L->ngot++;
        L->pc = G_C_COUNT;
        return 1;
    }
    case G_C_COUNT: {
        s->taken[L->seg]++;
        if (L->pos % G != G - 1) { L->op++; L->pc = G_NEXT; return 1; }
        L->c = s->taken[L->seg];
        L->pc = G_C_CLOSE_WAIT;
        return 1;
    }
    case G_C_CLOSE_WAIT: {
        if (mut != GMUT_CLOSE_EARLY) {
            if (x->list && s->taken[L->seg] != G) {
                /* a list segment may have been retired by another loop
                 * already: the front moved past it */
                if ((int8_t)(s->q[L->q].front_s - L->pos / G) > 0) { L->op++; L->pc = G_NEXT; return 1; }
                return 0;
            }
            if (s->taken[L->seg] != G) return 0;
        }
        L->rc = 0;
        L->pc = x->list ? G_R_FRONT : G_C_RESET;
        return 1;
    }
    case G_C_RESET:
        if (mut != GMUT_KEEP_COUNT) s->taken[L->seg] = 0;
        L->pc = G_C_DIR;
        return 1;
    case G_C_DIR: {
        queue_t* Q = &s->q[L->q];
        Q->dir[(L->pos / G) % x->D] = GM_E;
        L->hand = L->seg;
        L->pc = G_S_PUT_TAIL;
        return 1;
    }
    case G_S_PUT_TAIL:
        L->c = s->stail++;
        L->pc = G_S_PUT;
        return 1;
    case G_S_PUT: {
        uint8_t* sl = &s->sslot[L->c % x->M];
        if (*sl != GM_E) return 0;
        *sl = L->hand;
        L->hand = GM_E;
        L->pc = G_S_PUT_PUB;
        return 1;
    }
    case G_S_PUT_PUB:
        s->sC++;
        /* list retirer: look again for the next front segment */
        if (x->list) { L->pc = G_R_FRONT; return 1; }
        L->op++;
        L->pc = G_NEXT;
        return 1;
    /* ---- list retire loop (closer, linker, or after a retire) ---- */
    case G_R_FRONT: {
        queue_t* Q = &s->q[L->q];
        L->rf_s = Q->front_s;
        L->rf_m = Q->front_m;
        L->pc = G_R_COUNT;
        return 1;
    }
    case G_R_COUNT:
        /* a front segment goes only once all its slots are consumed (the
         * planted mistake skips the count) */
        L->c = s->taken[L->rf_m];
        L->pc = (L->c == G || mut == GMUT_RETIRE_UNCOUNTED) ? G_R_LINK : G_R_UNLINK;
        return 1;
    case G_R_LINK:
        L->walk_m = s->next[L->rf_m];
        L->pc = L->walk_m != GM_E ? G_R_CAS : G_R_UNLINK;
        return 1;
    case G_R_CAS: {
        queue_t* Q = &s->q[L->q];
        if (Q->front_s == L->rf_s && Q->front_m == L->rf_m) {
            Q->front_s = (uint8_t)(L->rf_s + 1);
            Q->front_m = L->walk_m;
            L->hand = L->rf_m;   /* this retirer owns the old front */
            L->pc = G_R_RESET;
        } else {
            L->pc = G_R_FRONT;   /* someone else moved it: look again */
        }
        return 1;
    }
    case G_R_RESET:
        /* the retirer owns the segment: reset its count and link (its tag
         * stays until the segment is tagged again) */
        if (mut != GMUT_KEEP_COUNT) s->taken[L->hand] = 0;
        s->next[L->hand] = GM_E;
        L->pc = G_S_PUT_TAIL;
        return 1;
    case G_R_UNLINK:
        /* nothing (more) to retire: the linker goes on to put its value, the
         * closer is done */
        if (L->rc == 1) { L->rc = 0; L->pc = G_P_PUT; return 1; }
        L->op++;
        L->pc = G_NEXT;
        return 1;
    }
    return 0;
}

static void gdfs(gctx* x, const gstate* s)
{
    int any = 0, all_done = 1;
    check_segments(x, s);
    for (int l = 0; l < x->p->n_leaders; ++l) {
        if (s->L[l].pc == G_DONE) continue;
        all_done = 0;
        gstate n = *s;
        if (!gstep(x, &n, l)) continue;
        any = 1;
        const int v = g_visit(x, &n);
        if (v < 0) { x->r->truncated = 1; return; }
        if (v == 1) gdfs(x, &n);
        if (x->r->truncated) return;
    }
    if (all_done) {
        x->r->terminals++;
        check_final(x, s);
    } else if (!any) {
        x->r->deadlocks++;
        g_violation(x, 90, NULL);
    }
}

int orc_seg_model_run(const orc_seg_params* p, orc_seg_result* r)
{
    memset(r, 0, sizeof(*r));
    if (p->n_queues < 1 || p->n_queues > GM_Q || p->n_leaders < 1 || p->n_leaders > GM_L || p->segments < 2 ||
        p->segments > GM_M)
        return -1;
    gctx x;
    memset(&x, 0, sizeof(x));
    x.p = p;
    x.r = r;
    x.G = GM_G;
    x.D = GM_D;
    x.M = p->segments;
    x.list = p->list != 0;
    gstate s0;
    memset(&s0, 0, sizeof(s0));
    memset(s0.slot, GM_E, sizeof(s0.slot));
    memset(s0.tag_q, GM_E, sizeof(s0.tag_q));
    memset(s0.tag_s, GM_E, sizeof(s0.tag_s));
    memset(s0.next, GM_E, sizeof(s0.next));
    memset(s0.sslot, GM_E, sizeof(s0.sslot));
    uint8_t first_free = 0;
    for (int q = 0; q < p->n_queues; ++q) {
        queue_t* Q = &s0.q[q];
        memset(Q->dir, GM_E, sizeof(Q->dir));
        if (x.list) {
            /* a list queue always keeps one segment: number 0 */
            Q->front_s = Q->back_s = 0;
            Q->front_m = Q->back_m = first_free;
            s0.tag_q[first_free] = (uint8_t)q;
            s0.tag_s[first_free] = 0;
            first_free++;
        }
    }
    for (int m = first_free; m < x.M; ++m) {
        s0.sslot[s0.stail % x.M] = (uint8_t)m;
        s0.stail++;
        s0.sC++;
    }
    for (int l = 0; l < GM_L; ++l) s0.L[l].hand = GM_E;
    for (int l = 0; l < p->n_leaders; ++l) {
        if (p->n_ops[l] < 0 || p->n_ops[l] > GM_OPS) return -2;
        for (int i = 0; i < p->n_ops[l]; ++i) {
            const orc_seg_op* op = &p->ops[l][i];
            if (op->queue < 0 || op->queue >= p->n_queues) return -3;
            if (op->kind == ORC_GOP_PUT && (op->value < 0 || op->value >= 32)) return -4;
        }
        s0.L[l].pc = G_NEXT;
    }
    x.cap = 1ull << 20;
    while (x.cap < (uint64_t)p->max_states + (uint64_t)p->max_states / 2) x.cap <<= 1;
    x.tab = (gstate*)malloc(x.cap * sizeof(gstate));
    x.used = (uint8_t*)calloc(x.cap, 1);
    if (!x.tab || !x.used) { free(x.tab); free(x.used); return -8; }
    g_visit(&x, &s0);
    gdfs(&x, &s0);
    free(x.tab);
    free(x.used);
    return 0;
}
