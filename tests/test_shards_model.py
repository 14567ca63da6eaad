"""Brute-force enumeration of interleavings across shards (CPU).

The shards model (oracle/hbheap_shards_model.c) restates the page variant
one atomic step at a time over two or three shards: each wave's passes on
its home shard, the scan that reads every shard's pool, state word, head and
tail in that order, stealing from the first shard that shows something, and
the NULL answer when a scan finds every shard empty with nothing in flight.
Frees publish into their own shard's queue concurrently.

On the clean algorithm every schedule must end without a deadlock, with a
consistent final state, and every NULL answer must be exact: no pool chunk
left, no refill in flight holding unpublished pages, and every published
entry either reserved by an allocation, still owed to an unfinished free,
or published after the scan read that shard's tail (with no frees running:
nothing left at all).  Each planted mistake must be caught on the
configuration that exercises it.
"""
import pytest

import oracle as O

A, F = O.SOP_ALLOC, O.SOP_FREE

# pages: v = (shard * chunks + chunk) * ppc + page; taken[j] chunks of shard j
# start owned by the class, prealloc[j] marks their allocated pages (the
# others start published)
CONFIGS = {
    # shard 0 drained, shard 1 holds one chunk in its pool: one wave refills
    # there, the other must find the leftover page by scanning
    "steal_refill": dict(n_shards=2, chunks=1, ppc=2, ops=[(A, 1, 1), (A, 1, 0)], taken=(1, 0), prealloc=(0b11, 0)),
    "steal_refill3": dict(n_shards=2, chunks=1, ppc=4, ops=[(A, 1, 1), (A, 2, 0), (A, 1, 0)], taken=(1, 0),
                          prealloc=(0b1111, 0)),
    # more pages wanted than exist: exactly the capacity succeeds
    "oom_exact": dict(n_shards=2, chunks=1, ppc=2, ops=[(A, 2, 1), (A, 1, 0)], taken=(1, 0), prealloc=(0b11, 0)),
    "oom_three": dict(n_shards=2, chunks=1, ppc=2, ops=[(A, 2, 1), (A, 1, 0), (A, 1, 0)], taken=(1, 0),
                      prealloc=(0b11, 0)),
    # a first pass over-asks on shard 1 while a free publishes there; a wave
    # of the drained shard 0 scans
    "overask_free": dict(n_shards=2, chunks=1, ppc=2, ops=[(A, 2, 1), (F, 2, 1), (A, 1, 0)], taken=(1, 1),
                         prealloc=(0b11, 0b11)),
    "free_cross": dict(n_shards=2, chunks=1, ppc=2, ops=[(A, 1, 0), (F, 2, 2), (A, 2, 0)], taken=(1, 1),
                       prealloc=(0b11, 0b11)),
    "two_pools": dict(n_shards=2, chunks=2, ppc=2, ops=[(A, 2, 0), (A, 2, 1), (A, 2, 0)], taken=(1, 1),
                      prealloc=(0b0011, 0b0011)),
    "three_shards": dict(n_shards=3, chunks=1, ppc=2, ops=[(A, 2, 0), (A, 1, 2), (A, 2, 1)], taken=(1, 0, 0),
                         prealloc=(0b11, 0, 0)),
    # a room cap of one chunk per shard (two in each pool): the refills race
    # on the room counter; the pages that fit the caps are exactly demanded
    "room_race": dict(n_shards=2, chunks=2, ppc=2, room=1, ops=[(A, 2, 0), (A, 1, 0), (A, 1, 1)]),
    # a refill that wants two chunks where one fits: it keeps one, gives the
    # other back, and finds the rest on the other shard
    "room_partial": dict(n_shards=2, chunks=2, ppc=2, room=1, ops=[(A, 3, 0), (A, 1, 0)]),
    # one page more than the caps allow: some request is answered NULL, and
    # every NULL is exact
    "room_short": dict(n_shards=2, chunks=2, ppc=2, room=1, ops=[(A, 3, 0), (A, 2, 1)]),
    # a free races the capped refills (a page short of the demand)
    "room_free": dict(n_shards=2, chunks=2, ppc=2, room=1, ops=[(A, 2, 1), (F, 0, 1), (A, 2, 0)], taken=(1, 0),
                      prealloc=(0b11, 0)),
}
LARGE = ("steal_refill3", "oom_three")  # about 2 M states each (about 2 GB of visited states)
SHORT = ("oom_exact", "oom_three", "two_pools", "three_shards", "room_short", "room_free")  # fewer pages than requested


@pytest.mark.parametrize("name", [pytest.param(n, marks=pytest.mark.slow) if n in LARGE else n for n in CONFIGS])
def test_shards_model_clean(name):
    r = O.shards_model_run(**CONFIGS[name])
    assert not r["truncated"], r
    assert r["violations"] == 0 and r["deadlocks"] == 0, r
    assert r["terminals"] > 0
    if name in SHORT:
        # not every request can be served, in every schedule
        assert r["null_outcomes"] == r["terminals"], r
    elif name in ("steal_refill", "steal_refill3", "room_race", "room_partial"):
        # exactly as many pages as the pools, caps and frees provide
        assert r["null_outcomes"] == 0, r


# each planted mistake, and a configuration on which it answers NULL with
# pages left (first_violation 100 + leader: a NULL answer was not exact)
MUTANT_PINS = [
    ("state_before_pool", "steal_refill"),   # a refill takes the pool's last chunk between the two reads
    ("ignore_positions", "overask_free"),    # a free's entry hidden by an over-asking first pass
    ("ignore_holds", "oom_exact"),           # a refill in flight not yet published
    ("home_only", "two_pools"),              # chunks left in another shard's pool
]


# planted mistakes in the room counter's add-and-give-back, caught by the
# final state (first_violation 260 + shard: the counter differs from the
# chunks the class owns, or these pass the cap)
ROOM_MUTANT_PINS = [
    ("room_no_cap", "room_race"),        # a refill keeps all it added: a second chunk past the cap
    ("room_keep_excess", "room_race"),   # the excess stays on the counter
    ("room_back_all", "room_partial"),   # the give-back returns the granted chunk as well
]


@pytest.mark.parametrize("mutation,name", ROOM_MUTANT_PINS)
def test_shards_model_catches_room_mistake(mutation, name):
    r = O.shards_model_run(mutation=O.SHARDS_MUTATIONS[mutation], **CONFIGS[name])
    assert not r["truncated"]
    assert r["final_violations"] > 0 and 260 <= r["first_violation"] < 263, r


def test_shards_model_keep_excess_is_harmless_to_exactness():
    """An excess never given back only misstates the counter: every answer
    stays exact (the adder that passed the cap took all the room left), which
    is why a reading at or above the cap may be trusted."""
    r = O.shards_model_run(mutation=O.SHARDS_MUTATIONS["room_keep_excess"], **CONFIGS["room_short"])
    assert r["oom_violations"] == 0 and r["deadlocks"] == 0 and r["final_violations"] > 0, r


@pytest.mark.parametrize("mutation,name", MUTANT_PINS)
def test_shards_model_catches_planted_mistake(mutation, name):
    r = O.shards_model_run(mutation=O.SHARDS_MUTATIONS[mutation], **CONFIGS[name])
    assert not r["truncated"]
    assert r["oom_violations"] > 0 and 100 <= r["first_violation"] < 103, r


def test_shards_model_state_before_pool_needs_the_race():
    """The state-before-pool mistake is harmless without a refill racing the
    scan: on a configuration where every chunk is already owned (no refill
    can run) the mistaken order finds nothing to report."""
    cfg = dict(CONFIGS["free_cross"])
    r = O.shards_model_run(mutation=O.SHARDS_MUTATIONS["state_before_pool"], **cfg)
    assert r["violations"] == 0, r


def test_shards_model_rejects_bad_parameters():
    with pytest.raises(ValueError):
        O.shards_model_run(n_shards=4, chunks=1, ppc=2, ops=[(A, 1, 0)])
    with pytest.raises(ValueError):
        O.shards_model_run(n_shards=2, chunks=1, ppc=2, ops=[(A, 5, 0)])   # more than two chunks
    with pytest.raises(ValueError):
        O.shards_model_run(n_shards=2, chunks=2, ppc=2, room=3, ops=[(A, 1, 0)])   # cap above the chunks
    with pytest.raises(ValueError):
        O.shards_model_run(n_shards=2, chunks=2, ppc=2, room=1, taken=(2, 0), ops=[(A, 1, 0)])   # owns past the cap
    with pytest.raises(ValueError):
        O.shards_model_run(n_shards=2, chunks=1, ppc=2, ops=[(F, 0, 1)])   # page 0 not allocated
