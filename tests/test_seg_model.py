"""Brute-force enumeration of interleavings of the virtualised queues (CPU).

The segment model (oracle/hbheap_seg_model.c) restates, one atomic step at a
time, queues whose positions live in 2-slot segments taken on demand from a
store the queues share: the virtualised array form (a directory entry per
segment number, installed by the producer of the segment's first slot, and
emptied by the consumer of its last slot once every slot is counted) and the
virtualised list form (tagged segments linked from the back, consumers
walking from the front and trusting a link only while the segment still
carries the expected tag, fully consumed front segments unlinked by a
compare-and-swap on the front word).  On the clean protocol every schedule
must end without deadlock, every value must be taken exactly once from the
position it was written at, every segment id must be in exactly one place
at every step, and the final directory or chain must cover exactly the live
positions.  Each planted mistake must be caught on the configuration that
exercises it.
"""
import pytest

import oracle as O

P, G = O.GOP_PUT, O.GOP_GET

# (list form?, configuration); values are distinct, all taken by the end
CONFIGS = {
    "one_queue": dict(n_queues=1, segments=3, leaders=[[(P, 0, 1), (P, 0, 2), (P, 0, 3)], [(G, 0)] * 3]),
    "two_producers": dict(n_queues=1, segments=3,
                          leaders=[[(P, 0, 1), (P, 0, 2)], [(P, 0, 3), (P, 0, 4)], [(G, 0)] * 4]),
    "two_consumers": dict(n_queues=1, segments=3,
                          leaders=[[(P, 0, 1), (P, 0, 2), (P, 0, 3), (P, 0, 4)], [(G, 0)] * 2, [(G, 0)] * 2]),
    "two_queues": dict(n_queues=2, segments=4, leaders=[[(P, 0, 1), (P, 0, 2), (P, 0, 3)],
                                                         [(P, 1, 4), (G, 0), (G, 0), (P, 1, 5)],
                                                         [(G, 0), (G, 1), (G, 1)]]),
    "wrap": dict(n_queues=1, segments=2, leaders=[[(P, 0, 1), (P, 0, 2), (P, 0, 3), (P, 0, 4)], [(G, 0)] * 4]),
    # segments reused: three segment numbers over two ids (array) or three
    "reuse": dict(n_queues=1, segments=2, leaders=[[(P, 0, 1), (P, 0, 2), (P, 0, 3)],
                                                    [(P, 0, 4), (P, 0, 5), (P, 0, 6)], [(G, 0)] * 6]),
    "reuse3": dict(n_queues=1, segments=3, leaders=[[(P, 0, 1), (P, 0, 2), (P, 0, 3), (P, 0, 4), (P, 0, 5)],
                                                     [(G, 0)] * 3, [(G, 0)] * 2]),
    # two list queues handing segments to each other through the store
    "cross": dict(n_queues=2, segments=3, leaders=[[(P, 0, 1), (P, 0, 2), (P, 0, 3), (P, 0, 4)], [(G, 0)] * 4,
                                                    [(P, 1, 5), (P, 1, 6), (G, 1), (P, 1, 7), (G, 1), (G, 1)]]),
    # three producers: the producer of segment 2's first slot can take its
    # segment while segment 1 is not linked yet (values left in the queue)
    "ahead": dict(n_queues=1, segments=4, consume_all=False,
                  leaders=[[(P, 0, 1), (P, 0, 2)], [(P, 0, 3), (P, 0, 4)], [(P, 0, 5)]]),
    "ahead_get": dict(n_queues=1, segments=4, consume_all=False,
                      leaders=[[(P, 0, 1), (P, 0, 2), (G, 0)], [(P, 0, 3), (P, 0, 4)], [(P, 0, 5), (G, 0)]]),
}
ARRAY = ["one_queue", "two_producers", "two_consumers", "two_queues", "wrap", "reuse", "reuse3"]
LIST = ["one_queue", "two_producers", "two_consumers", "two_queues", "wrap", "reuse", "cross", "ahead", "ahead_get"]
LARGE = {(True, "reuse")}  # about 1.9 M states


def _cases():
    for form, names in ((False, ARRAY), (True, LIST)):
        for n in names:
            marks = [pytest.mark.slow] if (form, n) in LARGE else []
            yield pytest.param(form, n, marks=marks, id=f"{'list' if form else 'array'}-{n}")


@pytest.mark.parametrize("list_form,name", list(_cases()))
def test_seg_model_clean(list_form, name):
    r = O.seg_model_run(list_form, max_states=2_200_000, **CONFIGS[name])
    assert not r["truncated"], r
    assert r["violations"] == 0 and r["deadlocks"] == 0, r
    assert r["terminals"] > 0


# planted mistakes: (form, mistake, configuration, what must show)
MUTANT_PINS = [
    # array closer that does not wait for the count: a consumer of the
    # segment never finds it again
    (False, "close_early", "reuse3", "deadlocks"),
    # installer that does not wait for the directory entry to empty: the
    # live segment it overwrites is lost
    (False, "install_blind", "reuse3", "segment_violations"),
    # count not reset on retirement: the reused segment's closer waits for
    # ever (array and list)
    (False, "keep_count", "reuse", "deadlocks"),
    (True, "keep_count", "cross", "deadlocks"),
    # list retirement that does not check the count: a segment leaves the
    # chain with a slot still to be taken
    (True, "retire_uncounted", "cross", "deadlocks"),
    # list installer that links its segment, taken ahead, without waiting
    # for the back to be the segment before: a link is overwritten
    (True, "link_early", "ahead", "segment_violations"),
]


@pytest.mark.parametrize("list_form,mutation,name,field", MUTANT_PINS)
def test_seg_model_catches_planted_mistake(list_form, mutation, name, field):
    r = O.seg_model_run(list_form, mutation=O.SEG_MUTATIONS[mutation], max_states=2_200_000, **CONFIGS[name])
    assert r[field] > 0 and r["violations"] > 0, r


def test_seg_model_list_closer_is_backed_by_the_retire_check():
    """In the list form the closer's wait for the count is backed up by the
    retirement loop's own count check, so skipping it breaks nothing."""
    r = O.seg_model_run(True, mutation=O.SEG_MUTATIONS["close_early"], **CONFIGS["cross"])
    assert r["violations"] == 0 and not r["truncated"], r


def test_seg_model_rejects_bad_parameters():
    with pytest.raises(ValueError):
        O.seg_model_run(False, n_queues=3, segments=3, leaders=[[(P, 0, 1)]])
    with pytest.raises(ValueError):
        O.seg_model_run(False, n_queues=1, segments=3, leaders=[[(P, 1, 1)]])  # no queue 1
