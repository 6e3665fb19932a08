"""Host logic of the serving loop: the admission choice (arrival order with backfilling and a
bound on how long a request that does not fit may be passed over)."""
from paper_2007_10196_amd.serving import backfill_choice

GB = 1 << 30


def test_everything_that_fits_is_admitted_in_arrival_order_up_to_the_free_slots():
    fps = [1 * GB, 2 * GB, 1 * GB, 1 * GB]
    assert backfill_choice(fps, [0.0] * 4, 0, 10 * GB, 8, 0.5) == [0, 1, 2, 3]
    assert backfill_choice(fps, [0.0] * 4, 0, 10 * GB, 2, 0.5) == [0, 1]
    assert backfill_choice(fps, [0.0] * 4, 7 * GB, 10 * GB, 8, 0.5) == [0, 1]


def test_later_requests_pass_a_large_one_only_while_it_is_young():
    fps = [8 * GB, 1 * GB, 9 * GB, 1 * GB]
    # 5 GB in use: the head does not fit; the small ones behind it do
    assert backfill_choice(fps, [0.1, 0.05, 0.04, 0.0], 5 * GB, 10 * GB, 8, 0.5) == [1, 3]
    # the head has waited its bound: nothing is admitted ahead of it
    assert backfill_choice(fps, [0.6, 0.05, 0.04, 0.0], 5 * GB, 10 * GB, 8, 0.5) == []
    # a later large request that has waited its bound stops the scan there
    assert backfill_choice(fps, [0.1, 0.7, 0.6, 0.0], 5 * GB, 10 * GB, 8, 0.5) == [1]
    # a bound of 0: strict arrival order
    assert backfill_choice(fps, [0.0, 0.0, 0.0, 0.0], 5 * GB, 10 * GB, 8, 0.0) == []
    assert backfill_choice(fps, [0.0] * 4, 0, 10 * GB, 8, 0.0) == [0, 1]


def test_admitted_footprints_never_exceed_the_budget():
    import random
    rnd = random.Random(5)
    for _ in range(200):
        n = rnd.randint(1, 12)
        fps = [rnd.randint(1, 6) * GB for _ in range(n)]
        waits = [rnd.random() for _ in range(n)]
        used = rnd.randint(0, 8) * GB
        slots, bound = rnd.randint(0, 6), rnd.choice([0.0, 0.3, 2.0])
        picks = backfill_choice(fps, waits, used, 10 * GB, slots, bound)
        assert picks == sorted(set(picks)) and len(picks) <= slots
        assert used + sum(fps[i] for i in picks) <= 10 * GB
        # no request is admitted past one that was passed over after waiting its bound
        blocked = [j for j in range(n) if j not in picks and waits[j] >= bound
                   and (not picks or j < picks[-1])]
        assert all(i < min(blocked) for i in picks) if blocked else True
