"""Host logic of the serving loop (no GPU): admission by memory budget and
slots, and the request generator."""
import synth
from paper_2509_15948_amd.serve import Admission


def test_admission_respects_budget_and_slots():
    a = Admission(budget_bytes=100, max_active=2)
    assert a.can_admit(60)
    a.admit(60)
    assert not a.can_admit(50)          # over budget
    assert a.can_admit(40)
    a.admit(40)
    assert not a.can_admit(1)           # slots and budget full
    a.retire(60)
    assert a.can_admit(60) and not a.can_admit(61)
    a.retire(40)
    assert a.used == 0 and a.active == 0


def test_a_request_larger_than_the_budget_runs_alone():
    a = Admission(budget_bytes=100, max_active=4)
    assert a.can_admit(500)             # nothing active: it may start
    a.admit(500)
    assert not a.can_admit(1)
    a.retire(500)


def test_serving_requests_are_seeded_and_in_range():
    r1 = synth.serving_requests(7, 50, rate=3.0)
    r2 = synth.serving_requests(7, 50, rate=3.0)
    assert [(t, c.n_tracks, c.n_subgroups, c.seconds, s) for t, c, s in r1] == \
           [(t, c.n_tracks, c.n_subgroups, c.seconds, s) for t, c, s in r2]
    times = [t for t, _, _ in r1]
    assert times == sorted(times) and times[0] > 0
    for _, c, _ in r1:
        assert 4 <= c.n_tracks <= 32 and 2 <= c.n_subgroups <= min(8, c.n_tracks)
        assert 5.0 <= c.seconds <= 30.0
    # mean gap close to 1 / rate
    gaps = [b - a for a, b in zip(times, times[1:])]
    assert 0.15 < sum(gaps) / len(gaps) < 0.6
