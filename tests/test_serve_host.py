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


def test_threshold_is_carried_across_rounds():
    """Alg. 2 takes L_min once, from the trained console, and only lowers it.
    Fine-tuning on the smaller graph drifts the loss up by 0.9 tau per round
    in this synthetic table.  A threshold reset to the current loss every
    round would keep accepting, and the accepted loss would end near
    L0 (1 + 9 tau).  Every accepted prefix must stay below L0 (1 + tau)."""
    import numpy as np
    from paper_2509_15948_amd.serve import PruneThreshold
    tau, L0 = 1e-3, 0.5
    thr = PruneThreshold(tau)
    accepted = []
    for r in range(10):
        L_now = L0 * (1 + 0.9 * tau * r)       # the console's loss this round
        thr.observe(L_now)
        cand = np.arange(4, dtype=np.int32)
        L_cand = L_now * (1 + np.array([1e-5, 2e-5, 3e-5, 5e-3]))
        order = thr.order(cand, L_cand)
        L_prefix = L_now * (1 + np.cumsum([1e-5, 2e-5, 3e-5][:len(order)]))
        k = thr.accept(L_prefix) if len(order) else 0
        if k:
            accepted.append(float(L_prefix[k - 1]))
    assert thr.L_min == L0 or thr.L_min < L0
    assert accepted and all(a < L0 * (1 + tau) for a in accepted), accepted
    # rounds whose loss has drifted past the tolerance accept nothing
    assert len(accepted) == 2
