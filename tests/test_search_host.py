"""Host-side summaries of the search driver (no GPU): the rank correlation
of a candidate's dry/wet weight with the loss increase of bypassing it."""
import numpy as np
import scipy.stats

from paper_2509_15948_amd import search as S


def test_ranks_give_ties_their_mean_rank():
    assert S._ranks(np.array([3.0, 1.0, 2.0, 2.0])).tolist() == [3.0, 0.0, 1.5, 1.5]


def test_w_delta_summary_matches_a_library_spearman():
    rng = np.random.default_rng(5)
    w = rng.random(80)
    d = 0.05 * w ** 2 + 0.01 * rng.standard_normal(80)
    d[::7] = d[0]  # ties
    types = rng.integers(3, 11, 80)
    out = S.w_delta_summary(list(zip(w.tolist(), d.tolist(), types.tolist())), tau=0.01)
    ref = scipy.stats.spearmanr(w, d).statistic
    assert abs(out["spearman_w_delta"] - ref) < 1e-4
    assert out["candidates"] == 80
    assert sum(b["n"] for b in out["by_w_quarter"]) == 80
    # a monotone relation ranks perfectly
    mono = S.w_delta_summary([(float(x), float(x) ** 3, 3) for x in w], tau=0.01)
    assert mono["spearman_w_delta"] == 1.0
    assert S.w_delta_summary([], tau=0.01) == {}
