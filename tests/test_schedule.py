"""Type scheduling of general DAGs (Sec. 4.1-4.2, host only): every rule
gives a node subset sequence that is a partition, causal and homogeneous;
the beam search with a beam wide enough to keep every state finds the
shortest sequence, which a brute-force search over all type strings
confirms; on a graph where the greedy rule is not optimal the default
(shortest of console walk, greedy and beam) is."""
import itertools

import numpy as np
import pytest

import synth
from paper_2509_15948_amd import mixgraph as MG
from paper_2509_15948_amd import workloads as W

PROC = "ecnxsgdr"


def _create(types, edges, rule=0, width=0):
    cfg = W.binding_config(synth.small_config())
    cfg.schedule_rule = rule
    cfg.beam_width = width
    tracks = [0 if t == "i" else -1 for t in types]
    return MG.mg_graph_create([MG.TYPE_CODES[t] for t in types], np.array(edges, np.int32).T.reshape(2, -1),
                              tracks, 1, 2, cfg)


def _schedule(types, edges, rule=0, width=0):
    h = _create(types, edges, rule, width)
    info = MG.mg_graph_info(h)
    po, pi, st, tr, sched = MG.mg_graph_layout(h, len(types), info.n_stages)
    MG.mg_graph_destroy(h)
    return list(st), sched


def _valid(types, edges, st, sched):
    # partition: every node in exactly one stage; homogeneous; causal
    assert len(st) == len(types) and min(st) == 0 and max(st) == len(sched) - 1
    for v, s in enumerate(st):
        assert sched[s] == types[v]
    for a, b in edges:
        assert st[a] < st[b]


def _shortest(types, edges):
    """Brute force: breadth-first search over processed-node sets, each
    step processing every computable node of one type (the output last)."""
    n = len(types)
    preds = [[a for a, b in edges if b == v] for v in range(n)]
    start = frozenset(v for v in range(n) if types[v] == "i")
    frontier, depth = {start}, 1
    while True:
        if any(len(s) == n for s in frontier):
            return depth
        nxt = set()
        for s in frontier:
            ready = {}
            for v in range(n):
                if v not in s and all(p in s for p in preds[v]):
                    ready.setdefault(types[v], []).append(v)
            for t, vs in ready.items():
                if t == "o" and len(ready) > 1:
                    continue
                nxt.add(s | frozenset(vs))
        frontier, depth = nxt, depth + 1


def _random_dag(rng, n_in=2, n_mid=8):
    types = ["i"] * n_in + [str(rng.choice(list(PROC + "m"))) for _ in range(n_mid)] + ["o"]
    edges = []
    n = len(types)
    for v in range(n_in, n - 1):
        k = 1 if types[v] != "m" else int(rng.integers(1, 3))
        srcs = rng.choice(v, size=min(k, v), replace=False)
        edges += [(int(s), v) for s in srcs]
    # every node without a consumer feeds the output
    has_out = {a for a, _ in edges}
    edges += [(v, n - 1) for v in range(n - 1) if v not in has_out]
    return types, edges


@pytest.mark.parametrize("seed", range(25))
def test_wide_beam_is_shortest_and_every_rule_is_valid(seed):
    rng = np.random.default_rng(seed)
    types, edges = _random_dag(rng)
    best = _shortest(types, edges)
    lens = {}
    for rule in (0, 1, 2, 3):
        st, sched = _schedule(types, edges, rule, 4096)
        _valid(types, edges, st, sched)
        lens[rule] = len(sched)
    assert lens[3] == best
    assert lens[0] == min(lens[1], lens[2], lens[3])
    assert min(lens.values()) >= best


def test_beam_beats_greedy_where_greedy_is_short_sighted():
    """A DAG with fan-out where the greedy rule (the type with the most
    computable nodes) needs 10 stages; the shortest sequence has 8, which an
    8-wide beam finds and the default rule returns."""
    types = ["i", "i", "i", "r", "g", "s", "n", "n", "e", "e", "e", "c", "o"]
    edges = [(2, 3), (2, 4), (4, 5), (3, 6), (4, 7), (7, 8), (6, 9), (6, 10), (5, 11), (0, 12), (1, 12), (8, 12),
             (9, 12), (10, 12), (11, 12)]
    assert _shortest(types, edges) == 8
    st, g_sched = _schedule(types, edges, 2)
    _valid(types, edges, st, g_sched)
    st, b_sched = _schedule(types, edges, 3, 8)
    _valid(types, edges, st, b_sched)
    _, d_sched = _schedule(types, edges, 0)
    assert len(g_sched) == 10
    assert len(b_sched) == 8 and len(d_sched) == 8


def test_console_schedule_unchanged_by_the_default_rule():
    g = synth.make_console(5, synth.subgroup_labels(1, 5, 2), "ecxsgdr")
    st, sched = _schedule(g.types, g.edges, 0)
    assert sched == "iecxsgdrmecxsgdro"
