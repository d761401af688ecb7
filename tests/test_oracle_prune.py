"""Pins of the oracle's pruning-round rule (oracle/prune.py): a hand-worked
additive example, tie-breaking, limiting tolerances, and brute force over
every mask of a small console evaluated by the oracle itself."""
import itertools

import numpy as np
import pytest
import torch

import synth
from oracle import console as OC
from oracle import loss as LS
from oracle import prune as PR
from oracle import train as TR


def additive(L0, c):
    """L(mask) = L0 + sum of c_j over bypassed j."""
    return lambda alive: L0 + sum(cj for cj, a in zip(c, alive) if not a)


def test_hand_worked_round():
    # w orders the candidates p1 (0.1), p5 (0.2), p3 (0.3), p2 (0.5); p2 costs
    # more than tau * L0 = 1e-3 alone; the others in Delta order p3, p5, p1
    # give prefix losses 1.0002, 1.0006, 1.0011, so the first two go.
    w = [0.9, 0.1, 0.5, 0.3, 0.7, 0.2]
    c = [0.0, 0.0005, 0.002, 0.0002, 0.0, 0.0004]
    alive, L_new, info = PR.prune_round(additive(1.0, c), [True] * 6, w, 1.0, tau=1e-3, max_candidates=4)
    assert info["candidates"] == [1, 5, 3, 2]
    assert info["order"] == [3, 5, 1]
    assert np.allclose(info["L_prefix"], [1.0002, 1.0006, 1.0011])
    assert info["k"] == 2
    assert alive == [True, True, True, False, True, False]
    assert L_new == 1.0


def test_improving_bypass_lowers_the_best_loss():
    alive, L_new, info = PR.prune_round(additive(2.0, [-0.5, 0.0001]), [True, True], [0.2, 0.1], 2.0, tau=1e-3)
    assert info["order"] == [0, 1]           # Delta -0.5 first, then 1e-4
    assert alive == [False, False]
    assert L_new == pytest.approx(1.5001)


def test_ties_break_by_index():
    w = [0.5, 0.5, 0.5]
    c = [1e-5, 1e-5, 1e-5]
    _, _, info = PR.prune_round(additive(1.0, c), [True] * 3, w, 1.0, tau=1e-3, max_candidates=2)
    assert info["candidates"] == [0, 1]
    assert info["order"] == [0, 1]


def test_dead_processors_are_not_candidates():
    _, _, info = PR.prune_round(additive(1.0, [0, 0, 0]), [True, False, True], [0.1, 0.0, 0.2], 1.0)
    assert info["candidates"] == [0, 2]


def test_limits_of_the_tolerance():
    c = [0.01, 0.02, 0.03]
    alive, _, _ = PR.prune_round(additive(1.0, c), [True] * 3, [0.1, 0.2, 0.3], 1.0, tau=1e9)
    assert alive == [False, False, False]
    alive, _, info = PR.prune_round(additive(1.0, c), [True] * 3, [0.1, 0.2, 0.3], 1.0, tau=0.0)
    assert alive == [True, True, True] and info["order"] == []


def _small_console():
    cfg = synth.small_config(seconds=0.3, fs=8000, n_tracks=2, n_subgroups=1, chain="eg", stereo_tracks=False,
                             eq_taps=63, loss_ffts=(256, 512))
    g, dry, noise = synth.song(11, cfg)
    return cfg, g, dry, noise


def test_brute_force_over_every_mask_of_a_small_console():
    """Every mask of a 6-processor console evaluated by the oracle; the round's
    result must be jointly within tolerance, maximal along its order, and made
    of processors that were each within tolerance alone."""
    cfg, g, dry, noise = _small_console()
    procs = g.processors()
    P = len(procs)
    assert P <= 8
    gt, gw = synth.ground_truth_params(111, g, cfg)
    target = TR.render(g, cfg, dry, noise, gt, gw)
    th, we = synth.random_params(11, g, cfg, std=0.3)
    table = {}
    for bits in itertools.product([True, False], repeat=P):
        mask = {v: (1.0 if b else 0.0) for v, b in zip(procs, bits)}
        table[bits] = TR.losses(g, cfg, dry, noise, target, th, we, mask)["La"]
    L_min = table[(True,) * P]
    w = [1.0 / (1.0 + np.exp(-we[v])) for v in procs]
    # a tolerance that lets some, not all, processors go
    deltas = sorted(table[tuple(i != j for i in range(P))] - L_min for j in range(P))
    tau = float(np.median(deltas) / L_min)
    if tau <= 0:
        tau = 1e-3
    alive, L_new, info = PR.prune_round(lambda a: table[tuple(bool(x) for x in a)], [True] * P, w, L_min, tau=tau)
    k = info["k"]
    if k:
        assert table[tuple(alive)] < L_min * (1 + tau)
        assert L_new == min(L_min, table[tuple(alive)])
    for kk in range(k + 1, len(info["order"]) + 1):
        m = [True] * P
        for j in info["order"][:kk]:
            m[j] = False
        assert table[tuple(m)] >= L_min * (1 + tau)
    for j in info["order"]:
        single = tuple(i != j for i in range(P))
        assert table[single] - L_min < tau * L_min
    dropped = [j for j in range(P) if not alive[j]]
    assert dropped == sorted(info["order"][:k])


def test_bypass_mask_equals_the_pruned_graph():
    """Sec. 1.2: bypassing a processor (w = 0) and deleting it with its edges
    rerouted give the same mix."""
    cfg, g, dry, noise = _small_console()
    th, we = synth.random_params(12, g, cfg, std=0.3)
    drop = g.processors()[1]
    mix_masked = TR.render(g, cfg, dry, noise, th, we, {drop: 0.0})
    keep = [v for v in range(g.n_nodes) if v != drop]
    new_id = {v: i for i, v in enumerate(keep)}
    edges = []
    for s, d in g.edges:
        if d == drop:
            continue
        if s == drop:
            for s2, d2 in g.edges:
                if d2 == drop:
                    edges.append((new_id[s2], new_id[d]))
        else:
            edges.append((new_id[s], new_id[d]))
    g2 = synth.Graph([g.types[v] for v in keep], edges, {new_id[v]: t for v, t in g.track_of_input.items()})
    th2 = {new_id[v]: p for v, p in th.items() if v != drop}
    we2 = {new_id[v]: x for v, x in we.items() if v != drop}
    mix_pruned = TR.render(g2, cfg, dry, noise, th2, we2)
    assert np.array_equal(mix_masked, mix_pruned)
