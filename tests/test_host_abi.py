"""Host-side tests of the C-ABI library (no GPU needed): symbols, graph
validation and error codes, type schedule (Sec. 4.1-4.2), node order and
parameter layout (Alg. 1 Reorder), pruning surgery (Sec. 1.2 bypass)."""
import ctypes
import os
import re

import numpy as np
import pytest
import torch

import synth
from oracle import train as TR
from paper_2509_15948_amd import mixgraph as MG
from paper_2509_15948_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "mixgraph.h")).read()
    declared = sorted(set(re.findall(r"\b(mg_[a-z_]+)\s*\(", hdr)))
    assert len(declared) >= 12
    L = MG.lib()
    for name in declared:
        assert hasattr(L, name), name
    assert set(MG.EXPORTS) <= set(declared)


def _graph(chain="ecxsgdr", K=5, S=2, **kw):
    cfg = synth.small_config(n_tracks=K, n_subgroups=S, chain=chain, **kw)
    g = synth.make_console(K, synth.subgroup_labels(1, K, S), chain)
    return cfg, g, W.binding_graph(g, cfg)


@pytest.mark.parametrize("chain", ["ecxsgdr", "ecnsgdr", "ecg"])
def test_console_schedule_is_the_console_type_string(chain):
    cfg, g, bg = _graph(chain, comp_mode="single")
    assert bg.schedule == "i" + chain + "m" + chain + "o"
    # partition, causal and homogeneous (Sec. 4.1)
    for s, d in g.edges:
        assert bg.stage[s] < bg.stage[d]
    for st in range(bg.info.n_stages):
        ts = {g.types[v] for v in range(g.n_nodes) if bg.stage[v] == st}
        assert len(ts) == 1


def test_layout_is_type_major_and_contiguous_per_stage():
    cfg, g, bg = _graph()
    np_of = {t: cfg.n_params(t) for t in "ecnxsgdr"}
    offs = []
    for v in g.processors():
        offs.append((int(bg.param_offset[v]), np_of[g.types[v]], v))
    offs.sort()
    pos = 0
    for o, n, v in offs:
        assert o == pos, (o, pos, g.types[v])
        pos += n
    assert pos == bg.n_theta
    assert sorted(int(bg.proc_index[v]) for v in g.processors()) == list(range(len(g.processors())))
    # rows of one stage are consecutive
    for st in range(1, bg.info.n_stages):
        rows = sorted(int(bg.type_row[v]) for v in range(g.n_nodes) if bg.stage[v] == st)
        assert rows == list(range(rows[0], rows[0] + len(rows)))


def _create(types, edges, tracks=None, n_tracks=1):
    cfg = W.binding_config(synth.small_config())
    if tracks is None:
        tracks = [0 if t == "i" else -1 for t in types]
    return MG.mg_graph_create([MG.TYPE_CODES[t] for t in types], np.array(edges, np.int32).T.reshape(2, -1),
                              tracks, n_tracks, 2, cfg)


def test_error_codes():
    with pytest.raises(MG.MixgraphError, match="error 2"):       # cycle
        _create(["i", "g", "s", "o"], [(0, 1), (1, 2), (2, 1), (2, 3)])
    with pytest.raises(MG.MixgraphError, match="error 2"):       # two outputs
        _create(["i", "g", "o", "o"], [(0, 1), (1, 2), (1, 3)])
    with pytest.raises(MG.MixgraphError, match="error 2"):       # processor without input
        _create(["i", "g", "s", "o"], [(0, 1), (1, 3), (2, 3)])
    with pytest.raises(MG.MixgraphError, match="error 2"):       # dangling node
        _create(["i", "g", "s", "o"], [(0, 1), (1, 3), (1, 2)])
    with pytest.raises(MG.MixgraphError, match="error 2"):       # unknown type
        cfg = W.binding_config(synth.small_config())
        MG.mg_graph_create([0, 42, 2], np.array([[0, 1], [1, 2]], np.int32), [0, -1, -1], 1, 2, cfg)
    with pytest.raises(MG.MixgraphError, match="error 1"):       # bad config (even EQ length)
        cfg = W.binding_config(synth.small_config(eq_taps=254))
        MG.mg_graph_create([0, 3, 2], np.array([[0, 1], [1, 2]], np.int32), [0, -1, -1], 1, 2, cfg)
    L = MG.lib()
    assert L.mg_forward(None, None, None, None, None, None, None, None) == 1
    assert L.mg_backward(None, None, None, None) == 1
    assert L.mg_node_output(None, 0, None, None) == 1


def test_decision_rule_rejects_a_nonfinite_threshold():
    """A search whose own loss is NaN or infinite has failed: the rule says so
    (MG_ERR_NONFINITE) instead of deciding.  A NaN trial loss only fails its
    own test."""
    cand = np.array([3, 1, 2], np.int32)
    for bad in (float("nan"), float("inf")):
        with pytest.raises(MG.MixgraphError, match="error 8"):
            MG.mg_prune_order(cand, np.array([1.0, 1.0, 1.0]), bad, 1e-3)
        with pytest.raises(MG.MixgraphError, match="error 8"):
            MG.mg_prune_accept(np.array([1.0]), bad, 1e-3)
    order = MG.mg_prune_order(cand, np.array([1.0, float("nan"), 1.0000001]), 1.0, 1e-3)
    assert order.tolist() == [3, 2]
    assert MG.mg_prune_accept(np.array([1.0, float("nan")]), 1.0, 1e-3) == 1


def test_greedy_schedule_for_a_general_dag():
    # i -> e -> c -> o ; i -> c -> s ... a DAG that is not a console
    types = ["i", "i", "e", "c", "c", "s", "m", "g", "o"]
    edges = [(0, 2), (2, 3), (1, 4), (3, 6), (4, 5), (5, 6), (6, 7), (7, 8)]
    h = _create(types, edges, tracks=[0, 0, -1, -1, -1, -1, -1, -1, -1])
    info = MG.mg_graph_info(h)
    po, pi, st, tr, sched = MG.mg_graph_layout(h, len(types), info.n_stages)
    for s, d in edges:
        assert st[s] < st[d]
    assert sched[0] == "i" and sched[-1] == "o"
    assert len(sched) <= 7      # i, e/c, c, s, m, g, o at most
    MG.mg_graph_destroy(h)


def test_workspace_size_positive_and_mode_monotone():
    cfg, g, bg = _graph()
    a = MG.mg_workspace_size(bg.h, 0)
    b = MG.mg_workspace_size(bg.h, 1)
    assert 0 < a < b


def test_prune_is_bypass_in_the_oracle():
    """Removing processors by graph surgery equals zeroing their dry/wet."""
    cfg = synth.small_config(seconds=0.1, fs=8000, n_tracks=3, n_subgroups=2, loss_ffts=(256,), eq_taps=31,
                             delay_range_s=0.04, reverb_seconds=0.05)
    g, dry, noise = synth.song(2, cfg)
    bg = W.binding_graph(g, cfg)
    th, we = synth.random_params(2, g, cfg)
    procs = g.processors()
    rng = np.random.default_rng(0)
    drop = set(int(v) for v in rng.choice(procs, size=len(procs) // 2, replace=False))
    keep = np.ones(bg.n_proc, np.uint8)
    for v in drop:
        keep[int(bg.proc_index[v])] = 0
    pg, o2n = bg.prune(keep)
    masked = TR.render(g, cfg, dry, noise, th, we, {v: 0.0 for v in drop})
    # rebuild the pruned graph for the oracle from the library's edges
    import synth as S
    new_types = pg.types
    n = len(new_types)
    # map parameters
    th2 = {int(o2n[v]): th[v] for v in procs if v not in drop}
    we2 = {int(o2n[v]): we[v] for v in procs if v not in drop}
    noise2 = {int(o2n[v]): noise[v] for v in noise if v not in drop}
    # edges of the pruned graph: rebuild by bypass rule in python for the oracle
    keep_nodes = [v for v in range(g.n_nodes) if v not in drop]
    preds = {v: [] for v in range(g.n_nodes)}
    for s_, d_ in g.edges:
        preds[d_].append(s_)
    edges = []
    for v in keep_nodes:
        stack = list(preds[v])
        srcs = set()
        while stack:
            p = stack.pop()
            if p in drop:
                stack.extend(preds[p])
            else:
                srcs.add(p)
        edges += [(int(o2n[p]), int(o2n[v])) for p in sorted(srcs)]
    tin = {int(o2n[v]): k for v, k in g.track_of_input.items()}
    g2 = S.Graph(new_types, edges, tin)
    mix2 = TR.render(g2, cfg, dry, noise2, th2, we2)
    assert np.allclose(mix2, masked, rtol=1e-12, atol=1e-14)
    assert pg.schedule.startswith("i") and pg.schedule.endswith("o")
    assert len(pg.schedule) <= len(bg.schedule)


def test_pruning_rule_matches_the_oracle_rule():
    """The C-ABI decision rule (host only) against oracle/prune.py on random
    weights, liveness and losses, ties included."""
    from oracle import prune as OP
    rng = np.random.default_rng(5)
    for trial in range(50):
        P = int(rng.integers(1, 40))
        wet = rng.normal(size=P).astype(np.float32)
        if trial % 5 == 0:
            wet[: P // 2] = wet[0]                       # ties in w
        mask = (rng.random(P) < 0.8).astype(np.float32) if trial % 2 else None
        alive = (rng.random(P) < 0.9).astype(np.uint8)
        n = int(rng.integers(0, P + 3))
        w32 = (np.float32(1.0) / (np.float32(1.0) + np.exp(-wet))).astype(np.float32)
        if mask is not None:
            w32 = w32 * mask
        cand = MG.mg_prune_candidates(wet, mask, alive, n)
        assert cand.tolist() == OP.candidates(w32.tolist(), alive.tolist(), n)
        L_min = 1.0 + rng.random()
        tau = float(rng.choice([1e-3, 1e-2, 0.1]))
        L_cand = L_min + rng.normal(scale=tau * L_min, size=len(cand))
        if len(cand) > 2:
            L_cand[1] = L_cand[0]                         # ties in Delta
        order = MG.mg_prune_order(cand, L_cand, L_min, tau)
        assert order.tolist() == OP.order_within_tolerance(cand.tolist(), L_cand.tolist(), L_min, tau)
        L_prefix = L_min * (1 + tau * rng.normal(size=len(order)))
        assert MG.mg_prune_accept(L_prefix, L_min, tau) == OP.accept_prefix(L_prefix.tolist(), L_min, tau)


def test_static_setup_rejects_a_workspace_beyond_the_scratch():
    """mg_setup_static checks the size on the host before touching a device:
    a graph whose workspace exceeds the static scratch gets MG_ERR_BUDGET."""
    cfg = synth.small_config(seconds=20.0, fs=44100, n_tracks=8, n_subgroups=2, chain="ecxsgdr")
    g = synth.make_console(8, synth.subgroup_labels(1, 8, 2), "ecxsgdr")
    bg = W.binding_graph(g, cfg)
    assert MG.mg_workspace_size(bg.h, 1) > (64 << 20)
    rc = MG.lib().mg_setup_static(bg.h, 1, None, 1, None)
    assert rc == 6, rc  # MG_ERR_BUDGET
    assert b"static scratch" in MG.lib().mg_last_error()


def test_footprint_covers_workspace_and_caller_buffers():
    """mg_footprint: the workspace of mg_workspace_size plus the caller-side
    buffers of one search (dry tracks, noise, target, mix, parameters with
    gradients and two moments, loss records), growing with the length."""
    cfg, g, bg = _graph()
    ws, st = MG.mg_footprint(bg.h, 1)
    assert ws == MG.mg_workspace_size(bg.h, 1)
    L = cfg.length
    floor = cfg.n_tracks * 2 * L * 4 + 4 * 4 * (bg.n_theta + bg.n_proc) + 2 * 2 * L * 4
    assert st >= floor
    cfg2, g2, bg2 = _graph(seconds=2 * cfg.seconds)
    ws2, st2 = MG.mg_footprint(bg2.h, 1)
    assert ws2 > ws and st2 > st


def test_build_rejects_kernels_that_use_scratch():
    """The build's scan of the compiler's resource remarks finds each kernel
    with nonzero scratch bytes per lane and nothing else; only the listed EQ
    window kernels may use any."""
    from paper_2509_15948_amd.build import scratch_kernels
    remarks = "\n".join([
        "k.hip:10:1: remark: Function Name: _Z5k_onePf [-Rpass-analysis=kernel-resource-usage]",
        "k.hip:10:1: remark:     VGPRs: 40 [-Rpass-analysis=kernel-resource-usage]",
        "k.hip:10:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]",
        "k.hip:20:1: remark: Function Name: _Z5k_twoPf [-Rpass-analysis=kernel-resource-usage]",
        "k.hip:20:1: remark:     ScratchSize [bytes/lane]: 64 [-Rpass-analysis=kernel-resource-usage]",
    ])
    assert scratch_kernels(remarks) == [("_Z5k_twoPf", 64)]
    assert scratch_kernels("") == []
    from paper_2509_15948_amd.build import _allowed
    assert _allowed("_ZN2mg8k_eq_bwdENS_6EqArgsE") == 32
    assert _allowed("_ZN2mg8k_eq_fwdENS_6EqArgsE") == 0
    assert _allowed("_ZN2mg6k_colsILi1024ELi8ENS_5LdFirEEEvT1_P15HIP_vector_typeIfLj2EENS_10EngineArgsE") == 0
