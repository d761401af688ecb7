"""A general processing graph (not a console) through the C-ABI against the
oracle: processors with several inputs (their input is the sum), nodes with
several consumers (a send to a second bus; the backward sums what each
consumer passes back), a mix feeding two processors, every processor type;
the type schedule the library picks for it (shortest of console walk, greedy
and beam).  Mix, every node output, losses and gradients.

The songs run 2 s at 16 kHz: at 0.75 s the oracle's own gradients of these
graphs move by 0.2-4 % (EQ, delay, reverb) when FP32-level noise is added at
every processor output, more than the stated 1e-3, so no FP32 implementation
could be held to it there; at 2 s that sensitivity is 1e-4 to 2e-3.  Losses
and gradients are held to the same oracle-derived bounds as the per-type
console cases (the stated tolerance, or 3 x the measured sensitivity up to
10 x the stated tolerance)."""
import types
import numpy as np
import pytest
import torch

import synth
from oracle import console as OC
from oracle import train as TR
from paper_2509_15948_amd import mixgraph as MG
from paper_2509_15948_amd import workloads as W

from gpu_cases import f32, grad_tolerances, loss_tolerances, rel_l2

pytestmark = pytest.mark.gpu


def _dag(kind="both"):
    if kind == "multi":
        # a processor with two inputs, no fan-out: e(3) -> c(4) and x(5) -> s(6)
        types = ["i", "i", "i", "e", "c", "x", "s", "g", "m", "r", "o"]
        edges = [(0, 3), (3, 4), (1, 5), (4, 6), (5, 6), (2, 7), (6, 8), (7, 8), (8, 9), (9, 10)]
        return synth.Graph(types, edges, {0: 0, 1: 1, 2: 2})
    if kind == "fanout":
        # fan-out only: c(4) feeds g(5) and d(6); m(7) sums them
        types = ["i", "i", "e", "c", "g", "d", "m", "x", "o"]
        edges = [(0, 2), (2, 3), (3, 4), (3, 5), (4, 6), (5, 6), (1, 7), (7, 6), (6, 8)]
        return synth.Graph(types, edges, {0: 0, 1: 1})
    # both: 0,1,2 inputs.  0 -> e(3) -> c(4) ; 1 -> x(5) ; 2 -> g(6)
    # c(4) and x(5) -> s(7) (two inputs); c(4) also -> d(8) (send)
    # g(6) -> m(9); s(7) -> m(9); d(8) -> r(10) ; m(9) -> n(11) and -> e(12)
    # r(10), n(11), e(12) -> o(13)
    types = ["i", "i", "i", "e", "c", "x", "g", "s", "d", "m", "r", "n", "e", "o"]
    edges = [(0, 3), (3, 4), (1, 5), (2, 6), (4, 7), (5, 7), (4, 8), (6, 9), (7, 9), (8, 10), (9, 11), (9, 12),
             (10, 13), (11, 13), (12, 13)]
    return synth.Graph(types, edges, {0: 0, 1: 1, 2: 2})


@pytest.mark.parametrize("kind", ["multi", "fanout", "both"])
def test_general_dag_against_the_oracle(kind):
    g = _dag(kind)
    n_in = sum(1 for t in g.types if t == "i")
    cfg = synth.small_config(seconds=2.0, fs=16000, n_tracks=n_in, n_subgroups=1)
    dry = synth.dry_tracks(21, cfg)
    noise = synth.reverb_noise_all(21, g, cfg)
    gt, gw = synth.ground_truth_params(121, g, cfg)
    target = TR.render(g, cfg, dry, noise, gt, gw).astype(np.float32)
    th, we = synth.random_params(21, g, cfg, std=0.3)
    th = {v: f32(p) for v, p in th.items()}
    we = {v: float(np.float32(w)) for v, w in we.items()}
    bg = W.binding_graph(g, cfg, 1e-3, 1e-2)
    print("schedule", bg.schedule, flush=True)
    noise_d = torch.from_numpy(W.noise_rows(bg, noise, cfg.reverb_length)).cuda()
    sess = MG.Session(bg, noise_d, torch.from_numpy(target).cuda(), mode=1)
    th_f, we_f = bg.flatten(th, we)
    theta, wet = torch.from_numpy(th_f).cuda(), torch.from_numpy(we_f).cuda()
    mix = torch.empty(2, cfg.length, device="cuda")
    losses = torch.zeros(7, dtype=torch.float64, device="cuda")
    dry_d = torch.from_numpy(dry).cuda()   # read again by the backward: kept alive
    sess.forward(dry_d, theta, wet, None, mix, losses)
    nodes = {}
    buf = torch.empty(2, cfg.length, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    for v, t in enumerate(g.types):
        if t != "i":
            MG.mg_node_output(bg.h, v, buf, st)
            torch.cuda.synchronize()
            nodes[v] = buf.cpu().numpy().astype(np.float64)
    gth = torch.empty_like(theta)
    gwe = torch.empty_like(wet)
    sess.backward(gth, gwe)
    torch.cuda.synchronize()
    vals, oth, owe, omix = TR.loss_and_grad(g, cfg, dry, noise, target.astype(np.float64), th, we, None, 1e-3, 1e-2)
    with torch.no_grad():
        ev = OC.evaluate(g, cfg, dry, noise, {v: torch.tensor(p) for v, p in th.items()},
                         {v: torch.tensor(w, dtype=torch.float64) for v, w in we.items()}, None, keep_nodes=True)
    err = rel_l2(mix.cpu().numpy(), omix)
    print("dag wave", err, flush=True)
    assert err <= 1e-4
    for v, y in nodes.items():
        e = rel_l2(y, ev["y"][v].numpy())
        print("node", v, g.types[v], e, flush=True)
        assert e <= 1e-4, (v, g.types[v], e)
    gl = dict(zip(MG.LOSS_KEYS, losses.cpu().numpy().tolist()))
    case = types.SimpleNamespace(g=g, cfg=cfg, dry=dry, noise=noise, th=th, we=we, target=target, alpha_g=1e-3,
                                 alpha_p=1e-2)
    ltol = loss_tolerances(case)
    for k in ("La", "Llr", "Lm", "Ls", "Lg", "Lp", "L"):
        bound = max(1e-5 * abs(vals[k]), ltol[k])
        print("loss", k, gl[k], vals[k], "err", abs(gl[k] - vals[k]), "bound", bound, flush=True)
        assert abs(gl[k] - vals[k]) <= bound or abs(gl[k] - vals[k]) < 1e-9, k
    sizes = {v: len(p) for v, p in th.items()}
    gth_h, gwe_h = bg.unflatten(gth.cpu().numpy(), gwe.cpu().numpy(), sizes)
    for v in g.processors():
        print("grad", v, g.types[v], rel_l2(gth_h[v], oth[v]), flush=True)
    tol, sens = grad_tolerances(case, oth, owe)
    procs = g.processors()
    bad = []
    for t in sorted({g.types[v] for v in procs}):
        vs = [v for v in procs if g.types[v] == t]
        e = rel_l2(np.concatenate([gth_h[v] for v in vs]), np.concatenate([oth[v] for v in vs]))
        print(kind, t, "grad err", e, "oracle FP32 sensitivity", sens[t], "bound", tol[t], flush=True)
        if e > tol[t]:
            bad.append((t, e, tol[t]))
    e = rel_l2([gwe_h[v] for v in procs], [owe[v] for v in procs])
    print(kind, "wet grad err", e, "oracle FP32 sensitivity", sens["w"], "bound", tol["w"], flush=True)
    assert not bad, bad
    assert e <= tol["w"]
