"""The paper's training regime through the C-ABI: AdamW against the oracle's
update, a new target (mg_target_prepare) against a session set up on it,
regulariser weights set at run time (mg_set_alpha) against a graph compiled
with them, the warm-up skip of a segment against the oracle, and a short
search (console phase, hybrid pruning iterations, graph surgery)."""
import dataclasses

import numpy as np
import pytest
import torch

import synth
from oracle import train as TR
from paper_2509_15948_amd import mixgraph as MG
from paper_2509_15948_amd import search as SR
from paper_2509_15948_amd import workloads as W

from gpu_cases import Case, grad_tolerances, loss_tolerances, rel_l2

pytestmark = pytest.mark.gpu


def _small(chain="ecnsgdr", **kw):
    base = dict(seconds=0.75, fs=16000, n_tracks=3, n_subgroups=2, chain=chain)
    base.update(kw)
    return synth.small_config(**base)


def test_adamw_matches_the_oracle_update():
    rng = np.random.default_rng(3)
    n = 100003
    th = rng.normal(size=n).astype(np.float32)
    m = (0.1 * rng.normal(size=n)).astype(np.float32)
    v = (0.01 * rng.random(n)).astype(np.float32)
    g = rng.normal(size=n).astype(np.float32)
    d = [torch.from_numpy(x.copy()).cuda() for x in (th, m, v, g)]
    st = torch.cuda.current_stream().cuda_stream
    MG.mg_adamw_step(d[0], d[1], d[2], d[3], n, 1e-2, 0.9, 0.999, 1e-8, 0.05, 7, st)
    torch.cuda.synchronize()
    t64, m64, v64 = th.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    # the kernel sees the FP32 values of the hyper-parameters (1 - beta2 in
    # FP32 differs from 0.001 by 1.3e-5 relative)
    f = lambda x: float(np.float32(x))
    TR.adamw_step(t64, m64, v64, g.astype(np.float64), 7, lr=f(1e-2), b1=f(0.9), b2=f(0.999), eps=f(1e-8),
                  weight_decay=f(0.05))
    err = np.abs(d[0].cpu().numpy() - t64).max()
    print("adamw max abs err", err, flush=True)
    assert err < 1e-6
    assert rel_l2(d[1].cpu().numpy(), m64) < 1e-6 and rel_l2(d[2].cpu().numpy(), v64) < 1e-6
    # weight decay 0 is Adam, bit for bit
    a = [torch.from_numpy(x.copy()).cuda() for x in (th, m, v, g)]
    b = [torch.from_numpy(x.copy()).cuda() for x in (th, m, v, g)]
    MG.mg_adamw_step(a[0], a[1], a[2], a[3], n, 1e-2, 0.9, 0.999, 1e-8, 0.0, 3, st)
    MG.mg_adam_step(b[0], b[1], b[2], b[3], n, 1e-2, 0.9, 0.999, 1e-8, 3, st)
    torch.cuda.synchronize()
    assert all(torch.equal(x, y) for x, y in zip(a, b))


def test_new_target_equals_a_session_set_up_on_it():
    case = Case(_small(), alpha_p=1e-2)
    other = torch.from_numpy((0.7 * case.target[::-1]).copy()).cuda()
    MG.mg_target_prepare(case.bg.h, other, torch.cuda.current_stream().cuda_stream)
    mix, gl = case.gpu_forward()
    gth, gwe = case.gpu_backward()
    bg2 = W.binding_graph(case.g, case.cfg, 1e-3, 1e-2)
    s2 = MG.Session(bg2, case.noise_d, other, mode=1)
    out = torch.zeros(7, dtype=torch.float64, device="cuda")
    s2.forward(case.dry_d, case.theta_d, case.wet_d, None, None, out)
    g2t = torch.empty(bg2.n_theta, device="cuda")
    g2w = torch.empty(bg2.n_proc, device="cuda")
    s2.backward(g2t, g2w)
    torch.cuda.synchronize()
    assert out.cpu().numpy().tolist() == [gl[k] for k in MG.LOSS_KEYS]
    t, w = bg2.unflatten(g2t.cpu().numpy(), g2w.cpu().numpy(), case.sizes)
    assert all(np.array_equal(t[v], gth[v]) for v in t) and w == gwe
    # a pending backward is dropped by a new target
    case.gpu_forward()
    MG.mg_target_prepare(case.bg.h, other, torch.cuda.current_stream().cuda_stream)
    with pytest.raises(MG.MixgraphError):
        case.gpu_backward()


def test_weights_set_at_run_time_equal_compiled_weights():
    case = Case(_small(), alpha_g=1e-3, alpha_p=0.0)
    MG.mg_set_alpha(case.bg.h, 2e-3, 5e-2)
    mix, gl = case.gpu_forward()
    with pytest.raises(MG.MixgraphError):
        MG.mg_set_alpha(case.bg.h, 1e-3, 0.0)   # between a forward and its backward
    gth, gwe = case.gpu_backward()
    ref = Case(_small(), alpha_g=2e-3, alpha_p=5e-2)
    mix2, gl2 = ref.gpu_forward()
    gth2, gwe2 = ref.gpu_backward()
    assert gl == gl2
    assert all(np.array_equal(gth[v], gth2[v]) for v in gth) and gwe == gwe2


def test_warm_up_skip_against_the_oracle():
    """A 1.2 s segment at 16 kHz whose first 0.5 s is excluded from the loss
    (the loss frames lie inside [skip, L)): losses and gradients against the
    oracle with the same skip."""
    cfg = _small(seconds=1.2)
    case = Case(cfg, alpha_p=1e-2)
    skip = 8000
    bg = MG.Graph(case.g.types, case.g.edge_array(), [case.g.track_of_input.get(v, -1) for v in range(case.g.n_nodes)],
                  cfg.n_tracks, 2, W.binding_config(cfg, 1e-3, 1e-2, loss_skip=skip))
    sess = MG.Session(bg, case.noise_d, case.target_d, mode=1)
    out = torch.zeros(7, dtype=torch.float64, device="cuda")
    sess.forward(case.dry_d, case.theta_d, case.wet_d, None, None, out)
    gt = torch.empty(bg.n_theta, device="cuda")
    gw = torch.empty(bg.n_proc, device="cuda")
    sess.backward(gt, gw)
    torch.cuda.synchronize()
    gl = dict(zip(MG.LOSS_KEYS, out.cpu().numpy().tolist()))
    vals, oth, owe, _ = TR.loss_and_grad(case.g, cfg, case.dry, case.noise, case.target.astype(np.float64),
                                         case.th, case.we, None, 1e-3, 1e-2, skip)
    full = TR.losses(case.g, cfg, case.dry, case.noise, case.target.astype(np.float64), case.th, case.we, None,
                     1e-3, 1e-2)
    assert abs(vals["La"] - full["La"]) > 1e-3 * abs(full["La"])     # the skip changes the loss
    for k in ("La", "Llr", "Lm", "Ls"):
        print("skip loss", k, gl[k], vals[k], flush=True)
        assert abs(gl[k] - vals[k]) <= 1e-4 * abs(vals[k]), k
    gth, gwe = bg.unflatten(gt.cpu().numpy(), gw.cpu().numpy(), case.sizes)
    procs = case.g.processors()
    for t in sorted({case.g.types[v] for v in procs}):
        vs = [v for v in procs if case.g.types[v] == t]
        e = rel_l2(np.concatenate([gth[v] for v in vs]), np.concatenate([oth[v] for v in vs]))
        print("skip grad", t, e, flush=True)
        assert e <= 1e-2, t


def test_short_search_runs_the_regime_end_to_end():
    """Console phase on random segments, then hybrid iterations (dry/wet on
    1-3, brute force on 4) with graph surgery and an alpha_p ramp; the
    result's kept mask matches its processor count, and the final L_a is the
    evaluation graph's loss at the final parameters."""
    cfg = _small(seconds=2.0)
    g, dry, noise = synth.song(5, cfg)
    gt, gw = synth.ground_truth_params(105, g, cfg)
    target = TR.render(g, cfg, dry, noise, gt, gw).astype(np.float32)
    th0, we0 = synth.init_params(5, g, cfg)
    reg = SR.Regime(console_steps=40, rounds=4, finetune=10, segment_s=1.0, warmup_s=0.25, alpha_p_ramp=20,
                    tau=0.05, sampler="hybrid", seed=1)
    res = SR.run_search(g, cfg, dry, noise, target, reg, th0, we0, log=print)
    print({k: res[k] for k in ("La_console", "La_final", "processors_start", "processors_end")}, flush=True)
    assert [r["method"] for r in res["trace"]] == ["drywet", "drywet", "drywet", "brute"]
    kept_procs = sum(int(res["kept"][v]) for v in g.processors())
    assert kept_procs == res["processors_end"]
    assert res["processors_end"] == res["processors_start"] - sum(r["removed"] for r in res["trace"])
    assert np.isfinite(res["La_final"]) and res["La_final"] < 1.5 * res["La_console"] + 0.2
