"""GPU parity of the paths the per-type cases do not reach, through the C-ABI
against the FP64 oracle on the same seeded FP32 inputs:

  * the large-console geometry (48 kHz, 2 s reverb, five loss resolutions up
    to 4096 points, a 2^22-point FFT engine with 4096-point rows) at a size
    the oracle finishes;
  * every node output of a console, not only the mix (waveform relative L2
    <= 1e-4 per node);
  * the full console (16 tracks, 10 s at 44.1 kHz) near its ground truth,
    where the compressor coefficients sit close to 1 and the delay radii are
    0.5-0.95, held to the stated tolerances outright: waveform 1e-4 for the
    mix and every node, 1e-5 relative per loss term, 1e-3 per gradient
    tensor;
  * the torch.autograd wrapper of the forward and backward calls."""
import numpy as np
import pytest
import torch

import synth
from oracle import console as OC
from oracle import train as TR
from paper_2509_15948_amd import mixgraph as MG

from gpu_cases import Case, grad_tolerances, loss_tolerances, rel_l2

pytestmark = pytest.mark.gpu

WAVE_TOL = 1e-4
LOSS_TOL = 1e-5
GRAD_TOL = 1e-3


def _check_losses(gl, ol, tol=None, keys=("La", "Llr", "Lm", "Ls", "Lg", "Lp", "L")):
    for k in keys:
        ref = ol[k]
        bound = LOSS_TOL * abs(ref)
        if tol is not None and k in tol:
            bound = max(bound, tol[k])
        print("loss", k, gl[k], ref, "err", abs(gl[k] - ref), "rel", abs(gl[k] - ref) / max(abs(ref), 1e-300),
              "bound", bound, flush=True)
        assert abs(gl[k] - ref) <= bound or abs(gl[k] - ref) < 1e-9, (k, gl[k], ref, bound)


def _grad_errors(case, gth, gwe, oth, owe):
    out = {}
    procs = case.g.processors()
    for t in sorted({case.g.types[v] for v in procs}):
        vs = [v for v in procs if case.g.types[v] == t]
        out[t] = rel_l2(np.concatenate([gth[v] for v in vs]), np.concatenate([oth[v] for v in vs]))
    out["w"] = rel_l2([gwe[v] for v in procs], [owe[v] for v in procs])
    return out


def _node_outputs(case, mask=None):
    """Every non-input node's output from the GPU (mg_node_output)."""
    st = torch.cuda.current_stream().cuda_stream
    out = {}
    buf = torch.empty(2, case.cfg.length, dtype=torch.float32, device="cuda")
    for v, t in enumerate(case.g.types):
        if t == "i":
            continue
        MG.mg_node_output(case.bg.h, v, buf, st)
        torch.cuda.synchronize()
        out[v] = buf.cpu().numpy().astype(np.float64)
    return out


def _oracle_nodes(case, mask=None):
    with torch.no_grad():
        th = {v: torch.tensor(np.asarray(p, dtype=np.float64)) for v, p in case.th.items()}
        we = {v: torch.tensor(float(w), dtype=torch.float64) for v, w in case.we.items()}
        ev = OC.evaluate(case.g, case.cfg, case.dry, case.noise, th, we, mask, keep_nodes=True)
    return {v: y.numpy() for v, y in ev["y"].items()}


@pytest.mark.timeout(1200)
def test_large_console_geometry_against_the_oracle():
    """One delay + reverb chain per level, 45 s at 48 kHz, 2 s (96 000-tap)
    reverb, 0.5 s delay range, loss at 256/512/1024/2048/4096 points: the FFT
    engine is 3 x 2^20 points (3072-point rows, each three 1024-point
    transforms and a radix-3 pass, and 1024-point columns in 8-column tiles),
    as in the large console.  Waveform, losses and the delay, reverb
    and dry/wet gradients against the oracle."""
    cfg = synth.small_config(seconds=45.0, fs=48000, n_tracks=1, n_subgroups=1, chain="dr", reverb_seconds=2.0,
                             delay_range_s=0.5, loss_ffts=(256, 512, 1024, 2048, 4096))
    case = Case(cfg, alpha_p=1e-2)
    assert case.bg.info.fft_size == 3 << 20       # 3072-point rows x 1024-point columns
    assert cfg.reverb_length == 96000
    mix, gl = case.gpu_forward()
    gth, gwe = case.gpu_backward()
    omix, ol, oth, owe = case.oracle()
    err = rel_l2(mix, omix)
    print("large geometry wave", err, flush=True)
    assert err <= WAVE_TOL
    _check_losses(gl, ol, loss_tolerances(case, omix))
    tol, sens = grad_tolerances(case, oth, owe)
    for t, e in _grad_errors(case, gth, gwe, oth, owe).items():
        print("large geometry", t, "grad err", e, "oracle FP32 sensitivity", sens[t], "bound", tol[t], flush=True)
        assert e <= tol[t], (t, e, tol[t])


@pytest.mark.timeout(600)
def test_full_chain_at_48k_with_five_loss_resolutions():
    """Every processor type at 48 kHz with the large console's five loss
    resolutions (256 ... 4096 points), forward and backward."""
    cfg = synth.small_config(seconds=0.75, fs=48000, n_tracks=3, n_subgroups=2, chain="ecxsgdr",
                             loss_ffts=(256, 512, 1024, 2048, 4096))
    case = Case(cfg, alpha_p=1e-2)
    mix, gl = case.gpu_forward()
    gth, gwe = case.gpu_backward()
    omix, ol, oth, owe = case.oracle()
    err = rel_l2(mix, omix)
    print("48k wave", err, flush=True)
    assert err <= WAVE_TOL
    _check_losses(gl, ol, loss_tolerances(case, omix))
    tol, sens = grad_tolerances(case, oth, owe)
    for t, e in _grad_errors(case, gth, gwe, oth, owe).items():
        print("48k", t, "grad err", e, "oracle FP32 sensitivity", sens[t], "bound", tol[t], flush=True)
        assert e <= tol[t], (t, e, tol[t])


@pytest.mark.parametrize("masked", [False, True])
def test_every_node_output_of_a_console(masked):
    """Each node's output, not only the mix, against the oracle's (every
    processor type, both console levels; with a mask that bypasses a third
    of the processors, whose outputs then equal their inputs)."""
    case = Case(synth.small_config(seconds=0.75, fs=16000, n_tracks=3, n_subgroups=2, chain="ecxsgdr"))
    mask = None
    if masked:
        procs = case.g.processors()
        mask = {v: (0.0 if i % 3 == 0 else 1.0) for i, v in enumerate(procs)}
    case.gpu_forward(mask)
    got = _node_outputs(case)
    ref = _oracle_nodes(case, mask)
    worst = 0.0
    for v, y in got.items():
        e = rel_l2(y, ref[v])
        worst = max(worst, e)
        print("node", v, case.g.types[v], "wave", e, flush=True)
        assert e <= WAVE_TOL, (v, case.g.types[v], e)
    print("worst node", worst, flush=True)


@pytest.mark.timeout(1800)
def test_full_console_near_ground_truth_stated_tolerances():
    """16 stereo tracks, 4 subgroups, 10 s at 44.1 kHz, every processor type,
    at ground truth + N(0, 0.3^2): compressor coefficients near 1 (time
    constants 5-100 ms, so 108 chunk carries per node chain an envelope with
    alpha -> 1), delay radii 0.5-0.95.  Held to the stated tolerances with no
    noise-derived widening: mix and every node output 1e-4, every loss term
    1e-5 relative, every gradient tensor 1e-3."""
    cfg = synth.CONFIGS["full"]
    case = Case(cfg, seed=1, params="random")
    alphas = [1.0 / (1.0 + np.exp(-case.th[v][0])) for v in case.g.processors() if case.g.types[v] == "c"]
    print("compressor alpha range", min(alphas), max(alphas), flush=True)
    assert min(alphas) > 0.99
    mix, gl = case.gpu_forward()
    nodes = _node_outputs(case)
    gth, gwe = case.gpu_backward()
    omix, ol, oth, owe = case.oracle()
    err = rel_l2(mix, omix)
    print("near-GT full wave", err, flush=True)
    assert err <= WAVE_TOL
    _check_losses(gl, ol)
    errs = _grad_errors(case, gth, gwe, oth, owe)
    for t, e in errs.items():
        print("near-GT full", t, "grad err", e, flush=True)
    del omix, oth
    ref = _oracle_nodes(case)
    worst = {}
    for v, y in nodes.items():
        e = rel_l2(y, ref[v])
        t = case.g.types[v]
        worst[t] = max(worst.get(t, 0.0), e)
    print("near-GT full worst node error by type", worst, flush=True)
    for t, e in errs.items():
        assert e <= GRAD_TOL, (t, e)
    for t, e in worst.items():
        assert e <= WAVE_TOL, (t, e)


def test_console_loss_autograd_wrapper():
    """console_loss (torch.autograd.Function over mg_forward / mg_backward):
    the gradient that reaches theta and the dry/wet logits is mg_backward's,
    bit for bit, scaled by the incoming gradient of L; the loss vector carries
    no gradient; a backward after another forward on the session raises."""
    case = Case(synth.small_config(seconds=0.75, fs=16000, n_tracks=3, n_subgroups=2, chain="ecxsgdr"),
                alpha_p=1e-2)
    th = case.theta_d.clone().requires_grad_(True)
    we = case.wet_d.clone().requires_grad_(True)
    L, losses = MG.console_loss(case.sess, case.dry_d, th, we)
    assert not losses.requires_grad
    (2.5 * L).backward()
    torch.cuda.synchronize()
    _, gl = case.gpu_forward()
    gth_ref = torch.empty(case.bg.n_theta, dtype=torch.float32, device="cuda")
    gwe_ref = torch.empty(case.bg.n_proc, dtype=torch.float32, device="cuda")
    case.sess.backward(gth_ref, gwe_ref)
    torch.cuda.synchronize()
    assert float(L) == gl["L"]
    assert torch.equal(th.grad, gth_ref * 2.5)
    assert torch.equal(we.grad, gwe_ref * 2.5)
    # the same gradient against the oracle
    gth, gwe = case.bg.unflatten((th.grad / 2.5).cpu().numpy(), (we.grad / 2.5).cpu().numpy(), case.sizes)
    omix, ol, oth, owe = case.oracle()
    tol, _ = grad_tolerances(case, oth, owe)
    for t, e in _grad_errors(case, gth, gwe, oth, owe).items():
        print("autograd", t, "grad err", e, "bound", tol[t], flush=True)
        assert e <= tol[t]
    # a stale backward raises instead of returning another forward's gradient
    th2 = case.theta_d.clone().requires_grad_(True)
    L1, _ = MG.console_loss(case.sess, case.dry_d, th2, case.wet_d)
    L2, _ = MG.console_loss(case.sess, case.dry_d, th2, case.wet_d)
    with pytest.raises(MG.MixgraphError):
        L1.backward()
    L2.backward()
    assert torch.equal(th2.grad, gth_ref)
