"""mg_setup_static (the entry point that allocates nothing: the workspace is
the library's static device scratch) against mg_setup with a caller-owned
workspace, through the C-ABI: two bindings in a row, the second graph
smaller than the first, each giving the same mix, losses and gradients bit
for bit; the first graph's calls fail once the second has taken the
scratch over."""
import numpy as np
import pytest
import torch

import synth
from oracle import train as TR
from paper_2509_15948_amd import mixgraph as MG
from paper_2509_15948_amd import workloads as W

pytestmark = pytest.mark.gpu

STATIC_BYTES = 64 << 20


def _song(cfg, seed):
    g, dry, noise = synth.song(seed, cfg)
    gt, gw = synth.ground_truth_params(seed + 100, g, cfg)
    target = TR.render(g, cfg, dry, noise, gt, gw).astype(np.float32)
    th, we = synth.random_params(seed, g, cfg, std=0.3)
    return g, dry, noise, target, th, we


def _run(bg, cfg, dry, noise, target, th, we, static):
    dev = "cuda"
    noise_d = torch.from_numpy(W.noise_rows(bg, noise, cfg.reverb_length)).to(dev)
    target_d = torch.from_numpy(target).to(dev)
    sess = MG.Session(bg, noise_d, target_d, mode=1, static=static)
    th_f, we_f = bg.flatten(th, we)
    theta = torch.from_numpy(th_f).to(dev)
    wet = torch.from_numpy(we_f).to(dev)
    mix = torch.empty(2, cfg.length, device=dev)
    losses = torch.zeros(7, dtype=torch.float64, device=dev)
    dry_d = torch.from_numpy(dry).to(dev)
    sess.forward(dry_d, theta, wet, None, mix, losses)
    gth = torch.empty_like(theta)
    gwe = torch.empty_like(wet)
    sess.backward(gth, gwe)
    torch.cuda.synchronize()
    return sess, (dry_d, theta, wet), mix.cpu(), losses.cpu(), gth.cpu(), gwe.cpu()


def _compare(name, cfg, seed):
    g, dry, noise, target, th, we = _song(cfg, seed)
    ref_graph = W.binding_graph(g, cfg, alpha_p=1e-2)
    st_graph = W.binding_graph(g, cfg, alpha_p=1e-2)
    need = MG.mg_workspace_size(st_graph.h, 1)
    assert need <= STATIC_BYTES
    _, _, mix_r, los_r, gth_r, gwe_r = _run(ref_graph, cfg, dry, noise, target, th, we, static=False)
    sess, args, mix_s, los_s, gth_s, gwe_s = _run(st_graph, cfg, dry, noise, target, th, we, static=True)
    print(name, "workspace", need, "bytes; L_a", float(los_s[1]), "vs", float(los_r[1]),
          "max |mix diff|", float((mix_s - mix_r).abs().max()), flush=True)
    assert torch.equal(mix_s, mix_r)
    assert torch.equal(los_s, los_r)
    assert torch.equal(gth_s, gth_r)
    assert torch.equal(gwe_s, gwe_r)
    return sess, args


def test_static_scratch_equals_caller_workspace_twice_second_smaller():
    # first: the tiny console at full size (4 mono tracks, 2 s at 44.1 kHz,
    # EQ 1023 taps, attack/release compressor), about 41 MiB of workspace
    s1, a1 = _compare("tiny", synth.CONFIGS["tiny"], 11)
    # second, smaller: every processor type, 3 tracks, 0.75 s at 16 kHz
    small = synth.small_config(seconds=0.75, fs=16000, n_tracks=3, n_subgroups=2, chain="ecxsgdr")
    s2, _ = _compare("small", small, 12)
    # the first graph's binding is stale now
    losses = torch.zeros(7, dtype=torch.float64, device="cuda")
    with pytest.raises(MG.MixgraphError):
        s1.forward(a1[0], a1[1], a1[2], None, None, losses)
    torch.cuda.synchronize()
