#!/usr/bin/env python3
"""Benchmark of the batched mixing-console step on one MI355X.

A step is one pass of the hot path on one synthetic song: the batched
forward pass of the full console (every stage one launch per processor
type), the fused MRSTFT loss against the resident target, the backward pass
through every processor's adjoint, and Adam on all parameters.  The default
workload is the full console: 16 stereo tracks, 4 subgroups, 10 s at
44.1 kHz, chain e c x s g d r on every track and subgroup.

Prints one JSON line.  Besides the headline (audio-seconds per second) it
reports the dominant kernel class's achieved bandwidth against the HBM peak
(timed live with HIP events over the timed region), the whole step against
the algorithmic byte model, the plain per-processor PyTorch loop on the same
GPU, the masked pruning evaluation (64 candidates), and the FP64 CPU oracle on
a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_CLASSES = ("conv_cols", "conv_rows", "conv_icols", "eq_conv", "eq_spec", "dyn", "pointwise", "sum", "loss",
                  "reverb_fir", "fir")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# ---------------------------------------------------------------- byte model
def model_bytes_per_step(g, cfg):
    """Algorithmic HBM bytes of one fwd+bwd step: every processor reads its
    input and writes its output once forward (16 B per stereo sample) and
    reads dL/dy, u, y and writes dL/du backward (32 B); a mix node reads each
    child and writes once; the loss reads the mix (and writes dL/dy) plus the
    resident target Mel features (4 combos x 96 bands x 4 B per hop)."""
    L = cfg.length
    n_proc = len(g.processors())
    preds = {}
    for s, d in g.edges:
        preds.setdefault(d, []).append(s)
    mix = sum(8 * len(preds[v]) + 8 for v, t in enumerate(g.types) if t in "mo")
    F = sum(4 * cfg.n_mels * 4 / (n // 4) for n in cfg.loss_ffts)
    return (n_proc * 48 + mix + (8 + F) + (16 + F)) * L


# ---------------------------------------------------------------- plain loop
def plain_loop_step(torch, g, cfg, dry, noise, target, th, we):
    """The reference loop that batched processing replaces: PyTorch eager ops,
    one node at a time in topological order, torch.fft convolutions, truncated
    IIR envelope (as a convolution), torch STFT loss, autograd backward."""
    import torch.nn.functional as Fn
    dev = dry.device
    L = cfg.length
    fs = cfg.fs

    def conv(x, h, lag0):
        n = 1 << (L + h.shape[-1] - 1).bit_length()
        c = torch.fft.irfft(torch.fft.rfft(x, n=n) * torch.fft.rfft(h, n=n), n=n)
        return c[..., -lag0:-lag0 + L] if lag0 <= 0 else Fn.pad(c[..., :L - lag0], (lag0, 0))

    def zp_fir(p, N):
        K = (N + 1) // 2
        n = torch.arange(-(N - 1) // 2, (N - 1) // 2 + 1, device=dev, dtype=torch.float32)
        k = torch.arange(1, K, device=dev, dtype=torch.float32)
        H = torch.exp(p)
        h0 = (H[0] + 2 * (H[1:, None] * torch.cos(2 * math.pi * k[:, None] * n[None, :] / N)).sum(0)) / N
        return torch.cos(math.pi * n / N) ** 2 * h0

    preds = {}
    for s, d in g.edges:
        preds.setdefault(d, []).append(s)
    y = {}
    # consoles list their nodes in a topological order already
    for v in range(g.n_nodes):
        t = g.types[v]
        if t == "i":
            src = dry[g.track_of_input[v]]
            y[v] = src.expand(2, L) if src.shape[0] == 1 else src
            continue
        u = sum(y[s] for s in preds[v])
        if t in "mo":
            y[v] = u
            continue
        p = th[v]
        if t == "g":
            yb = torch.exp(p)[:, None] * u
        elif t == "s":
            ym, ys = u[0] + u[1], torch.exp(p[0]) * (u[0] - u[1])
            yb = torch.stack([(ym + ys) / 2, (ym - ys) / 2])
        elif t == "x":
            yb = torch.exp(p[1]) * torch.tanh(torch.exp(p[0]) * u)
        elif t == "e":
            yb = conv(u, zp_fir(p, cfg.eq_taps)[None], -(cfg.eq_taps - 1) // 2)
        elif t == "c":
            a = torch.sigmoid(p[0])
            e = (u[0] + u[1]) ** 2
            ntr = int(min(L, max(16, math.ceil(math.log(1e-7) / math.log(max(float(a), 1e-6))))))
            hk = (1 - a) * a ** torch.arange(ntr, device=dev, dtype=torch.float32)
            genv = conv(e[None], hk[None], 0)[0].clamp_min(0)
            G = torch.log(genv + 1e-8)
            T, W, R = p[1], torch.exp(p[2]), 1 + torch.exp(p[3])
            Gy = torch.where(G >= T + W, T + (G - T) / R,
                             torch.where(G >= T - W, G + (1 / R - 1) * (G - T + W) ** 2 / (4 * W), G))
            yb = torch.exp(Gy - G)[None] * u
        elif t == "d":
            M, D, taps = cfg.delay_taps, cfg.delay_range, cfg.delay_fir_taps
            Kc = (taps + 1) // 2
            pv = p.view(2, M, 2 + Kc)
            Lh = M * D + taps - 1
            k = torch.arange(D, device=dev, dtype=torch.float32)
            hs = []
            for c in range(2):
                hc = torch.zeros(Lh, device=dev)
                for m in range(M):
                    cm = zp_fir(pv[c, m, 2:], taps)
                    phi = float(torch.atan2(pv[c, m, 1], pv[c, m, 0]))
                    d = m * D + int(math.floor(-phi * D / (2 * math.pi) + 0.5)) % D
                    z = torch.complex(pv[c, m, 0], pv[c, m, 1])
                    sur = torch.fft.ifft(torch.exp(k * torch.log(z))).real
                    seg = Fn.conv1d(sur.view(1, 1, -1), cm.detach().flip(0).view(1, 1, -1), padding=taps - 1).view(-1)
                    hc = hc + Fn.pad(cm, (d, Lh - d - taps))
                    hc = hc + Fn.pad(seg - seg.detach(), (m * D, Lh - m * D - (D + taps - 1)))
                hs.append(hc)
            yb = conv(u, torch.stack(hs), -(taps - 1) // 2)
        elif t == "r":
            nzv = noise[v]
            Lr = nzv.shape[-1]
            win = torch.hann_window(384, periodic=True, device=dev)
            nf = (Lr - 1) // 192 + 2
            pad = Fn.pad(nzv, (192, 192 + 384))
            fr = pad.unfold(-1, 384, 192)[:, :nf] * win
            U = torch.fft.rfft(fr)
            pv = p.view(2, 2, 192)
            mm = torch.arange(nf, device=dev, dtype=torch.float32)[:, None]
            beta = math.log(math.expm1(6.91 * 192 / (0.5 * fs)))
            g0 = -0.5 * math.log(0.5 * fs / (6 * 6.91))
            hs = []
            for x in range(2):
                mask = torch.exp(pv[x, 0] + g0 + mm * (-Fn.softplus(pv[x, 1] + beta)))
                Hm = torch.cat([U[x, :, :192] * mask, torch.zeros(nf, 1, device=dev, dtype=U.dtype)], 1)
                s = torch.fft.irfft(Hm, n=384) * win
                ola = Fn.fold(s.T[None], (1, (nf + 1) * 192), (1, 384), stride=(1, 192))[0, 0, 0]
                wsum = Fn.fold((win ** 2).repeat(nf, 1).T[None], (1, (nf + 1) * 192), (1, 384), stride=(1, 192))[0, 0, 0]
                hs.append((ola / wsum.clamp_min(1e-12))[192:192 + Lr])
            yb = conv(u, torch.stack([hs[0] + hs[1], hs[0] - hs[1]]), 0)
        w = torch.sigmoid(we[v])
        y[v] = w * yb + (1 - w) * u
    mix = y[g.n_nodes - 1]
    La = 0.0
    for n_fft in cfg.loss_ffts:
        hop = n_fft // 4
        win = torch.hann_window(n_fft, periodic=True, device=dev)

        def mel(x):
            X = torch.stft(x, n_fft, hop, window=win, center=False, return_complex=True)
            return {"l": X[0], "r": X[1], "m": X[0] + X[1], "s": X[0] - X[1]}
        A, B = mel(mix), mel(target)
        for k in "lrms":
            a, b = A[k].abs(), B[k].abs()
            La = La + 0.25 * (torch.mean(torch.abs(torch.log(a + 1e-7) - torch.log(b + 1e-7)))
                              + torch.linalg.norm(a - b) / torch.linalg.norm(b))
    La.backward()
    return float(La)


def time_plain_loop(torch, g, cfg, dry_d, noise, target_d, th, we, steps=2):
    dev = dry_d.device
    thd = {v: torch.tensor(np.asarray(p, np.float32), device=dev, requires_grad=True) for v, p in th.items()}
    wed = {v: torch.tensor(float(w), device=dev, requires_grad=True) for v, w in we.items()}
    nzd = {v: torch.tensor(n, device=dev) for v, n in noise.items()}
    plain_loop_step(torch, g, cfg, dry_d, nzd, target_d, thd, wed)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for t in list(thd.values()) + list(wed.values()):
            t.grad = None
        plain_loop_step(torch, g, cfg, dry_d, nzd, target_d, thd, wed)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


# ---------------------------------------------------------------- CPU oracle
def cpu_baseline(cfg_name, budget_s=20.0):
    """The FP64 oracle as it stands, timed on the host: fwd+bwd steps of the
    same workload until about budget_s seconds of work."""
    import torch
    import synth
    from oracle import train as TR
    cfg = synth.CONFIGS[cfg_name]
    g, dry, noise = synth.song(1, cfg)
    gt, gw = synth.ground_truth_params(101, g, cfg)
    target = TR.render(g, cfg, dry, noise, gt, gw)
    th, we = synth.init_params(1, g, cfg)
    n = 0
    t0 = time.perf_counter()
    while True:
        TR.loss_and_grad(g, cfg, dry, noise, target, th, we)
        n += 1
        if time.perf_counter() - t0 > budget_s or n >= 4:
            break
    dt = (time.perf_counter() - t0) / n
    return {"value": round(cfg.seconds / dt, 4), "unit": "audio-s/s", "cores": torch.get_num_threads(),
            "kind": "oracle",
            "sample": f"{n} fwd+bwd step(s) of the same {cfg.n_tracks}-track {cfg.seconds:g} s console, FP64, "
                      f"{dt:.2f} s per step on {os.cpu_count()} host cores"}


# ---------------------------------------------------------------- traffic
def committed_traffic(kernel_class, workload):
    """HBM bytes per launch from the committed rocprofv3 PMC summary of this
    kernel class and workload, if it was taken on the current kernel sources;
    else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel_class}_{workload}_console_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
        h = hashlib.sha256()
        for f in rec["sources"]:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        if h.hexdigest() != rec["sources_sha256"]:
            return None
        return rec["bytes_per_launch"]
    except Exception:
        return None


def serving_leg(args):
    """Whole-song searches arriving as a Poisson stream, served with
    continuous batching (serve.Server): p50/p99 latency and throughput."""
    import synth
    from paper_2509_15948_amd import serve as SV
    reqs = synth.serving_requests(3, args.serve_requests, rate=args.serve_rate, tracks=(4, 16), subgroups=(2, 4),
                                  seconds=(2.0, 6.0), fs=44100)
    spec = SV.SearchSpec(steps=args.serve_steps, rounds=2, finetune=5, tau=1e-3, candidates=16, quantum=4)
    server = SV.Server(budget_bytes=int(args.serve_budget_gb * (1 << 30)), max_active=4)
    out = server.run(reqs, lambda i, cfg, seed: SV.Search(i, cfg, seed, spec))
    removed = [sum(r["removed"] for r in res["trace"]) for res in out["results"]]
    final = [res["processors"] for res in out["results"]]
    return {"requests": len(reqs), "rate_per_s": args.serve_rate,
            "workload": f"tracks U{{4..16}}, subgroups U{{2..4}}, 2-6 s at 44.1 kHz, chain ecxsgdr; search = "
                        f"{spec.steps} steps + {spec.rounds} pruning rounds x ({spec.candidates} trials + "
                        f"{spec.finetune} fine-tune steps)",
            "p50_latency_s": round(out["p50_s"], 4), "p99_latency_s": round(out["p99_s"], 4),
            "songs_per_s": round(out["songs_per_s"], 3), "audio_s_per_s": round(out["audio_s_per_s"], 1),
            "makespan_s": round(out["makespan_s"], 3), "peak_active": out["peak_active"],
            "peak_gb": round(out["peak_bytes"] / (1 << 30), 3), "processors_removed": removed,
            "processors_left": final}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="full", choices=["full", "tiny", "large"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain-loop", action="store_true")
    ap.add_argument("--prune-masks", type=int, default=64)
    ap.add_argument("--serve-requests", type=int, default=12,
                    help="requests of the serving leg (0 skips it)")
    ap.add_argument("--serve-rate", type=float, default=20.0, help="Poisson arrival rate, requests/s")
    ap.add_argument("--serve-steps", type=int, default=20, help="optimisation steps per search")
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    ap.add_argument("--pmc-run", action="store_true",
                    help="for rocprofv3 counter runs: a calibration copy, then --steps steps, nothing else")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the console of one song lives on one device "
              "(multi-GPU sharding is a design note, not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_2509_15948_amd import mixgraph as MG
    from paper_2509_15948_amd import workloads as W

    cfg = synth.CONFIGS[args.config]
    dev = "cuda"
    g, dry, noise = synth.song(1, cfg)
    bg = W.binding_graph(g, cfg, max_trials=max(0, args.prune_masks))
    dry_d = torch.from_numpy(dry).to(dev)
    noise_d = torch.from_numpy(W.noise_rows(bg, noise, cfg.reverb_length)).to(dev)
    log(f"workload {args.config}: {g.n_nodes} nodes, {bg.n_proc} processors, schedule {bg.schedule}, "
        f"FFT {bg.info.fft_size}, theta {bg.n_theta}")

    # target mix: the same console with ground-truth parameters, rendered on the GPU
    gt, gw = synth.ground_truth_params(101, g, cfg)
    th_gt, we_gt = bg.flatten(gt, gw)
    tmp = MG.Session(bg, noise_d, torch.zeros(2, cfg.length, device=dev), mode=0)
    target_d = torch.empty(2, cfg.length, device=dev)
    tmp.forward(dry_d, torch.from_numpy(th_gt).to(dev), torch.from_numpy(we_gt).to(dev), None, target_d)
    torch.cuda.synchronize()
    del tmp

    sess = MG.Session(bg, noise_d, target_d, mode=1)
    th0, we0 = synth.init_params(1, g, cfg)
    th_f, we_f = bg.flatten(th0, we0)
    theta = torch.from_numpy(th_f).to(dev)
    wet = torch.from_numpy(we_f).to(dev)
    gth = torch.empty_like(theta)
    gwe = torch.empty_like(wet)
    m_t, v_t = torch.zeros_like(theta), torch.zeros_like(theta)
    m_w, v_w = torch.zeros_like(wet), torch.zeros_like(wet)
    losses = torch.zeros(7, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream().cuda_stream
    step_no = [0]

    def step():
        step_no[0] += 1
        sess.forward(dry_d, theta, wet, None, None, losses)
        sess.backward(gth, gwe)
        MG.mg_adam_step(theta, m_t, v_t, gth, bg.n_theta, cfg.lr, 0.9, 0.999, 1e-8, step_no[0], stream)
        MG.mg_adam_step(wet, m_w, v_w, gwe, bg.n_proc, cfg.lr, 0.9, 0.999, 1e-8, step_no[0], stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"warm-up done, loss {losses.cpu().numpy()[1]:.4f}")

    if args.pmc_run:
        from paper_2509_15948_amd.profiling import CALIB_BYTES
        src = torch.ones(CALIB_BYTES // 4, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)          # calibration: CALIB_BYTES read and written once
        torch.cuda.synchronize()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        log(f"pmc run: calibration copy of {CALIB_BYTES} bytes, then {args.steps} steps")
        return

    # one profiled step per kernel class to find the dominant one
    per_class = {}
    for cls in KERNEL_CLASSES:
        MG.mg_profile_enable(bg.h, cls)
        step()
        ms, n, b = MG.mg_profile_read(bg.h)
        per_class[cls] = (ms, n, b)
    MG.mg_profile_enable(bg.h, None)
    dominant = max(per_class, key=lambda k: per_class[k][0])
    log("per step by kernel class (ms): " + ", ".join(f"{k} {v[0]:.3f}" for k, v in per_class.items()))

    # timed region
    MG.mg_profile_enable(bg.h, dominant)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(args.steps):
        step()
    t1.record()
    torch.cuda.synchronize()
    total_ms = t0.elapsed_time(t1)
    k_ms, k_n, k_bytes = MG.mg_profile_read(bg.h)
    MG.mg_profile_enable(bg.h, None)
    ms_step = total_ms / args.steps
    value = cfg.seconds * args.steps / (total_ms / 1000.0)
    log(f"timed {args.steps} steps: {ms_step:.3f} ms/step, {value:.1f} audio-s/s, loss {losses.cpu().numpy()[1]:.4f}")

    achieved = (k_bytes / k_n) / ((k_ms / k_n) / 1000.0) / 1e9 if k_n else 0.0
    roofline = {"bound": "hbm", "kernel": dominant, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": committed_traffic(dominant, args.config),
                "launches": k_n, "avg_launch_us": round(1000.0 * k_ms / max(k_n, 1), 2),
                "alg_bytes_per_launch": round(k_bytes / max(k_n, 1))}
    mb = model_bytes_per_step(g, cfg)
    hbm_model = {"bytes_per_step": int(mb), "achieved_GBs": round(mb / (ms_step / 1000.0) / 1e9, 1),
                 "frac_of_peak": round(mb / (ms_step / 1000.0) / 1e9 / HBM_PEAK_GBS, 4)}

    # pruning evaluation: B single-processor trials (the B lowest dry/wet
    # weights) by suffix recomputation after one forward at the current
    # parameters, and the same masks as complete forwards for comparison
    prune = None
    if args.prune_masks > 0:
        B = min(args.prune_masks, bg.n_proc)
        cand = MG.mg_prune_candidates(wet.cpu().numpy(), None, np.ones(bg.n_proc, np.uint8), B)
        keep = np.ones((B, bg.n_proc), np.uint8)
        keep[np.arange(B), cand] = 0
        out = torch.zeros(B, 7, dtype=torch.float64, device=dev)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e2 = torch.cuda.Event(enable_timing=True)
        for rep in range(2):  # the first pass warms up
            e0.record()
            sess.forward(dry_d, theta, wet, None, None, losses)
            e1.record()
            sess.forward_trials(keep, out)
            e2.record()
            torch.cuda.synchronize()
        fwd_ms, trial_ms = e0.elapsed_time(e1), e1.elapsed_time(e2)
        masks = torch.from_numpy(keep.astype(np.float32)).to(dev)
        ref = torch.zeros(B, 7, dtype=torch.float64, device=dev)
        e0.record()
        sess.forward_masked(dry_d, theta, wet, masks, ref)
        e1.record()
        torch.cuda.synchronize()
        full_ms = e0.elapsed_time(e1)
        prune = {"candidates": B, "forward_ms": round(fwd_ms, 3), "trials_ms": round(trial_ms, 3),
                 "candidates_per_s": round(B / ((fwd_ms + trial_ms) / 1000.0), 1),
                 "complete_forwards_ms": round(full_ms, 3),
                 "speedup_vs_complete_forwards": round(full_ms / (fwd_ms + trial_ms), 2),
                 "bitwise_equal_to_complete_forwards": bool(torch.equal(out, ref))}

    plain = None
    if not args.no_plain_loop:
        try:
            th_np, we_np = bg.unflatten(theta.cpu().numpy(), wet.cpu().numpy(),
                                        {v: len(p) for v, p in th0.items()})
            dt = time_plain_loop(torch, g, cfg, dry_d, noise, target_d, th_np, we_np)
            plain = {"ms_per_step": round(1000 * dt, 2), "audio_s_per_s": round(cfg.seconds / dt, 2),
                     "speedup": round((1000 * dt) / ms_step, 2),
                     "what": "PyTorch eager, one node at a time, torch.fft convolutions, truncated-IIR "
                             "envelope, torch.stft loss, autograd backward"}
        except Exception as e:  # the baseline must not break the headline
            plain = {"error": repr(e)[:200]}

    serving = None
    if args.serve_requests > 0:
        try:
            serving = serving_leg(args)
        except Exception as e:  # the serving leg must not break the headline
            serving = {"error": repr(e)[:300]}

    cpu = None
    if not args.no_cpu_baseline:
        try:
            cpu = cpu_baseline(args.config)
        except Exception as e:
            cpu = {"error": repr(e)[:200]}

    rec = {
        "metric": "console fwd+bwd audio-sec/s",
        "value": round(value, 2),
        "unit": "audio-s/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{cfg.name} console: {cfg.n_tracks} stereo tracks, {cfg.n_subgroups} subgroups, "
                               f"{cfg.seconds:g} s at {cfg.fs} Hz, chain {cfg.chain} per track and subgroup; "
                               "step = forward + MRSTFT loss + backward + Adam",
                   "tracks": cfg.n_tracks, "subgroups": cfg.n_subgroups, "seconds": cfg.seconds,
                   "sample_rate": cfg.fs, "processors": bg.n_proc, "schedule": bg.schedule,
                   "fft_size": bg.info.fft_size, "parallelism": "single GPU"},
        "roofline": roofline,
        "hbm_model": hbm_model,
        "kernel_classes": {k: {"ms_per_step": round(v[0], 4), "launches": v[1],
                               "alg_bytes_per_launch": round(v[2] / max(v[1], 1)),
                               "alg_GBs": round(v[2] / (v[0] / 1000.0) / 1e9, 1) if v[0] > 0 else None,
                               "traffic_bytes_per_launch": committed_traffic(k, args.config)}
                           for k, v in per_class.items()},
        "prune_eval": prune,
        "plain_loop": plain,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
