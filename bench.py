#!/usr/bin/env python3
"""Benchmark of the batched mixing-console step on one MI355X.

A step is one pass of the hot path on one synthetic song: the batched
forward pass of the console (every stage one launch per processor type), the
fused MRSTFT loss against the resident target, the backward pass through
every processor's adjoint, and Adam on all parameters.  The headline
workload is the large console: 64 stereo tracks, 8 subgroups, 60 s at
48 kHz, chain e c x s g d r on every track and subgroup, 2 s reverb, loss at
five resolutions (256 ... 4096 points).

Prints one JSON line.  Besides the headline (audio-seconds per second) it
reports the dominant kernel class against the HBM peak under the paper's
byte model (each processor reads its input and writes its output once
forward, reads dL/dy, u, y and writes dL/du backward; timed live with HIP
events over the timed region), a device copy measured in the same run, the
full console (16 tracks, 10 s at 44.1 kHz) with the plain per-processor
PyTorch loop beside it, the masked pruning evaluation (64 candidates), the
pruning schedule of the optimised full console (up to 30 rounds of 64
candidates and 50 fine-tune steps), a short serving stream, and the FP64 CPU
oracle on a bounded sample.
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
def _mix_children(g):
    preds = {}
    for s, d in g.edges:
        preds.setdefault(d, []).append(s)
    return [len(preds[v]) for v, t in enumerate(g.types) if t in "mo"]


def _mel_bytes_per_sample(cfg):
    """Resident target Mel features read per sample and loss pass: 4 combos
    (l, r, m, s) x n_mels bands x 4 B per frame, one frame per hop."""
    return sum(4 * cfg.n_mels * 4 / (n // 4) for n in cfg.loss_ffts)


def model_bytes_per_step(g, cfg):
    """Algorithmic HBM bytes of one fwd+bwd step under the paper's byte model:
    every processor reads its input and writes its output once forward (16 B
    per stereo sample) and reads dL/dy, u, y and writes dL/du backward (32 B);
    a mix node reads each child and writes once (its backward is an alias);
    the loss reads the mix (and writes dL/dy) plus the resident target Mel
    features."""
    return model_total(g, cfg)


def class_model_bytes(g, cfg):
    """The byte model split by the kernel class that serves each term: per
    step, the bytes of the processor stages (and mix nodes, loss) whose work
    runs in that class.  The three FFT-engine classes serve the same delay and
    reverb stages, so each is charged all of their bytes; FIR synthesis
    (eq_spec, fir, reverb_fir) moves parameters only and has no term."""
    L = cfg.length
    n = {t: sum(1 for x in g.types if x == t) for t in "ecnxsgdr"}
    F = _mel_bytes_per_sample(cfg)
    conv = 48 * L * (n["d"] + n["r"])
    return {"conv_cols": conv, "conv_rows": conv, "conv_icols": conv, "eq_conv": 48 * L * n["e"],
            "eq_spec": 0, "dyn": 48 * L * (n["c"] + n["n"]), "pointwise": 48 * L * (n["x"] + n["s"] + n["g"]),
            "sum": sum(8 * k + 8 for k in _mix_children(g)) * L, "loss": (8 + F + 16 + F) * L,
            "reverb_fir": 0, "fir": 0}


def model_total(g, cfg):
    d = class_model_bytes(g, cfg)
    # the engine classes share one term; count it once
    return sum(v for k, v in d.items() if k not in ("conv_rows", "conv_icols"))


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
def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg_name, excerpt_s=None, budget_s=20.0):
    """The FP64 oracle as it stands, timed on the host: fwd+bwd steps of the
    same console (on its first excerpt_s seconds when given) until about
    budget_s seconds of work."""
    import dataclasses
    import torch
    import synth
    from oracle import train as TR
    cfg = synth.CONFIGS[cfg_name]
    if excerpt_s is not None and excerpt_s < cfg.seconds:
        cfg = dataclasses.replace(cfg, seconds=excerpt_s)
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
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"{n} fwd+bwd step(s) of the {cfg_name} console ({cfg.n_tracks} tracks, {cfg.n_subgroups} "
                      f"subgroups, {cfg.fs} Hz) on its first {cfg.seconds:g} s, FP64, {dt:.2f} s per step, "
                      f"{torch.get_num_threads()} threads of {os.cpu_count()} host cores"}


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
    """Whole-song searches of the serving configuration's shape (tracks
    U{4..32}, subgroups U{2..8}, 5-30 s at 44.1 kHz; 300 steps, then 10
    rounds of 64 candidates and 50 fine-tune steps) arriving as a Poisson
    stream, served with continuous batching (serve.Server): p50/p99 latency
    and throughput.  A short stream (--serve-requests); the long one is
    `python -m paper_2509_15948_amd.serve`."""
    import synth
    from paper_2509_15948_amd import serve as SV
    reqs = synth.serving_requests(3, args.serve_requests, rate=args.serve_rate, tracks=(4, 32), subgroups=(2, 8),
                                  seconds=(5.0, 30.0), fs=44100)
    spec = SV.SearchSpec(steps=args.serve_steps, rounds=10, finetune=50, tau=1e-3, candidates=64, quantum=8)
    import torch
    # as in the serving entry point: torch's cached blocks stay below 85 % of
    # device memory, so the runtime keeps room for its own allocations
    torch.cuda.set_per_process_memory_fraction(0.85)
    budget = min(int(args.serve_budget_gb * (1 << 30)), int(0.68 * torch.cuda.get_device_properties(0).total_memory))
    server = SV.Server(budget_bytes=budget, max_active=8)
    out = server.run(reqs, lambda i, cfg, seed: SV.Search(i, cfg, seed, spec))
    removed = [sum(r["removed"] for r in res["trace"]) for res in out["results"]]
    final = [res["processors"] for res in out["results"]]
    return {"requests": len(reqs), "rate_per_s": args.serve_rate,
            "workload": f"tracks U{{4..32}}, subgroups U{{2..8}}, 5-30 s at 44.1 kHz, chain ecxsgdr; search = "
                        f"{spec.steps} steps + {spec.rounds} pruning rounds x ({spec.candidates} candidates + "
                        f"{spec.finetune} fine-tune steps)",
            "p50_latency_s": round(out["p50_s"], 4), "p99_latency_s": round(out["p99_s"], 4),
            "songs_per_s": round(out["songs_per_s"], 3), "audio_s_per_s": round(out["audio_s_per_s"], 1),
            "makespan_s": round(out["makespan_s"], 3), "peak_active": out["peak_active"],
            "peak_gb": round(out["peak_bytes"] / (1 << 30), 3), "processors_removed": removed,
            "processors_left": final}


class Console:
    """One workload on the device: song, graph, target (rendered by the
    library from ground-truth parameters), session and optimiser state."""

    def __init__(self, torch, cfg_name, max_trials=0):
        import synth
        from paper_2509_15948_amd import mixgraph as MG
        from paper_2509_15948_amd import workloads as W
        self.torch, self.MG = torch, MG
        self.name = cfg_name
        self.cfg = cfg = synth.CONFIGS[cfg_name]
        dev = "cuda"
        self.g, dry, self.noise = synth.song(1, cfg)
        self.bg = bg = W.binding_graph(self.g, cfg, max_trials=max_trials)
        self.dry_d = torch.from_numpy(dry).to(dev)
        self.noise_d = torch.from_numpy(W.noise_rows(bg, self.noise, cfg.reverb_length)).to(dev)
        log(f"workload {cfg_name}: {self.g.n_nodes} nodes, {bg.n_proc} processors, schedule {bg.schedule}, "
            f"FFT {bg.info.fft_size}, theta {bg.n_theta}, workspace {MG.mg_workspace_size(bg.h, 1) / 2**30:.2f} GiB")
        gt, gw = synth.ground_truth_params(101, self.g, cfg)
        th_gt, we_gt = bg.flatten(gt, gw)
        tmp = MG.Session(bg, self.noise_d, torch.zeros(2, cfg.length, device=dev), mode=0)
        self.target_d = torch.empty(2, cfg.length, device=dev)
        tmp.forward(self.dry_d, torch.from_numpy(th_gt).to(dev), torch.from_numpy(we_gt).to(dev), None,
                    self.target_d)
        torch.cuda.synchronize()
        del tmp
        self.sess = MG.Session(bg, self.noise_d, self.target_d, mode=1)
        self.th0, we0 = synth.init_params(1, self.g, cfg)
        th_f, we_f = bg.flatten(self.th0, we0)
        self.theta = torch.from_numpy(th_f).to(dev)
        self.wet = torch.from_numpy(we_f).to(dev)
        self.gth = torch.empty_like(self.theta)
        self.gwe = torch.empty_like(self.wet)
        self.m_t, self.v_t = torch.zeros_like(self.theta), torch.zeros_like(self.theta)
        self.m_w, self.v_w = torch.zeros_like(self.wet), torch.zeros_like(self.wet)
        self.losses = torch.zeros(7, dtype=torch.float64, device=dev)
        self.stream = torch.cuda.current_stream().cuda_stream
        self.n = 0

    def step(self):
        MG, bg = self.MG, self.bg
        self.n += 1
        self.sess.forward(self.dry_d, self.theta, self.wet, None, None, self.losses)
        self.sess.backward(self.gth, self.gwe)
        MG.mg_adam_step(self.theta, self.m_t, self.v_t, self.gth, bg.n_theta, self.cfg.lr, 0.9, 0.999, 1e-8, self.n,
                        self.stream)
        MG.mg_adam_step(self.wet, self.m_w, self.v_w, self.gwe, bg.n_proc, self.cfg.lr, 0.9, 0.999, 1e-8, self.n,
                        self.stream)

    def release(self):
        for k in ("sess", "dry_d", "noise_d", "target_d", "theta", "wet", "gth", "gwe", "m_t", "v_t", "m_w", "v_w"):
            if hasattr(self, k):
                delattr(self, k)
        self.torch.cuda.empty_cache()


def measure(con, steps, warmup):
    """Warm-up, one profiled step per kernel class, then `steps` timed steps
    with the dominant class timed live by its own dispatch events."""
    torch, MG, bg, cfg = con.torch, con.MG, con.bg, con.cfg
    for _ in range(warmup):
        con.step()
    torch.cuda.synchronize()
    log(f"{con.name}: warm-up done, L_a {con.losses.cpu().numpy()[1]:.4f}")
    per_class = {}
    for cls in KERNEL_CLASSES:
        MG.mg_profile_enable(bg.h, cls)
        con.step()
        ms, n, b = MG.mg_profile_read(bg.h)
        per_class[cls] = (ms, n, b)
    MG.mg_profile_enable(bg.h, None)
    dominant = max(per_class, key=lambda k: per_class[k][0])
    log(f"{con.name} per step by kernel class (ms): " + ", ".join(f"{k} {v[0]:.3f}" for k, v in per_class.items()))
    MG.mg_profile_enable(bg.h, dominant)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(steps):
        con.step()
    t1.record()
    torch.cuda.synchronize()
    total_ms = t0.elapsed_time(t1)
    k_ms, k_n, k_bytes = MG.mg_profile_read(bg.h)
    MG.mg_profile_enable(bg.h, None)
    ms_step = total_ms / steps
    value = cfg.seconds * steps / (total_ms / 1000.0)
    log(f"{con.name}: timed {steps} steps: {ms_step:.3f} ms/step, {value:.1f} audio-s/s, "
        f"L_a {con.losses.cpu().numpy()[1]:.4f}")
    cmb = class_model_bytes(con.g, cfg)
    launches_per_step = max(per_class[dominant][1], 1)
    model_per_launch = cmb[dominant] / launches_per_step
    avg_s = (k_ms / max(k_n, 1)) / 1000.0
    achieved = model_per_launch / avg_s / 1e9 if k_n else 0.0
    engine = ("conv_cols", "conv_rows", "conv_icols")
    engine_ms = sum(per_class[k][0] for k in engine)
    roofline = {"bound": "hbm", "kernel": dominant, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": committed_traffic(dominant, cfg.name),
                "launches": k_n, "avg_launch_us": round(1e6 * avg_s, 2),
                "alg_bytes_per_launch": round(model_per_launch),
                "alg_bytes_rule": "paper byte model: the processor stages this class serves, 16 B fwd + 32 B bwd "
                                  "per stereo sample and node, over its launches in a step",
                "engine_bytes_per_launch": round(k_bytes / max(k_n, 1)),
                "engine_bytes_frac": round((k_bytes / max(k_n, 1)) / avg_s / 1e9 / HBM_PEAK_GBS, 4) if k_n else None}
    mb = model_total(con.g, cfg)
    hbm_model = {"bytes_per_step": int(mb), "achieved_GBs": round(mb / (ms_step / 1000.0) / 1e9, 1),
                 "frac_of_peak": round(mb / (ms_step / 1000.0) / 1e9 / HBM_PEAK_GBS, 4),
                 "fft_engine_frac": round(cmb["conv_rows"] / (engine_ms / 1000.0) / 1e9 / HBM_PEAK_GBS, 4)
                 if engine_ms > 0 else None}
    classes = {k: {"ms_per_step": round(v[0], 4), "launches": v[1],
                   "model_bytes_per_step": int(cmb[k]),
                   "model_frac": round(cmb[k] / (v[0] / 1000.0) / 1e9 / HBM_PEAK_GBS, 4) if v[0] > 0 and cmb[k] else None,
                   "engine_bytes_per_launch": round(v[2] / max(v[1], 1)),
                   "traffic_bytes_per_launch": committed_traffic(k, cfg.name)}
               for k, v in per_class.items()}
    return {"ms_per_step": ms_step, "value": value, "roofline": roofline, "hbm_model": hbm_model,
            "kernel_classes": classes}


def copy_ceiling(torch, nbytes=2 << 30, reps=5):
    """A device-to-device copy of nbytes (read once, written once), the
    achievable streaming rate in this run."""
    src = torch.ones(nbytes // 4, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * nbytes * reps / (e0.elapsed_time(e1) / 1000.0) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return {"GBs": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
            "what": f"torch device copy of {nbytes >> 20} MiB, read + write counted, {reps} reps"}


def prune_eval(con, B):
    """B single-processor trials (the B lowest dry/wet weights) by suffix
    recomputation after one forward at the current parameters, next to the
    same masks as complete forwards."""
    torch, MG, bg = con.torch, con.MG, con.bg
    B = min(B, bg.n_proc)
    cand = MG.mg_prune_candidates(con.wet.cpu().numpy(), None, np.ones(bg.n_proc, np.uint8), B)
    keep = np.ones((B, bg.n_proc), np.uint8)
    keep[np.arange(B), cand] = 0
    out = torch.zeros(B, 7, dtype=torch.float64, device="cuda")
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    for _ in range(2):  # the first pass warms up
        e0.record()
        con.sess.forward(con.dry_d, con.theta, con.wet, None, None, con.losses)
        e1.record()
        con.sess.forward_trials(keep, out)
        e2.record()
        torch.cuda.synchronize()
    fwd_ms, trial_ms = e0.elapsed_time(e1), e1.elapsed_time(e2)
    # one more trial batch per kernel class, each class timed by its own
    # dispatch events (the batch's time by where it goes)
    by_class = {}
    for cls in KERNEL_CLASSES:
        MG.mg_profile_enable(bg.h, cls)
        con.sess.forward_trials(keep, out)
        ms, n, _ = MG.mg_profile_read(bg.h)
        if n:
            by_class[cls] = round(ms, 3)
    MG.mg_profile_enable(bg.h, None)
    torch.cuda.synchronize()
    masks = torch.from_numpy(keep.astype(np.float32)).to("cuda")
    ref = torch.zeros(B, 7, dtype=torch.float64, device="cuda")
    e0.record()
    con.sess.forward_masked(con.dry_d, con.theta, con.wet, masks, ref)
    e1.record()
    torch.cuda.synchronize()
    full_ms = e0.elapsed_time(e1)
    return {"candidates": B, "forward_ms": round(fwd_ms, 3), "trials_ms": round(trial_ms, 3),
            "candidates_per_s": round(B / ((fwd_ms + trial_ms) / 1000.0), 1),
            "complete_forwards_ms": round(full_ms, 3),
            "speedup_vs_complete_forwards": round(full_ms / (fwd_ms + trial_ms), 2),
            "bitwise_equal_to_complete_forwards": bool(torch.equal(out, ref)),
            "trial_ms_by_class": by_class}


def prune_schedule_leg(steps=500, rounds=30, finetune=50, candidates=64, tau=1e-3):
    """The pruning schedule of the full console: `steps` Adam steps, then up
    to `rounds` rounds of (candidate trials, prefix trials, the accept rule,
    graph surgery, `finetune` fine-tune steps), stopping at the first round
    that removes nothing."""
    import torch
    import synth
    from paper_2509_15948_amd import serve as SV
    cfg = synth.CONFIGS["full"]
    spec = SV.SearchSpec(steps=steps, rounds=rounds, finetune=finetune, tau=tau, candidates=candidates,
                         quantum=25, stop_when_none=True)
    s = SV.Search(0, cfg, 1, spec)
    t0 = time.perf_counter()
    res = SV.run_alone(s)
    total = time.perf_counter() - t0
    tr = res["trace"]
    rt = [r["seconds"] for r in tr]
    return {"workload": f"full console after {steps} Adam steps; rounds of {candidates} single-bypass trials, "
                        f"prefix trials, relative tolerance {tau}, graph surgery, {finetune} fine-tune steps",
            "rounds_run": len(tr), "processors_start": 7 * (cfg.n_tracks + cfg.n_subgroups),
            "processors_end": res["processors"], "removed_per_round": [r["removed"] for r in tr],
            "round_s_mean": round(float(np.mean(rt)), 4) if rt else None,
            "round_s": [round(x, 4) for x in rt],
            "trial_ms_mean": round(float(np.mean([r["trial_ms"] for r in tr])), 3) if tr else None,
            "L_a_console": round(float(tr[0]["L_start"]), 6) if tr else None,
            "L_a_final": round(float(res["losses"][1]), 6), "total_s": round(total, 3)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="large", choices=["full", "tiny", "large"],
                    help="headline workload (default: the large console)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain-loop", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="headline only: skip the full-console, pruning, serving and copy legs")
    ap.add_argument("--prune-masks", type=int, default=64)
    ap.add_argument("--prune-rounds", type=int, default=30, help="rounds of the pruning schedule (0 skips it)")
    ap.add_argument("--serve-requests", type=int, default=12,
                    help="requests of the serving leg (0 skips it)")
    ap.add_argument("--serve-rate", type=float, default=0.35, help="Poisson arrival rate, requests/s")
    ap.add_argument("--serve-steps", type=int, default=300, help="optimisation steps per search")
    ap.add_argument("--serve-budget-gb", type=float, default=160.0)
    ap.add_argument("--pmc-run", action="store_true",
                    help="for rocprofv3 counter runs: a calibration copy, then --steps steps, nothing else")
    ap.add_argument("--trials-run", action="store_true",
                    help="for rocprofv3 kernel traces of the pruning trials: on the full console, --steps "
                         "times one forward and a batch of --prune-masks trials, nothing else")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the console of one song lives on one device "
              "(multi-GPU sharding is a design note, not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.trials_run:
        fc = Console(torch, "full", max_trials=args.prune_masks)
        B = min(args.prune_masks, fc.bg.n_proc)
        cand = fc.MG.mg_prune_candidates(fc.wet.cpu().numpy(), None, np.ones(fc.bg.n_proc, np.uint8), B)
        keep = np.ones((B, fc.bg.n_proc), np.uint8)
        keep[np.arange(B), cand] = 0
        out = torch.zeros(B, 7, dtype=torch.float64, device="cuda")
        for _ in range(args.steps):
            fc.sess.forward(fc.dry_d, fc.theta, fc.wet, None, None, fc.losses)
            fc.sess.forward_trials(keep, out)
        torch.cuda.synchronize()
        log(f"trials run: {args.steps} x (one forward + {B} trials) on the full console")
        return
    con = Console(torch, args.config, max_trials=0)
    cfg = con.cfg

    if args.pmc_run:
        from paper_2509_15948_amd.profiling import CALIB_BYTES
        for _ in range(args.warmup):
            con.step()
        src = torch.ones(CALIB_BYTES // 4, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)          # calibration: CALIB_BYTES read and written once
        torch.cuda.synchronize()
        for _ in range(args.steps):
            con.step()
        torch.cuda.synchronize()
        log(f"pmc run: calibration copy of {CALIB_BYTES} bytes, then {args.steps} steps")
        return

    head = measure(con, args.steps, args.warmup)
    n_proc = con.bg.n_proc
    schedule, fft = con.bg.schedule, con.bg.info.fft_size
    con.release()
    del con

    copy = None if args.no_extra else copy_ceiling(torch)

    full = None
    if not args.no_extra and args.config != "full":
        fc = Console(torch, "full", max_trials=max(0, args.prune_masks))
        fm = measure(fc, max(args.steps, 20), args.warmup)
        full = {"ms_per_step": round(fm["ms_per_step"], 4), "audio_s_per_s": round(fm["value"], 2),
                "hbm_model": fm["hbm_model"], "dominant": {k: fm["roofline"][k] for k in
                                                           ("kernel", "achieved", "frac", "avg_launch_us")},
                "kernel_ms_per_step": {k: v["ms_per_step"] for k, v in fm["kernel_classes"].items()}}
        if args.prune_masks > 0:
            full["prune_eval"] = prune_eval(fc, args.prune_masks)
        if not args.no_plain_loop:
            try:
                th_np, we_np = fc.bg.unflatten(fc.theta.cpu().numpy(), fc.wet.cpu().numpy(),
                                               {v: len(p) for v, p in fc.th0.items()})
                dt = time_plain_loop(torch, fc.g, fc.cfg, fc.dry_d, fc.noise, fc.target_d, th_np, we_np)
                full["plain_loop"] = {"ms_per_step": round(1000 * dt, 2), "audio_s_per_s": round(fc.cfg.seconds / dt, 2),
                                      "speedup": round((1000 * dt) / fm["ms_per_step"], 2),
                                      "what": "PyTorch eager, one node at a time, torch.fft convolutions, "
                                              "truncated-IIR envelope, torch.stft loss, autograd backward"}
            except Exception as e:  # the baseline must not break the headline
                full["plain_loop"] = {"error": repr(e)[:200]}
        fc.release()
        del fc

    schedule_leg = None
    if not args.no_extra and args.prune_rounds > 0:
        try:
            schedule_leg = prune_schedule_leg(rounds=args.prune_rounds)
        except Exception as e:
            schedule_leg = {"error": repr(e)[:300]}

    serving = None
    if not args.no_extra and args.serve_requests > 0:
        try:
            serving = serving_leg(args)
        except Exception as e:  # the serving leg must not break the headline
            serving = {"error": repr(e)[:300]}

    cpu = None
    if not args.no_cpu_baseline:
        try:
            cpu = cpu_baseline(args.config, excerpt_s=10.0 if args.config == "large" else None)
        except Exception as e:
            cpu = {"error": repr(e)[:200]}

    rec = {
        "metric": "console fwd+bwd audio-sec/s",
        "value": round(head["value"], 2),
        "unit": "audio-s/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{cfg.name} console: {cfg.n_tracks} stereo tracks, {cfg.n_subgroups} subgroups, "
                               f"{cfg.seconds:g} s at {cfg.fs} Hz, chain {cfg.chain} per track and subgroup, "
                               f"{cfg.reverb_seconds:g} s reverb, loss FFTs {list(cfg.loss_ffts)}; "
                               "step = forward + MRSTFT loss + backward + Adam",
                   "tracks": cfg.n_tracks, "subgroups": cfg.n_subgroups, "seconds": cfg.seconds,
                   "sample_rate": cfg.fs, "processors": n_proc, "schedule": schedule,
                   "fft_size": fft, "parallelism": "single GPU"},
        "roofline": head["roofline"],
        "hbm_model": head["hbm_model"],
        "copy_ceiling": copy,
        "kernel_classes": head["kernel_classes"],
        "full_console": full,
        "prune_schedule": schedule_leg,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
