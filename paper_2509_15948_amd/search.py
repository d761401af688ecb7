"""The paper's search regime on the library (host control only; every step
of the arithmetic runs in libmixgraph):

  * console phase: AdamW steps on random segments of the song, the first
    second of each segment excluded from the loss (it warms up the
    processors with long states), Sec. 5.1;
  * pruning phase: iterations of candidate trials and graph surgery, each
    followed by fine-tuning, with the dry/wet l1 weight alpha_p ramped
    linearly from 0 over the first steps of the phase, Sec. 6.3; candidates
    from the brute-force method (batched single bypasses and prefix trials),
    the dry/wet method (Alg. 3) or the hybrid of the two (Sec. 6.2), with an
    absolute tolerance tau;
  * the consistency check of Sec. 7.7: the pruned graph and its mix become a
    synthetic ground truth, the search runs again on that mix, and the two
    graphs are compared processor by processor (per type: accuracy,
    precision, recall, F1).

Two sessions share one parameter vector: a training graph compiled for the
segment length, and an evaluation graph for the whole song, which the
pruning trials and L_min use.  Both have the same topology, so the same
parameter layout.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import mixgraph as MG
from . import workloads as W


@dataclasses.dataclass(frozen=True)
class Regime:
    console_steps: int = 6000     # console training (Sec. 6.3: 6k)
    rounds: int = 12              # pruning iterations (N_iter = 12)
    finetune: int = 500           # fine-tune steps after each iteration
    segment_s: float = 3.8        # random segment per step (Sec. 5.1)
    warmup_s: float = 1.0         # leading part of a segment excluded from the loss
    lr: float = 1e-2
    weight_decay: float = 1e-2    # AdamW; the paper does not state it (PyTorch's default)
    alpha_g: float = 1e-3
    alpha_p: float = 1e-4         # final weight of the dry/wet l1 term
    alpha_p_ramp: int = 4000      # steps of the pruning phase over which alpha_p rises from 0
    tau: float = 0.01             # absolute tolerance (the paper's default)
    sampler: str = "hybrid"       # "brute", "drywet" or "hybrid"
    seed: int = 0                 # segment offsets and type draws


def _alpha_p(reg: Regime, t: int) -> float:
    return reg.alpha_p * min(1.0, t / max(1, reg.alpha_p_ramp))


class _State:
    """Graphs, sessions and parameters of one search (device tensors)."""

    def __init__(self, torch, song_graph, cfg, dry_d, noise: Dict[int, np.ndarray], target_d, th0, we0, reg, dev):
        self.torch, self.cfg, self.reg, self.dev = torch, cfg, reg, dev
        self.seg_len = int(round(reg.segment_s * cfg.fs))
        if self.seg_len > cfg.length:
            raise ValueError("the song is shorter than one segment")
        seg_cfg = dataclasses.replace(cfg, seconds=self.seg_len / cfg.fs)
        self.seg_cfg = seg_cfg
        skip = int(round(reg.warmup_s * cfg.fs))
        P = len(song_graph.processors())
        self.train_g = MG.Graph(song_graph.types, song_graph.edge_array(), self._tracks(song_graph),
                                cfg.n_tracks, 2 if cfg.stereo_tracks else 1,
                                W.binding_config(seg_cfg, reg.alpha_g, 0.0, loss_skip=skip))
        self.eval_g = MG.Graph(song_graph.types, song_graph.edge_array(), self._tracks(song_graph), cfg.n_tracks,
                               2 if cfg.stereo_tracks else 1,
                               W.binding_config(cfg, reg.alpha_g, 0.0, loss_skip=skip, max_trials=P,
                                                trial_slots=4 * song_graph.n_nodes))
        self.dry_d, self.target_d = dry_d, target_d
        self.noise = dict(noise)
        self.orig = list(range(song_graph.n_nodes))      # current node -> node of the first console
        self.seg_dry = torch.empty(cfg.n_tracks, dry_d.shape[1], self.seg_len, device=dev)
        self.seg_tgt = torch.empty(2, self.seg_len, device=dev)
        self._sessions()
        th, we = self.eval_g.flatten(th0, we0)
        self.theta = torch.from_numpy(th).to(dev)
        self.wet = torch.from_numpy(we).to(dev)
        self.m_t, self.v_t = torch.zeros_like(self.theta), torch.zeros_like(self.theta)
        self.m_w, self.v_w = torch.zeros_like(self.wet), torch.zeros_like(self.wet)
        self.gth, self.gwe = torch.empty_like(self.theta), torch.empty_like(self.wet)
        self.n_step = 0

    @staticmethod
    def _tracks(g):
        return [g.track_of_input.get(v, -1) for v in range(g.n_nodes)]

    def _noise_rows(self, g: MG.Graph):
        rows = g.reverb_rows()
        if not rows:
            return np.zeros((1, 2, max(self.cfg.reverb_length, 1)), np.float32)
        return np.stack([self.noise[self.orig[v]] for v in rows]).astype(np.float32)

    def _sessions(self):
        torch = self.torch
        self.train_s = None
        self.eval_s = None
        self.noise_tr = torch.from_numpy(self._noise_rows(self.train_g)).to(self.dev)
        self.eval_s = MG.Session(self.eval_g, self.noise_tr, self.target_d, mode=0, device=self.dev)
        self.seg_tgt.copy_(self.target_d[:, :self.seg_len])
        self.train_s = MG.Session(self.train_g, self.noise_tr, self.seg_tgt, mode=1, device=self.dev)

    def step(self, rng: np.random.Generator, alpha_p: float):
        torch, reg = self.torch, self.reg
        off = int(rng.integers(0, self.cfg.length - self.seg_len + 1))
        self.seg_dry.copy_(self.dry_d[:, :, off:off + self.seg_len])
        self.seg_tgt.copy_(self.target_d[:, off:off + self.seg_len])
        s = self.train_s
        st = s.stream()
        MG.mg_set_alpha(self.train_g.h, reg.alpha_g, alpha_p)
        MG.mg_target_prepare(self.train_g.h, self.seg_tgt, st)
        s.forward(self.seg_dry, self.theta, self.wet)
        s.backward(self.gth, self.gwe)
        self.n_step += 1
        MG.mg_adamw_step(self.theta, self.m_t, self.v_t, self.gth, self.train_g.n_theta, reg.lr, 0.9, 0.999, 1e-8,
                         reg.weight_decay, self.n_step, st)
        MG.mg_adamw_step(self.wet, self.m_w, self.v_w, self.gwe, self.train_g.n_proc, reg.lr, 0.9, 0.999, 1e-8,
                         reg.weight_decay, self.n_step, st)

    def evaluate(self) -> float:
        out = self.torch.zeros(7, dtype=self.torch.float64, device=self.dev)
        self.eval_s.forward(self.dry_d, self.theta, self.wet, None, None, out)
        return float(out[1].item())

    def mix(self):
        out = self.torch.zeros(7, dtype=self.torch.float64, device=self.dev)
        y = self.torch.empty(2, self.cfg.length, device=self.dev)
        self.eval_s.forward(self.dry_d, self.theta, self.wet, None, y, out)
        return y, float(out[1].item())

    def compact(self, alive: np.ndarray):
        """Graph surgery on both graphs, parameters and AdamW moments carried
        over (Sec. 1.2: bypass equals removal)."""
        torch = self.torch
        self.train_s = None
        self.eval_s = None
        new_eval, o2n = self.eval_g.prune(np.asarray(alive, np.uint8))
        new_train, o2n_t = self.train_g.prune(np.asarray(alive, np.uint8))
        assert np.array_equal(o2n, o2n_t)
        st = torch.cuda.current_stream().cuda_stream
        out = []
        for a in (self.theta, self.m_t, self.v_t):
            b = torch.empty(new_eval.n_theta, dtype=torch.float32, device=self.dev)
            MG.mg_remap_params(self.eval_g.h, new_eval.h, o2n, a, b, None, None, st)
            out.append(b)
        outw = []
        for a in (self.wet, self.m_w, self.v_w):
            b = torch.empty(new_eval.n_proc, dtype=torch.float32, device=self.dev)
            MG.mg_remap_params(self.eval_g.h, new_eval.h, o2n, None, None, a, b, st)
            outw.append(b)
        torch.cuda.synchronize()
        orig = [0] * int((o2n >= 0).sum())
        for v, u in enumerate(o2n):
            if u >= 0:
                orig[u] = self.orig[v]
        self.orig = orig
        self.eval_g, self.train_g = new_eval, new_train
        self.theta, self.m_t, self.v_t = out
        self.wet, self.m_w, self.v_w = outw
        self.gth, self.gwe = torch.empty_like(self.theta), torch.empty_like(self.wet)
        self._sessions()

    def kept(self, n_orig_nodes: int) -> np.ndarray:
        """1 for every node of the first console still in the graph."""
        k = np.zeros(n_orig_nodes, np.uint8)
        k[self.orig] = 1
        return k


def run_search(song_graph, cfg, dry: np.ndarray, noise: Dict[int, np.ndarray], target, reg: Regime,
               th0, we0, device: str = "cuda", log=None) -> Dict:
    """The whole search of one song (console phase, then the pruning
    iterations).  target: host float32 [2][L] or a device tensor."""
    import torch
    dev = device
    dry_d = torch.from_numpy(np.ascontiguousarray(dry, np.float32)).to(dev)
    target_d = (torch.from_numpy(np.ascontiguousarray(target, np.float32)).to(dev)
                if isinstance(target, np.ndarray) else target)
    S = _State(torch, song_graph, cfg, dry_d, noise, target_d, th0, we0, reg, dev)
    rng = np.random.default_rng([reg.seed, 1])
    draws = np.random.default_rng([reg.seed, 2])
    t0 = time.perf_counter()
    for _ in range(reg.console_steps):
        S.step(rng, 0.0)
    torch.cuda.synchronize()
    t_console = time.perf_counter() - t0
    L_min = S.evaluate()
    La_console = L_min
    if log:
        log(f"console phase: {reg.console_steps} steps in {t_console:.1f} s, L_a {La_console:.4f}")
    trace = []
    w_delta = []
    t_prune = 0
    P0 = S.eval_g.n_proc
    for n in range(1, reg.rounds + 1):
        method = reg.sampler if reg.sampler != "hybrid" else ("brute" if n % 4 == 0 else "drywet")
        t1 = time.perf_counter()
        P = S.eval_g.n_proc
        if method == "brute":
            w_now = 1.0 / (1.0 + np.exp(-S.wet.detach().cpu().numpy().astype(np.float64)))
            ptype = S.eval_g.proc_types()
            res = MG.prune_round(S.eval_s, S.dry_d, S.theta, S.wet, None, tau=reg.tau, max_candidates=P,
                                 L_min=L_min, relative=False)
            trials = len(res["candidates"]) + len(res["order"])
            # each candidate's dry/wet weight against the loss increase of
            # bypassing it alone (the relation the dry/wet method relies on)
            for j, Lj in zip(res["candidates"], res["L_cand"]):
                w_delta.append((float(w_now[j]), float(Lj) - float(res["La"]), int(ptype[j])))
        else:
            u = draws.random(4 * P + 64)
            res = MG.drywet_round(S.eval_s, S.dry_d, S.theta, S.wet, u, tau=reg.tau, relative=False, L_min=L_min)
            trials = res["trials"]
        L_min = res["L_min"]
        removed = int((res["alive"] == 0).sum())
        if removed:
            S.compact(res["alive"])
        for _ in range(reg.finetune):
            S.step(rng, _alpha_p(reg, t_prune))
            t_prune += 1
        torch.cuda.synchronize()
        trace.append({"round": n, "method": method, "trials": trials, "removed": removed,
                      "processors": S.eval_g.n_proc, "L_min": L_min, "seconds": time.perf_counter() - t1})
        if log:
            log(f"round {n} ({method}): {trials} trials, removed {removed}, {S.eval_g.n_proc} processors left")
    y, La_final = S.mix()
    kept = S.kept(song_graph.n_nodes)
    out = {"La_console": La_console, "La_final": La_final, "processors_start": P0,
           "processors_end": S.eval_g.n_proc, "pruning_ratio": 1.0 - S.eval_g.n_proc / max(P0, 1),
           "kept": kept, "trace": trace, "console_s": t_console, "total_s": time.perf_counter() - t0,
           "theta": S.theta.cpu().numpy(), "wet": S.wet.cpu().numpy(), "mix": y.cpu().numpy(),
           "types": list(S.eval_g.types), "orig": list(S.orig), "w_delta": w_delta}
    return out


def _ranks(x: np.ndarray) -> np.ndarray:
    """Ranks 0..n-1, ties given their mean rank."""
    order = np.argsort(x, kind="stable")
    r = np.empty(len(x), np.float64)
    r[order] = np.arange(len(x), dtype=np.float64)
    for v in np.unique(x):
        sel = x == v
        if sel.sum() > 1:
            r[sel] = r[sel].mean()
    return r


def w_delta_summary(pairs, tau: float) -> Dict:
    """Dry/wet weight w of every brute-force candidate against the loss
    increase Delta of bypassing it alone: the Spearman rank correlation, and
    per quarter of the candidates by w the median Delta and the share within
    the tolerance (Delta < tau), overall and by processor type."""
    if not pairs:
        return {}
    w = np.array([p[0] for p in pairs])
    d = np.array([p[1] for p in pairs])
    t = np.array([p[2] for p in pairs])

    def spearman(a, b):
        if len(a) < 3:
            return None
        ra, rb = _ranks(a), _ranks(b)
        ra, rb = ra - ra.mean(), rb - rb.mean()
        den = np.sqrt((ra * ra).sum() * (rb * rb).sum())
        return round(float((ra * rb).sum() / den), 4) if den > 0 else None

    q = np.quantile(w, [0.0, 0.25, 0.5, 0.75, 1.0])
    bins = []
    for i in range(4):
        sel = (w >= q[i]) & ((w <= q[i + 1]) if i == 3 else (w < q[i + 1]))
        if sel.any():
            bins.append({"w_range": [round(float(q[i]), 4), round(float(q[i + 1]), 4)], "n": int(sel.sum()),
                         "median_delta": round(float(np.median(d[sel])), 6),
                         "within_tau": round(float(np.mean(d[sel] < tau)), 3)})
    names = {v: k for k, v in MG.TYPE_CODES.items()}
    by_type = {names.get(int(k), str(k)): spearman(w[t == k], d[t == k]) for k in np.unique(t)}
    return {"candidates": len(pairs), "spearman_w_delta": spearman(w, d), "by_w_quarter": bins,
            "spearman_by_type": by_type}


def processor_agreement(types: Sequence[str], truth: np.ndarray, pred: np.ndarray) -> Dict:
    """Per processor type and micro-averaged over all processors: accuracy,
    precision, recall and F1 of `pred` (1 = the processor is kept) against
    `truth`, over the processors of the first console (Sec. 7.7: per track
    and subgroup, whether a type is present)."""
    out = {}
    procs = [v for v, t in enumerate(types) if t not in "imo"]

    def metrics(vs):
        t = truth[vs].astype(bool)
        p = pred[vs].astype(bool)
        tp, fp = int((t & p).sum()), int((~t & p).sum())
        fn, tn = int((t & ~p).sum()), int((~t & ~p).sum())
        acc = (tp + tn) / max(1, len(vs))
        prec = tp / (tp + fp) if tp + fp else 1.0
        rec = tp / (tp + fn) if tp + fn else 1.0
        f1 = 2 * prec * rec / (prec + rec) if prec + rec else 0.0
        return {"n": len(vs), "tp": tp, "fp": fp, "fn": fn, "tn": tn, "accuracy": acc, "precision": prec,
                "recall": rec, "f1": f1}

    for ty in sorted({types[v] for v in procs}):
        out[ty] = metrics([v for v in procs if types[v] == ty])
    out["micro"] = metrics(procs)
    return out


def consistency_check(song_graph, cfg, dry, noise, target, reg: Regime, init, device="cuda", log=None) -> Dict:
    """Sec. 7.7: search once on the target; take the pruned graph and its
    matched mix as a synthetic ground truth; search again from a fresh
    console on that mix; compare the two pruned graphs processor by
    processor."""
    th0, we0 = init
    first = run_search(song_graph, cfg, dry, noise, target, reg, th0, we0, device, log)
    reg2 = dataclasses.replace(reg, seed=reg.seed + 1)
    second = run_search(song_graph, cfg, dry, noise, first["mix"].astype(np.float32), reg2, th0, we0, device, log)
    agree = processor_agreement(song_graph.types, first["kept"], second["kept"])
    return {"first": {k: first[k] for k in ("La_console", "La_final", "processors_end", "pruning_ratio")},
            "second": {k: second[k] for k in ("La_console", "La_final", "processors_end", "pruning_ratio")},
            "agreement": agree}


def paper_song_config(n_tracks: int = 18, n_subgroups: int = 4, seconds: float = 30.0):
    """A synthetic song shaped like the paper's data (Sec. 5.3: 17.6 tracks on
    average in MedleyDB) and console (Sec. 3, Sec. 5.1): chain e c n s g d r,
    a 2047-tap EQ (1024 parameters), 20 delay taps over 2 s, a 2 s reverb,
    30 kHz, loss FFTs 512 / 1024 / 4096."""
    import synth
    return synth.ConsoleConfig("paper", n_tracks, n_subgroups, seconds, 30000, True, chain="ecnsgdr",
                               eq_taps=2047, delay_taps=20, delay_range_s=2.0, delay_fir_taps=39,
                               reverb_seconds=2.0, loss_ffts=(512, 1024, 4096))


def render(song_graph, cfg, dry: np.ndarray, noise: Dict[int, np.ndarray], theta, wet, device: str = "cuda"):
    """The mix of a graph for per-node raw parameters, rendered by the
    library (a forward-only session); host float32 [2][L]."""
    import torch
    bg = W.binding_graph(song_graph, cfg)
    noise_d = torch.from_numpy(W.noise_rows(bg, noise, cfg.reverb_length)).to(device)
    y = torch.zeros(2, cfg.length, device=device)
    sess = MG.Session(bg, noise_d, y, mode=0, device=device)
    th, we = bg.flatten(theta, wet)
    out = torch.zeros(7, dtype=torch.float64, device=device)
    sess.forward(torch.from_numpy(dry).to(device), torch.from_numpy(th).to(device), torch.from_numpy(we).to(device),
                 None, y, out)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def main(argv=None) -> None:
    """The paper's search on a synthetic song: a sweep over candidate samplers
    and tolerances (the analogue of the sampling-method comparison of Sec.
    7.4), then the consistency check of Sec. 7.7; one JSON line per run."""
    import argparse
    import json
    import sys

    import synth
    ap = argparse.ArgumentParser(description=main.__doc__.splitlines()[0])
    ap.add_argument("--tracks", type=int, default=18)
    ap.add_argument("--subgroups", type=int, default=4)
    ap.add_argument("--seconds", type=float, default=30.0)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--console-steps", type=int, default=6000)
    ap.add_argument("--rounds", type=int, default=12)
    ap.add_argument("--finetune", type=int, default=500)
    ap.add_argument("--samplers", default="brute,drywet,hybrid")
    ap.add_argument("--taus", default="0.001,0.01,0.1")
    ap.add_argument("--consistency", action="store_true", help="also run the consistency check (hybrid, tau 0.01)")
    a = ap.parse_args(argv)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    cfg = paper_song_config(a.tracks, a.subgroups, a.seconds)
    g, dry, noise = synth.song(a.seed, cfg)
    gt, gw = synth.ground_truth_params(a.seed + 100, g, cfg)
    target = render(g, cfg, dry, noise, gt, gw)
    init = synth.init_params(a.seed, g, cfg)
    base = Regime(console_steps=a.console_steps, rounds=a.rounds, finetune=a.finetune, seed=a.seed)
    types = g.types
    for sampler in a.samplers.split(","):
        for tau in [float(x) for x in a.taus.split(",")]:
            reg = dataclasses.replace(base, sampler=sampler, tau=tau)
            log(f"search: sampler {sampler}, tau {tau}")
            r = run_search(g, cfg, dry, noise, target, reg, init[0], init[1], log=log)
            kept_by_type = {}
            for v in g.processors():
                kept_by_type.setdefault(types[v], []).append(int(r["kept"][v]))
            print(json.dumps({
                "run": "search", "sampler": sampler, "tau": tau, "La_console": round(r["La_console"], 5),
                "La_final": round(r["La_final"], 5), "processors_start": r["processors_start"],
                "processors_end": r["processors_end"], "pruning_ratio": round(r["pruning_ratio"], 4),
                "kept_ratio_by_type": {t: round(float(np.mean(k)), 3) for t, k in kept_by_type.items()},
                "trials": sum(x["trials"] for x in r["trace"]), "console_s": round(r["console_s"], 2),
                "w_vs_delta": w_delta_summary(r["w_delta"], tau),
                "total_s": round(r["total_s"], 2),
                "workload": f"{cfg.n_tracks} tracks, {cfg.n_subgroups} subgroups, {cfg.seconds:g} s at {cfg.fs} Hz, "
                            f"chain {cfg.chain}; {reg.console_steps} console steps, {reg.rounds} rounds x "
                            f"{reg.finetune} fine-tune steps, {reg.segment_s} s segments"}), flush=True)
    if a.consistency:
        reg = dataclasses.replace(base, sampler="hybrid", tau=0.01)
        log("consistency check")
        c = consistency_check(g, cfg, dry, noise, target, reg, init, log=log)
        print(json.dumps({"run": "consistency", **c}, default=float), flush=True)


if __name__ == "__main__":
    main()
