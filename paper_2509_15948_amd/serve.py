"""Serving loop for whole-song mixing-graph searches (continuous batching).

Requests arrive over time.  Each one is a complete search on its own song:
optimisation steps of the full console, then pruning rounds (batched trials,
the decision rule, graph surgery, fine-tune steps on the smaller graph).  The
server

  * admits an arrived request as soon as a slot is free and its device
    footprint (workspace, tensors, Adam moments) fits the memory budget;
  * keeps every admitted search's state resident on the device until it
    retires (dry tracks, target features, parameters, moments, masks);
  * gives every active search its own HIP stream (default priority) and
    enqueues its work in quanta, so the kernels of different searches
    overlap on the GPU while the host prepares the next quanta;
  * reads a search's losses back only at its pruning decisions, waiting on
    events of that search's stream, never on the whole device.

Every search is a coroutine that yields a HIP event after each enqueued
quantum; the loop resumes it when the event has completed.  The arithmetic
of every step runs in libmixgraph; this module schedules and moves buffers.
Results of a search depend on its own inputs only (the kernels use no
atomics and no state shared between graphs), so a search gives the same bits
alone and in the mix.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Dict, List, Optional

import numpy as np

from . import mixgraph as MG
from . import workloads as W


@dataclasses.dataclass(frozen=True)
class SearchSpec:
    steps: int = 300          # optimisation steps before pruning
    rounds: int = 10          # pruning rounds
    finetune: int = 50        # fine-tune steps after each round
    tau: float = 1e-3         # relative loss tolerance of a round
    candidates: int = 64      # trials per round
    lr: float = 1e-2
    quantum: int = 4          # steps enqueued before yielding to the loop
    stop_when_none: bool = False  # end the rounds at the first that removes nothing
    # forward + backward replayed as one captured HIP graph (mixgraph.StepGraph).
    # Off: with it on, a serving test that admits searches one at a time
    # ended in a host segmentation fault inside the graph replay, whose cause
    # has not been found; the captured step itself replays bit for bit.
    graph_steps: bool = False


class PruneThreshold:
    """The loss threshold of Alg. 2 across the rounds of one search.

    L_min is the audio loss of the trained console, taken once at the first
    round; a round accepts the longest prefix of its ordered candidates whose
    loss stays below L_min (1 + tau), and an accepted prefix with a smaller
    loss lowers L_min (Alg. 2, the min update).  The threshold is never reset
    to the current loss, so the losses the rounds accept all stay within
    (1 + tau) of the console's.  The rule itself is the library's
    (mg_prune_order, mg_prune_accept)."""

    def __init__(self, tau: float, relative: bool = True):
        self.tau = tau
        self.relative = relative
        self.L_min: Optional[float] = None

    def observe(self, La: float) -> None:
        if self.L_min is None:
            self.L_min = float(La)

    def order(self, cand: np.ndarray, L_cand: np.ndarray) -> np.ndarray:
        if not len(cand):
            return np.zeros(0, np.int32)
        return MG.mg_prune_order(cand, L_cand, self.L_min, self.tau, self.relative)

    def accept(self, L_prefix: np.ndarray) -> int:
        k = MG.mg_prune_accept(L_prefix, self.L_min, self.tau, self.relative)
        if k:
            self.L_min = min(self.L_min, float(L_prefix[k - 1]))
        return k


class Search:
    """One request: host inputs, device state, and its search coroutine."""

    def __init__(self, rid: int, cfg, seed: int, spec: SearchSpec, song=None, params=None):
        import synth
        self.rid, self.cfg, self.seed, self.spec = rid, cfg, seed, spec
        self.g, self.dry, self.noise = song if song is not None else synth.song(seed, cfg)
        self.gt = synth.ground_truth_params(seed + 100, self.g, cfg)
        self.init = params if params is not None else synth.init_params(seed, self.g, cfg)
        self.bg = W.binding_graph(self.g, cfg, max_trials=spec.candidates)
        P, nt = self.bg.n_proc, self.bg.n_theta
        # the library's footprint of one search: workspace plus the buffers
        # its calls read and write (dry, noise, target, mix, parameters with
        # gradients and moments, loss records); the target render's
        # forward-only workspace is released before the search's own is made
        self.ws_bytes, state = MG.mg_footprint(self.bg.h, 1)
        self.bytes = self.ws_bytes + state
        self.trace: List[Dict] = []
        self.result: Optional[Dict] = None

    # ------------------------------------------------------------ device state
    def _setup(self, torch, dev):
        cfg, bg = self.cfg, self.bg
        self.dry_d = torch.from_numpy(self.dry).to(dev)
        self.noise_d = torch.from_numpy(W.noise_rows(bg, self.noise, cfg.reverb_length)).to(dev)
        th_gt, we_gt = bg.flatten(*self.gt)
        self.target_d = torch.zeros(2, cfg.length, device=dev)
        # the target: the same console with ground-truth parameters, rendered by
        # the library; the search's session is set up once the target holds it
        render = MG.Session(bg, self.noise_d, self.target_d, mode=0)
        render.forward(self.dry_d, torch.from_numpy(th_gt).to(dev), torch.from_numpy(we_gt).to(dev), None,
                       self.target_d)
        del render
        self.sess = MG.Session(bg, self.noise_d, self.target_d, mode=1)
        th, we = bg.flatten(*self.init)
        self.theta = torch.from_numpy(th).to(dev)
        self.wet = torch.from_numpy(we).to(dev)
        self.gth = torch.empty_like(self.theta)
        self.gwe = torch.empty_like(self.wet)
        self.m_t, self.v_t = torch.zeros_like(self.theta), torch.zeros_like(self.theta)
        self.m_w, self.v_w = torch.zeros_like(self.wet), torch.zeros_like(self.wet)
        self.mask = torch.ones(bg.n_proc, device=dev)
        self.alive = np.ones(bg.n_proc, np.uint8)
        self.noise_by_node = dict(self.noise)
        self.losses = torch.zeros(7, dtype=torch.float64, device=dev)
        self.n_step = 0
        self._graph = None

    def _compact(self, torch, dev):
        """Remove the pruned processors from the graph (graph surgery) and
        carry parameters and Adam moments over to the smaller graph.  The old
        workspace is released first (surgery and the parameter remap need the
        host graph and the parameter vectors only), so a compacting search
        never holds two workspaces.  The allocator orders the reuse of the
        freed workspace on this search's stream after the work that read it
        (the side stream's work has joined that stream by then)."""
        self.sess = None
        self._graph = None
        new, o2n, sess, noise_d, th, we = MG.compact(self.bg, self.alive, self.noise_by_node, self.cfg.reverb_length,
                                                     self.target_d, (self.theta, self.m_t, self.v_t),
                                                     (self.wet, self.m_w, self.v_w), dev)
        self.noise_by_node = {int(o2n[v]): nz for v, nz in self.noise_by_node.items() if o2n[v] >= 0}
        self.bg, self.sess, self.noise_d = new, sess, noise_d
        self.theta, self.m_t, self.v_t = th
        self.wet, self.m_w, self.v_w = we
        self.gth = torch.empty_like(self.theta)
        self.gwe = torch.empty_like(self.wet)
        self.mask = torch.ones(new.n_proc, device=dev)
        self.alive = np.ones(new.n_proc, np.uint8)

    def _step(self):
        s = self.sess
        st = s.stream()
        self.n_step += 1
        if self.spec.graph_steps:
            # captured at the first step on this session and these buffers
            # (graph surgery replaces both), then one launch per step
            if self._graph is None or self._graph.session is not s:
                self._graph = MG.StepGraph(s, self.dry_d, self.theta, self.wet, self.mask, self.losses, self.gth,
                                           self.gwe)
            self._graph.replay()
        else:
            s.forward(self.dry_d, self.theta, self.wet, self.mask, None, self.losses)
            s.backward(self.gth, self.gwe)
        MG.mg_adam_step(self.theta, self.m_t, self.v_t, self.gth, self.bg.n_theta, self.spec.lr, 0.9, 0.999, 1e-8,
                        self.n_step, st)
        MG.mg_adam_step(self.wet, self.m_w, self.v_w, self.gwe, self.bg.n_proc, self.spec.lr, 0.9, 0.999, 1e-8,
                        self.n_step, st)

    def run(self, torch, dev):
        """The search as a coroutine: yields an event after each quantum."""
        spec = self.spec
        self._setup(torch, dev)

        def mark():
            ev = torch.cuda.Event()
            ev.record()
            return ev

        yield mark()
        for i in range(spec.steps):
            self._step()
            if (i + 1) % spec.quantum == 0:
                yield mark()
        yield mark()
        P = self.bg.n_proc
        thr = PruneThreshold(spec.tau)

        def timed():
            ev = torch.cuda.Event(enable_timing=True)
            ev.record()
            return ev

        for r in range(spec.rounds):
            t_round = time.perf_counter()
            # forward at the current mask (the cache the trials read), then
            # single-bypass trials
            self.sess.forward(self.dry_d, self.theta, self.wet, self.mask, None, self.losses)
            yield mark()
            thr.observe(float(self.losses[1].item()))
            L_start = thr.L_min
            trial_ev = []
            cand = MG.mg_prune_candidates(self.wet.cpu().numpy(), self.mask.cpu().numpy(), self.alive,
                                          spec.candidates)
            out = torch.zeros(max(1, len(cand)), 7, dtype=torch.float64, device=dev)
            if len(cand):
                keep = np.ones((len(cand), P), np.uint8)
                keep[np.arange(len(cand)), cand] = 0
                trial_ev.append(timed())
                self.sess.forward_trials(keep, out)
                trial_ev.append(timed())
                yield mark()
            L_cand = out[:len(cand), 1].cpu().numpy()
            order = thr.order(cand, L_cand)
            k = 0
            if len(order):
                keep = np.ones((len(order), P), np.uint8)
                for j in range(len(order)):
                    keep[j, order[:j + 1]] = 0
                outp = torch.zeros(len(order), 7, dtype=torch.float64, device=dev)
                trial_ev.append(timed())
                self.sess.forward_trials(keep, outp)
                trial_ev.append(timed())
                yield mark()
                L_prefix = outp[:, 1].cpu().numpy()
                k = thr.accept(L_prefix)
            if k:
                self.alive[order[:k]] = 0
                self._compact(torch, dev)
            trial_ms = sum(a.elapsed_time(b) for a, b in zip(trial_ev[0::2], trial_ev[1::2]))
            entry = {"round": r, "L_start": L_start, "L_min": thr.L_min, "candidates": len(cand),
                     "within": len(order), "removed": int(k), "processors": int(self.bg.n_proc),
                     "trial_ms": trial_ms}
            self.trace.append(entry)
            P = self.bg.n_proc
            if k == 0 and spec.stop_when_none:
                entry["seconds"] = time.perf_counter() - t_round
                break
            for i in range(spec.finetune):
                self._step()
                if (i + 1) % spec.quantum == 0:
                    yield mark()
            yield mark()
            entry["seconds"] = time.perf_counter() - t_round
        # final loss at the final parameters and mask
        self.sess.forward(self.dry_d, self.theta, self.wet, self.mask, None, self.losses)
        yield mark()
        self.result = {"losses": self.losses.cpu().numpy().copy(), "theta": self.theta.cpu().numpy().copy(),
                       "wet": self.wet.cpu().numpy().copy(), "processors": int(self.bg.n_proc),
                       "types": list(self.bg.types), "trace": list(self.trace)}

    def release(self):
        for name in ("_graph", "sess", "dry_d", "noise_d", "target_d", "theta", "wet", "gth", "gwe", "m_t", "v_t",
                     "m_w", "v_w", "mask", "losses", "noise_by_node"):
            if hasattr(self, name):
                delattr(self, name)


class Admission:
    """Which arrived requests may start now: first come, first served, while
    a slot is free and the footprint fits the budget (a request larger than
    the whole budget runs alone)."""

    def __init__(self, budget_bytes: int, max_active: int):
        self.budget = budget_bytes
        self.max_active = max_active
        self.used = 0
        self.active = 0

    def can_admit(self, nbytes: int) -> bool:
        if self.active >= self.max_active:
            return False
        return self.used + nbytes <= self.budget or self.active == 0

    def admit(self, nbytes: int):
        self.used += nbytes
        self.active += 1

    def retire(self, nbytes: int):
        self.used -= nbytes
        self.active -= 1


class Server:
    def __init__(self, budget_bytes: int, max_active: int = 8, device: str = "cuda"):
        self.adm = Admission(budget_bytes, max_active)
        self.device = device

    def run(self, arrivals: List[tuple], make_search: Callable[[int, object, int], Search],
            clock=time.perf_counter, on_done: Optional[Callable[[int, float], None]] = None) -> Dict:
        """arrivals: (arrival time s, cfg, seed) sorted by time.  Requests are
        built on the host ahead of time (data preparation is not search
        latency); each is admitted at or after its arrival time."""
        import torch
        searches = [make_search(i, cfg, seed) for i, (_, cfg, seed) in enumerate(arrivals)]
        pending = collections.deque(range(len(arrivals)))
        active: Dict[int, tuple] = {}
        t0 = clock()
        start, finish, admitted_at = {}, {}, {}
        peak_active, peak_bytes = 0, 0
        while pending or active:
            now = clock() - t0
            while pending and arrivals[pending[0]][0] <= now and self.adm.can_admit(searches[pending[0]].bytes):
                i = pending.popleft()
                self.adm.admit(searches[i].bytes)
                stream = torch.cuda.Stream(device=self.device)
                with torch.cuda.stream(stream):
                    co = searches[i].run(torch, self.device)
                    ev = next(co)
                active[i] = (co, stream, ev)
                admitted_at[i] = now
                peak_active = max(peak_active, len(active))
                peak_bytes = max(peak_bytes, self.adm.used)
            progressed = False
            for i in list(active):
                co, stream, ev = active[i]
                if not ev.query():
                    continue
                progressed = True
                with torch.cuda.stream(stream):
                    try:
                        ev = next(co)
                        active[i] = (co, stream, ev)
                    except StopIteration:
                        finish[i] = clock() - t0
                        if on_done:
                            on_done(i, finish[i] - arrivals[i][0])
                        searches[i].release()
                        self.adm.retire(searches[i].bytes)
                        del active[i]
            if not progressed:
                if not active and pending:
                    wait = arrivals[pending[0]][0] - (clock() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 0.05))
                else:
                    time.sleep(50e-6)
        lat = np.array([finish[i] - arrivals[i][0] for i in range(len(arrivals))])
        audio = sum(cfg.seconds * (s.spec.steps + s.spec.rounds * s.spec.finetune)
                    for (_, cfg, _), s in zip(arrivals, searches))
        span = max(finish.values()) - min(a[0] for a in arrivals) if arrivals else 0.0
        return {"results": [s.result for s in searches], "latency_s": lat.tolist(),
                "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                "songs_per_s": len(arrivals) / span if span > 0 else 0.0,
                "audio_s_per_s": audio / span if span > 0 else 0.0, "makespan_s": span,
                "peak_active": peak_active, "peak_bytes": peak_bytes,
                "queue_wait_s": [admitted_at[i] - arrivals[i][0] for i in range(len(arrivals))]}


def run_alone(search: Search, device: str = "cuda") -> Dict:
    """One search by itself on its own stream (the reference for the mix)."""
    import torch
    stream = torch.cuda.Stream(device=device)
    with torch.cuda.stream(stream):
        for ev in search.run(torch, device):
            ev.synchronize()
    res = search.result
    search.release()
    return res


def main(argv=None) -> None:
    """A serving stream of whole-song searches (Poisson arrivals), printed as
    one JSON line: p50/p99 latency, throughput, concurrency.  The arrival
    rate is --load times the saturated throughput measured first by a
    closed-loop run (every request of a short stream arriving at once)."""
    import argparse
    import json
    import sys

    import torch

    import synth
    ap = argparse.ArgumentParser(description=main.__doc__.splitlines()[0])
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--tracks", type=int, nargs=2, default=(4, 32))
    ap.add_argument("--subgroups", type=int, nargs=2, default=(2, 8))
    ap.add_argument("--seconds", type=float, nargs=2, default=(5.0, 30.0))
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--rounds", type=int, default=10)
    ap.add_argument("--finetune", type=int, default=50)
    ap.add_argument("--candidates", type=int, default=64)
    ap.add_argument("--tau", type=float, default=1e-3)
    ap.add_argument("--load", type=float, default=0.8, help="arrival rate as a fraction of the saturated rate")
    ap.add_argument("--calib-requests", type=int, default=6)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--torch-fraction", type=float, default=0.85,
                    help="share of device memory torch's allocator may hold, cached blocks included")
    ap.add_argument("--max-active", type=int, default=8)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--graphs", action="store_true",
                    help="replay each step as a captured HIP graph (experimental: see SearchSpec.graph_steps)")
    a = ap.parse_args(argv)
    spec = SearchSpec(steps=a.steps, rounds=a.rounds, finetune=a.finetune, tau=a.tau, candidates=a.candidates,
                      quantum=8, graph_steps=a.graphs)
    budget = int(a.budget_gb * (1 << 30))
    # Searches of uneven sizes leave torch's allocator with cached blocks that
    # fit no later request; unchecked, the cache grows until device memory is
    # full, and then the runtime's own allocations (a queue's scratch, say)
    # fail and abort the queue.  Capped, torch releases cached blocks and
    # retries first, and the rest of device memory stays with the runtime.
    torch.cuda.set_per_process_memory_fraction(a.torch_fraction)
    # admitted footprints stay within 80 % of torch's share (the rest absorbs
    # the allocator's rounding and the target renders' transient workspaces)
    budget = min(budget, int(0.8 * a.torch_fraction * torch.cuda.get_device_properties(0).total_memory))

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    def make(i, cfg, seed):
        return Search(i, cfg, seed, spec)

    # closed loop: the saturated rate of this mix
    calib = synth.serving_requests(a.seed + 1000, a.calib_requests, rate=0.0, tracks=tuple(a.tracks),
                                   subgroups=tuple(a.subgroups), seconds=tuple(a.seconds))
    t0 = time.perf_counter()
    c = Server(budget, a.max_active).run(calib, make, on_done=lambda i, lat: log(f"calibration request {i} done"))
    sat = c["songs_per_s"]
    rate = a.load * sat
    log(f"saturated {sat:.3f} songs/s ({time.perf_counter() - t0:.1f} s); arrival rate {rate:.3f} songs/s")
    reqs = synth.serving_requests(a.seed, a.requests, rate=rate, tracks=tuple(a.tracks),
                                  subgroups=tuple(a.subgroups), seconds=tuple(a.seconds))
    n_done = [0]

    def done(i, lat):
        n_done[0] += 1
        log(f"request {i} done ({n_done[0]}/{len(reqs)}), latency {lat:.2f} s")

    out = Server(budget, a.max_active).run(reqs, make, on_done=done)
    removed = [sum(r["removed"] for r in res["trace"]) for res in out["results"]]
    starts = [7 * (cfg.n_tracks + cfg.n_subgroups) for _, cfg, _ in reqs]
    rec = {"requests": len(reqs), "saturated_songs_per_s": round(sat, 4), "arrival_rate_per_s": round(rate, 4),
           "load": a.load,
           "workload": f"tracks U{{{a.tracks[0]}..{a.tracks[1]}}}, subgroups U{{{a.subgroups[0]}..{a.subgroups[1]}}}, "
                       f"{a.seconds[0]:g}-{a.seconds[1]:g} s at 44.1 kHz, chain ecxsgdr; search = {spec.steps} steps "
                       f"+ {spec.rounds} rounds x ({spec.candidates} candidates + {spec.finetune} fine-tune steps)",
           "p50_latency_s": round(out["p50_s"], 3), "p99_latency_s": round(out["p99_s"], 3),
           "songs_per_s": round(out["songs_per_s"], 4), "audio_s_per_s": round(out["audio_s_per_s"], 1),
           "makespan_s": round(out["makespan_s"], 2), "peak_active": out["peak_active"],
           "peak_gb": round(out["peak_bytes"] / (1 << 30), 2), "budget_gb": round(budget / (1 << 30), 1),
           "mean_queue_wait_s": round(float(np.mean(out["queue_wait_s"])), 3), "graph_steps": spec.graph_steps,
           "pruning_ratio_mean": round(float(np.mean([r / s for r, s in zip(removed, starts)])), 4)}
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
