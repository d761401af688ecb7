"""FP64 node-by-node evaluation of a mixing graph.  Test infrastructure only.

Follows the paper's definition of a processing graph (Sec. 1.1, Sec. 3
preamble): every node's input is the sum of the outputs of the nodes cabled
into it; processors apply their function and the dry/wet mix; 'm' sums; the
single 'o' node's input sum is the mix.  Nodes are evaluated one at a time in
a topological order (the "one-by-one" schedule of Sec. 4.1), which makes the
oracle independent of any batched schedule.
"""
from __future__ import annotations

import heapq
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import processors as P

DT = torch.float64
LG_EPS = 1e-12     # added to the squared norms inside the gain-staging log


def topo_order(n: int, edges: Sequence[Tuple[int, int]]) -> List[int]:
    """Kahn's algorithm, smallest ready node first; raises on a cycle."""
    indeg = [0] * n
    out: List[List[int]] = [[] for _ in range(n)]
    for s, d in edges:
        out[s].append(d)
        indeg[d] += 1
    ready = [v for v in range(n) if indeg[v] == 0]
    heapq.heapify(ready)
    order = []
    while ready:
        v = heapq.heappop(ready)
        order.append(v)
        for d in out[v]:
            indeg[d] -= 1
            if indeg[d] == 0:
                heapq.heappush(ready, d)
    if len(order) != n:
        raise ValueError("graph has a cycle")
    return order


def _half_log_energy(x: torch.Tensor) -> torch.Tensor:
    """log ||x||_2 with LG_EPS inside the square root."""
    return 0.5 * torch.log(torch.sum(x * x) + LG_EPS)


def process(t: str, u: torch.Tensor, p: torch.Tensor, cfg, noise=None) -> torch.Tensor:
    """ybar = f_t(u, p) for one processor of type t."""
    if t == "g":
        return P.gain_pan(u, p)
    if t == "s":
        return P.imager(u, p)
    if t == "x":
        return P.tanh_dist(u, p)
    if t == "e":
        return P.equalizer(u, p, cfg.eq_taps)
    if t == "c":
        return P.dynamics(u, p, gate=False, attack_release=(cfg.comp_mode == "attack_release"))
    if t == "n":
        return P.dynamics(u, p, gate=True)
    if t == "d":
        return P.delay(u, p, cfg.delay_taps, cfg.delay_range, cfg.delay_fir_taps)
    if t == "r":
        return P.reverb(u, p, noise, cfg.fs)
    raise ValueError(t)


def evaluate(graph, cfg, dry: np.ndarray, noise: Dict[int, np.ndarray],
             theta: Dict[int, torch.Tensor], wet: Dict[int, torch.Tensor],
             mask: Optional[Dict[int, float]] = None, keep_nodes: bool = False):
    """Evaluate every node once.  Returns a dict with
      mix   [2, L] output of the 'o' node,
      Lg    gain-staging regulariser sum over e/r/d nodes (Sec. 5.1),
      Lp    l1 norm of the effective dry/wet weights (Sec. 6.3),
      y     {node: output} when keep_nodes."""
    n = graph.n_nodes
    order = topo_order(n, graph.edges)
    preds: List[List[int]] = [[] for _ in range(n)]
    for s, d in graph.edges:
        preds[d].append(s)
    L = dry.shape[-1]
    y: Dict[int, torch.Tensor] = {}
    Lg = torch.zeros((), dtype=DT)
    Lp = torch.zeros((), dtype=DT)
    mix = None
    for v in order:
        t = graph.types[v]
        if t == "i":
            src = torch.from_numpy(np.asarray(dry[graph.track_of_input[v]], dtype=np.float64))
            y[v] = src.expand(2, L).clone() if src.shape[0] == 1 else src.clone()
            continue
        u = torch.zeros(2, L, dtype=DT)
        for s in sorted(preds[v]):
            u = u + y[s]
        if t == "m":
            y[v] = u
            continue
        if t == "o":
            y[v] = u
            mix = u
            continue
        nz = None
        if t == "r":
            nz = torch.from_numpy(np.asarray(noise[v], dtype=np.float64))
        ybar = process(t, u, theta[v], cfg, nz)
        w = torch.sigmoid(wet[v])
        if mask is not None:
            w = w * float(mask.get(v, 1.0))
        y[v] = P.dry_wet(ybar, u, w)
        Lp = Lp + w
        if t in "erd":
            Lg = Lg + torch.abs(_half_log_energy(ybar[0] + ybar[1]) - _half_log_energy(u[0] + u[1]))
    out = {"mix": mix, "Lg": Lg, "Lp": Lp}
    if keep_nodes:
        out["y"] = y
    return out
