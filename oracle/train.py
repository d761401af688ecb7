"""FP64 objective, gradients and optimiser step.  Test infrastructure only.

L = L_a + alpha_g L_g + alpha_p L_p (Sec. 5.1 and Sec. 6.3).  Gradients come
from torch autograd over the FP64 definitions, with the two hand-written
recursion adjoints of ``processors.py``; the delay's z entries then follow the
gradient rule of Sec. 3.7 (normalised surrogate gradient plus the radius
term).  Adam follows Kingma & Ba with PyTorch's default betas and eps.
"""
from __future__ import annotations

import math
from typing import Dict, Optional

import numpy as np
import torch

from . import console as C
from . import loss as LS
from . import processors as P

DT = torch.float64
LOSS_KEYS = ("L", "La", "Llr", "Lm", "Ls", "Lg", "Lp")


def _leaf(x) -> torch.Tensor:
    return torch.tensor(np.asarray(x, dtype=np.float64), dtype=DT).requires_grad_(True)


def objective(graph, cfg, dry, noise, target, theta, wet, mask=None,
              alpha_g: float = 1e-3, alpha_p: float = 0.0, skip: int = 0,
              keep_nodes: bool = False):
    """Forward pass: dict of torch scalars for LOSS_KEYS plus 'mix'."""
    ev = C.evaluate(graph, cfg, dry, noise, theta, wet, mask, keep_nodes=keep_nodes)
    tgt = torch.from_numpy(np.asarray(target, dtype=np.float64))
    la = LS.mrstft(ev["mix"], tgt, cfg.loss_ffts, cfg.fs, cfg.n_mels, skip)
    out = dict(la)
    out["Lg"] = ev["Lg"]
    out["Lp"] = ev["Lp"]
    out["L"] = la["La"] + alpha_g * ev["Lg"] + alpha_p * ev["Lp"]
    out["mix"] = ev["mix"]
    if keep_nodes:
        out["y"] = ev["y"]
    return out


def render(graph, cfg, dry, noise, theta_np, wet_np, mask=None) -> np.ndarray:
    """Mix of the graph for raw parameters, [2, L] float64 (no gradients)."""
    with torch.no_grad():
        th = {v: torch.tensor(np.asarray(p, dtype=np.float64)) for v, p in theta_np.items()}
        we = {v: torch.tensor(float(w), dtype=DT) for v, w in wet_np.items()}
        return C.evaluate(graph, cfg, dry, noise, th, we, mask)["mix"].numpy()


def losses(graph, cfg, dry, noise, target, theta_np, wet_np, mask=None, alpha_g=1e-3,
           alpha_p=0.0, skip=0) -> Dict[str, float]:
    with torch.no_grad():
        th = {v: torch.tensor(np.asarray(p, dtype=np.float64)) for v, p in theta_np.items()}
        we = {v: torch.tensor(float(w), dtype=DT) for v, w in wet_np.items()}
        out = objective(graph, cfg, dry, noise, target, th, we, mask, alpha_g, alpha_p, skip)
        return {k: float(out[k]) for k in LOSS_KEYS}


def loss_and_grad(graph, cfg, dry, noise, target, theta_np, wet_np, mask=None,
                  alpha_g: float = 1e-3, alpha_p: float = 0.0, skip: int = 0,
                  delay_rule: bool = True):
    """Returns (losses, grad_theta, grad_wet, mix).

    grad_theta[v] has the layout of theta[v]; for delay nodes the (Re z, Im z)
    entries hold the Sec. 3.7 update direction when delay_rule is set, the raw
    surrogate gradient otherwise."""
    th = {v: _leaf(p) for v, p in theta_np.items()}
    we = {v: _leaf(float(w)) for v, w in wet_np.items()}
    out = objective(graph, cfg, dry, noise, target, th, we, mask, alpha_g, alpha_p, skip)
    out["L"].backward()
    gth = {v: (t.grad.numpy().copy() if t.grad is not None else np.zeros(t.shape)) for v, t in th.items()}
    gwe = {v: (float(t.grad) if t.grad is not None else 0.0) for v, t in we.items()}
    if delay_rule:
        Kc = (cfg.delay_fir_taps + 1) // 2
        for v, t in enumerate(graph.types):
            if t != "d":
                continue
            g = gth[v].reshape(2, cfg.delay_taps, 2 + Kc)
            z = np.asarray(theta_np[v], dtype=np.float64).reshape(2, cfg.delay_taps, 2 + Kc)
            for c in range(2):
                for m in range(cfg.delay_taps):
                    g[c, m, 0], g[c, m, 1] = P.delay_grad_rule(g[c, m, 0], g[c, m, 1],
                                                               z[c, m, 0], z[c, m, 1])
            gth[v] = g.reshape(-1)
    vals = {k: float(out[k]) for k in LOSS_KEYS}
    return vals, gth, gwe, out["mix"].detach().numpy()


def adam_step(theta: np.ndarray, m: np.ndarray, v: np.ndarray, g: np.ndarray, step: int,
              lr: float = 1e-2, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma & Ba, Alg. 1), in place; step counts from 1."""
    m *= b1
    m += (1.0 - b1) * g
    v *= b2
    v += (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    theta -= lr * mh / (np.sqrt(vh) + eps)
    return theta, m, v


def adamw_step(theta: np.ndarray, m: np.ndarray, v: np.ndarray, g: np.ndarray, step: int,
               lr: float = 1e-2, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8,
               weight_decay: float = 1e-2):
    """One AdamW update (Loshchilov & Hutter, decoupled weight decay), in
    place: the parameters shrink by lr * weight_decay times themselves, then
    take the Adam step; step counts from 1."""
    theta *= 1.0 - lr * weight_decay
    return adam_step(theta, m, v, g, step, lr, b1, b2, eps)
