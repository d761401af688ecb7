"""Marshalling of synthetic workloads (the ``synth`` input module) into the
binding: graph + configuration, per-node parameters -> flat device vectors,
reverb noise rows, masks.  No arithmetic of the method lives here."""
from __future__ import annotations

from typing import Dict

import numpy as np

from . import mixgraph as MG


def binding_config(cfg, alpha_g: float = 1e-3, alpha_p: float = 0.0, loss_skip: int = 0, max_trials: int = 0,
                   trial_slots: int = 0, unfused: bool = False) -> MG.mg_config:
    return MG.make_config(length=cfg.length, sample_rate=cfg.fs, eq_taps=cfg.eq_taps,
                          comp_mode=1 if cfg.comp_mode == "attack_release" else 0,
                          delay_taps=cfg.delay_taps, delay_range=cfg.delay_range,
                          delay_fir_taps=cfg.delay_fir_taps, reverb_length=cfg.reverb_length,
                          reverb_nfft=cfg.reverb_nfft, reverb_hop=cfg.reverb_hop, loss_ffts=cfg.loss_ffts,
                          n_mels=cfg.n_mels, loss_skip=loss_skip, alpha_g=alpha_g, alpha_p=alpha_p,
                          max_trials=max_trials, trial_slots=trial_slots, unfused=int(unfused))


def binding_graph(graph, cfg, alpha_g: float = 1e-3, alpha_p: float = 0.0, max_trials: int = 0,
                  trial_slots: int = 0, unfused: bool = False) -> MG.Graph:
    input_track = [graph.track_of_input.get(v, -1) for v in range(graph.n_nodes)]
    return MG.Graph(graph.types, graph.edge_array(), input_track, cfg.n_tracks,
                    2 if cfg.stereo_tracks else 1,
                    binding_config(cfg, alpha_g, alpha_p, max_trials=max_trials, trial_slots=trial_slots,
                                   unfused=unfused))


def noise_rows(g: MG.Graph, noise: Dict[int, np.ndarray], Lr: int) -> np.ndarray:
    rows = g.reverb_rows()
    if not rows:
        return np.zeros((1, 2, max(Lr, 1)), np.float32)
    return np.stack([noise[v] for v in rows]).astype(np.float32)
