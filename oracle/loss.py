"""FP64 multi-resolution STFT loss (paper Sec. 5.1).  Test infrastructure only.

L_a = 0.5 L_lr + 0.25 L_m + 0.25 L_s, each term a sum over FFT resolutions of
[ mean |log Y - log Yhat| + ||Y - Yhat||_F / ||Y||_F ] on 96-band Mel
spectrograms of A-weighted magnitude STFTs.  Readings where the paper is
silent: HTK Mel scale with unit-peak triangles over [0, fs/2]; IEC 61672
analog A-weighting applied as a per-bin magnitude weight (normalised to 0 dB
at 1 kHz); natural log with LOG_EPS; the l1 term averaged over all
(frame, band) cells; frames fully inside [skip, L) with a periodic Hann
window; mid = l + r and side = l - r formed from the spectra; the l/r term is
the mean of the left and right terms.
"""
from __future__ import annotations

import math

import numpy as np
import torch

DT = torch.float64
LOG_EPS = 1e-7
SC_EPS = 1e-12
WEIGHTS = {"lr": 0.5, "m": 0.25, "s": 0.25}


def hz_to_mel(f):
    return 2595.0 * np.log10(1.0 + np.asarray(f, dtype=np.float64) / 700.0)


def mel_to_hz(m):
    return 700.0 * (10.0 ** (np.asarray(m, dtype=np.float64) / 2595.0) - 1.0)


def mel_filterbank(n_fft: int, fs: int, n_mels: int = 96) -> np.ndarray:
    """[n_mels, n_fft/2 + 1] triangles with peak 1, band b spanning the Mel
    points b, b+1 (peak), b+2 of n_mels + 2 points equally spaced in Mel."""
    pts = mel_to_hz(np.linspace(0.0, hz_to_mel(fs / 2.0), n_mels + 2))
    f = np.arange(n_fft // 2 + 1) * fs / n_fft
    fb = np.zeros((n_mels, f.size))
    for b in range(n_mels):
        lo, c, hi = pts[b], pts[b + 1], pts[b + 2]
        up = (f - lo) / (c - lo)
        down = (hi - f) / (hi - c)
        fb[b] = np.maximum(0.0, np.minimum(up, down))
    return fb


def a_weighting_mag(f) -> np.ndarray:
    """IEC 61672 analog A-weighting magnitude, 1.0 at 1 kHz."""
    def ra(x):
        x2 = np.asarray(x, dtype=np.float64) ** 2
        return (12194.0 ** 2 * x2 * x2) / ((x2 + 20.6 ** 2)
                                           * np.sqrt((x2 + 107.7 ** 2) * (x2 + 737.9 ** 2))
                                           * (x2 + 12194.0 ** 2))
    return ra(f) / ra(1000.0)


def _frames(x: torch.Tensor, n_fft: int, hop: int, skip: int) -> torch.Tensor:
    L = x.shape[-1]
    F = 1 + (L - skip - n_fft) // hop
    idx = skip + torch.arange(F)[:, None] * hop + torch.arange(n_fft)[None, :]
    return x[..., idx]


def mel_spectra(x: torch.Tensor, n_fft: int, fs: int, n_mels: int = 96, skip: int = 0):
    """Mel magnitudes of the four combos (l, r, m, s), each [F, n_mels]."""
    hop = n_fft // 4
    n = torch.arange(n_fft, dtype=DT)
    win = 0.5 - 0.5 * torch.cos(2.0 * math.pi * n / n_fft)
    X = torch.fft.rfft(_frames(x, n_fft, hop, skip) * win, dim=-1)   # [2, F, nb]
    Aw = torch.from_numpy(a_weighting_mag(np.arange(n_fft // 2 + 1) * fs / n_fft))
    fb = torch.from_numpy(mel_filterbank(n_fft, fs, n_mels))
    combos = {"l": X[0], "r": X[1], "m": X[0] + X[1], "s": X[0] - X[1]}
    return {k: (v.abs() * Aw) @ fb.T for k, v in combos.items()}


def mrstft(yhat: torch.Tensor, y: torch.Tensor, ffts, fs: int, n_mels: int = 96, skip: int = 0):
    """Returns dict La, Llr, Lm, Ls (torch scalars) plus per-term details."""
    terms = {k: torch.zeros((), dtype=DT) for k in "lrms"}
    for n_fft in ffts:
        Yh = mel_spectra(yhat, n_fft, fs, n_mels, skip)
        with torch.no_grad():
            Yt = mel_spectra(y, n_fft, fs, n_mels, skip)
        for k in "lrms":
            lm = torch.mean(torch.abs(torch.log(Yt[k] + LOG_EPS) - torch.log(Yh[k] + LOG_EPS)))
            sc = torch.linalg.norm(Yt[k] - Yh[k]) / (torch.linalg.norm(Yt[k]) + SC_EPS)
            terms[k] = terms[k] + lm + sc
    Llr = 0.5 * (terms["l"] + terms["r"])
    Lm, Ls = terms["m"], terms["s"]
    La = WEIGHTS["lr"] * Llr + WEIGHTS["m"] * Lm + WEIGHTS["s"] * Ls
    return {"La": La, "Llr": Llr, "Lm": Lm, "Ls": Ls}
