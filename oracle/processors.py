"""FP64 reference processors (paper Sec. 3).  Test infrastructure only.

Audio is a torch float64 tensor of shape [2, L] (left, right).  Parameters are
the raw vectors of one node; the maps from raw values to physical quantities
are stated per processor.  Every function is differentiable with torch
autograd; the two recursions of the compressor carry hand-written adjoints
(checked against central finite differences in the tests).
"""
from __future__ import annotations

import functools
import math

import numpy as np
import torch
from scipy.signal import lfilter

DT = torch.float64
COMP_EPS = 1e-8          # epsilon inside the log of the energy envelope


# ---------------------------------------------------------------------------
# Sec. 3 preamble: dry/wet mix  y = w * ybar + (1 - w) * u
# ---------------------------------------------------------------------------
def dry_wet(ybar: torch.Tensor, u: torch.Tensor, w: torch.Tensor) -> torch.Tensor:
    return w * ybar + (1.0 - w) * u


# ---------------------------------------------------------------------------
# Sec. 3.1 gain/panning: one log-gain per channel
# ---------------------------------------------------------------------------
def gain_pan(u: torch.Tensor, p: torch.Tensor) -> torch.Tensor:
    return torch.exp(p).unsqueeze(1) * u


# ---------------------------------------------------------------------------
# Sec. 3.2 stereo imager: side channel scaled by exp(p)
# ---------------------------------------------------------------------------
def imager(u: torch.Tensor, p: torch.Tensor) -> torch.Tensor:
    ym = u[0] + u[1]
    ys = torch.exp(p[0]) * (u[0] - u[1])
    return torch.stack([(ym + ys) / 2.0, (ym - ys) / 2.0])


# ---------------------------------------------------------------------------
# tanh waveshaper of the benchmark processor set (not in the paper):
#   ybar = exp(p_out) * tanh(exp(p_in) * u)
# ---------------------------------------------------------------------------
def tanh_dist(u: torch.Tensor, p: torch.Tensor) -> torch.Tensor:
    return torch.exp(p[1]) * torch.tanh(torch.exp(p[0]) * u)


# ---------------------------------------------------------------------------
# Sec. 3.3 equalizer: zero-phase FIR from log-magnitudes
# ---------------------------------------------------------------------------
@functools.lru_cache(maxsize=8)
def _cos_table(N: int) -> torch.Tensor:
    """cos(2 pi k n / N) for k = 1..K-1 and n = -(N-1)/2..(N-1)/2, with the
    angle reduced exactly as ((k*n) mod N) before scaling."""
    K = (N + 1) // 2
    half = (N - 1) // 2
    k = np.arange(1, K, dtype=np.int64)[:, None]
    n = np.arange(-half, half + 1, dtype=np.int64)[None, :]
    r = np.mod(k * n, N).astype(np.float64)
    return torch.from_numpy(np.cos(2.0 * math.pi * r / N))


def zero_phase_fir(p: torch.Tensor, N: int) -> torch.Tensor:
    """Length-N zero-phase FIR (N odd) from K = (N+1)/2 log-magnitudes.

    H[k] = exp(p[k]) extended Hermitian-even (H[N-k] = H[k]); the inverse DFT
    is h0[n] = (H[0] + 2 sum_{k>=1} H[k] cos(2 pi k n / N)) / N over the centred
    index range n = -(N-1)/2..(N-1)/2, windowed by the centred Hann
    v[n] = cos^2(pi n / N).  Element i of the result is tap n = i - (N-1)/2."""
    K = (N + 1) // 2
    assert p.numel() == K, (p.numel(), K)
    H = torch.exp(p)
    h0 = (H[0] + 2.0 * (H[1:, None] * _cos_table(N)).sum(0)) / N
    half = (N - 1) // 2
    n = torch.arange(-half, half + 1, dtype=DT)
    v = torch.cos(math.pi * n / N) ** 2
    return v * h0


def fir_conv(x: torch.Tensor, h: torch.Tensor, lag0: int) -> torch.Tensor:
    """y[c, n] = sum_i h[c, i] * x[c, n - (i + lag0)] for n in [0, L), with x = 0
    outside [0, L).  h has shape [C, Nh] or [1, Nh] (shared by the channels).
    Computed as a zero-padded FFT product (a library primitive), which equals
    the direct sum exactly up to rounding."""
    C, L = x.shape
    Nh = h.shape[-1]
    M = L + Nh - 1
    nfft = 1 << (M - 1).bit_length()
    c = torch.fft.irfft(torch.fft.rfft(x, n=nfft) * torch.fft.rfft(h, n=nfft), n=nfft)[..., :M]
    if lag0 <= 0:
        return c[..., -lag0:-lag0 + L]
    return torch.cat([torch.zeros(c.shape[0], lag0, dtype=c.dtype), c[..., :L - lag0]], dim=-1)


def equalizer(u: torch.Tensor, p: torch.Tensor, N: int) -> torch.Tensor:
    """Sec. 3.3: the same zero-phase FIR on both channels, centred ("same")
    convolution with no latency."""
    h = zero_phase_fir(p, N)
    return fir_conv(u, h.unsqueeze(0), -((N - 1) // 2))


# ---------------------------------------------------------------------------
# Sec. 3.4 reverb: filtered-noise stereo FIR
# ---------------------------------------------------------------------------
def hann_periodic(N: int) -> torch.Tensor:
    n = torch.arange(N, dtype=DT)
    return 0.5 - 0.5 * torch.cos(2.0 * math.pi * n / N)


def reverb_decay_offset(fs: int, hop: int) -> float:
    """Offset beta of the decay map: softplus(beta) equals the per-frame
    log-magnitude decay of a 0.5 s RT60 (-60 dB = log(1e-3) = -6.91)."""
    return math.log(math.expm1(6.91 * hop / (0.5 * fs)))


def reverb_decay(theta_d: torch.Tensor, fs: int, hop: int) -> torch.Tensor:
    """Per-frame log-magnitude step of the reverb mask from the raw decay
    parameter: -softplus(theta + beta) (always a decay; 0.5 s RT60 at 0)."""
    return -torch.nn.functional.softplus(theta_d + reverb_decay_offset(fs, hop))


def reverb_gain_bias(fs: int) -> float:
    """Log-magnitude added to the learnable initial colouration so that raw
    parameters near 0 give a unit-energy FIR: U(-1, 1) noise has variance 1/3,
    and an exponential decay of 6.91 nepers per 0.5 s sums to 0.5 fs / (2 * 6.91)
    samples of unit energy, so the bias is -0.5 log(0.5 fs / (6 * 6.91))."""
    return -0.5 * math.log(0.5 * fs / (6.0 * 6.91))


def centred_frames(Lr: int, nfft: int, hop: int):
    """Frame m covers samples [m*hop - nfft/2, m*hop + nfft/2); frames
    m = 0 .. floor((Lr-1)/hop) + 1 cover every sample of [0, Lr) twice."""
    nf = (Lr - 1) // hop + 2
    start = torch.arange(nf) * hop - nfft // 2
    idx = start[:, None] + torch.arange(nfft)[None, :]
    return nf, idx


def reverb_fir(p: torch.Tensor, noise: torch.Tensor, fs: int, nfft: int = 384,
               hop: int = 192) -> torch.Tensor:
    """Stereo reverb FIR [2, Lr] (Sec. 3.4).

    For x in (mid, side): U_x = STFT of the fixed noise (periodic Hann, centred
    frames, zero padding), mask M_x[k, m] = exp(H0[k] + g0 + m * d[k]) with the decay
    d[k] = -softplus(Hd[k] + beta) (reverb_decay), for the
    nfft/2 bins below Nyquist (the Nyquist bin is 0), h_x = least-squares ISTFT
    of U_x * M_x.  Then h_l = h_m + h_s and h_r = h_m - h_s.  The gain bias g0
    (added to H0) is reverb_gain_bias."""
    nb = nfft // 2
    Lr = noise.shape[-1]
    pv = p.view(2, 2, nb)
    win = hann_periodic(nfft)
    nf, idx = centred_frames(Lr, nfft, hop)
    valid = (idx >= 0) & (idx < Lr)
    safe = idx.clamp(0, Lr - 1)
    gbias = reverb_gain_bias(fs)
    m = torch.arange(nf, dtype=DT)[:, None]
    flat = idx.reshape(-1)
    keep = valid.reshape(-1)
    wsum = torch.zeros(Lr, dtype=DT)
    wsum.index_add_(0, flat[keep], (win ** 2).repeat(nf)[keep])
    hs = []
    for x in range(2):
        frames = torch.where(valid, noise[x][safe], torch.zeros((), dtype=DT)) * win
        U = torch.fft.rfft(frames, dim=-1)                         # [nf, nb+1]
        mask = torch.exp(pv[x, 0][None, :] + gbias + m * reverb_decay(pv[x, 1], fs, hop)[None, :])
        Hm = torch.cat([U[:, :nb] * mask, torch.zeros(nf, 1, dtype=U.dtype)], dim=1)
        s = torch.fft.irfft(Hm, n=nfft, dim=-1) * win              # [nf, nfft]
        h = torch.zeros(Lr, dtype=DT)
        h = h.index_add(0, flat[keep], s.reshape(-1)[keep])
        hs.append(h / wsum)
    hm, hsd = hs
    return torch.stack([hm + hsd, hm - hsd])


def reverb(u: torch.Tensor, p: torch.Tensor, noise: torch.Tensor, fs: int) -> torch.Tensor:
    """Channel-wise causal convolution with the stereo FIR (Sec. 3.4)."""
    h = reverb_fir(p, noise, fs)
    return fir_conv(u, h, 0)


# ---------------------------------------------------------------------------
# Sec. 3.5 compressor / Sec. 3.6 noisegate
# ---------------------------------------------------------------------------
class OnePole(torch.autograd.Function):
    """Energy ballistics with one coefficient (Sec. 3.5, eq. envelope):
    g[n] = a g[n-1] + (1 - a) e[n], g[-1] = 0, a = sigmoid(theta),
    1 - a = sigmoid(-theta).  The exact recursion (no truncation).
    Forward uses scipy.signal.lfilter; the adjoint is the reverse recursion."""

    @staticmethod
    def forward(ctx, e, theta):
        a = torch.sigmoid(theta).item()
        b = torch.sigmoid(-theta).item()
        g = torch.from_numpy(lfilter([b], [1.0, -a], e.detach().numpy()))
        ctx.save_for_backward(e, g, theta)
        ctx.ab = (a, b)
        return g

    @staticmethod
    def backward(ctx, gg):
        e, g, theta = ctx.saved_tensors
        a, b = ctx.ab
        lam = lfilter([1.0], [1.0, -a], gg.numpy()[::-1])[::-1].copy()
        lam = torch.from_numpy(lam)
        gprev = torch.cat([torch.zeros(1, dtype=DT), g[:-1]])
        dtheta = a * b * torch.sum(lam * (gprev - e))
        return b * lam, dtheta.reshape(theta.shape)


class AttackRelease(torch.autograd.Function):
    """Two-coefficient ballistics (Sec. 3.5): a[n] = a_att when e[n] > g[n-1]
    (the envelope rises), else a_rel; g[n] = a[n] g[n-1] + (1 - a[n]) e[n].
    Plain sequential loop.  The branch is piecewise constant, so the adjoint
    is the reverse recursion with the recorded a[n]."""

    @staticmethod
    def forward(ctx, e, th_att, th_rel):
        aa, ba = torch.sigmoid(th_att).item(), torch.sigmoid(-th_att).item()
        ar, br = torch.sigmoid(th_rel).item(), torch.sigmoid(-th_rel).item()
        ev = e.detach().numpy().tolist()
        g = [0.0] * len(ev)
        att = [False] * len(ev)
        prev = 0.0
        for n, en in enumerate(ev):
            if en > prev:
                prev = aa * prev + ba * en
                att[n] = True
            else:
                prev = ar * prev + br * en
            g[n] = prev
        g = torch.tensor(g, dtype=DT)
        ctx.save_for_backward(e, g, th_att, th_rel)
        ctx.att = att
        ctx.coef = (aa, ba, ar, br)
        return g

    @staticmethod
    def backward(ctx, gg):
        e, g, th_att, th_rel = ctx.saved_tensors
        aa, ba, ar, br = ctx.coef
        att = ctx.att
        gv = gg.numpy().tolist()
        ev = e.detach().numpy().tolist()
        gl = g.numpy().tolist()
        L = len(gv)
        de = [0.0] * L
        lam_next = 0.0
        a_next = 0.0
        s_att = 0.0
        s_rel = 0.0
        for n in range(L - 1, -1, -1):
            lam = gv[n] + a_next * lam_next
            gp = gl[n - 1] if n > 0 else 0.0
            if att[n]:
                de[n] = ba * lam
                s_att += lam * (gp - ev[n])
                a_next = aa
            else:
                de[n] = br * lam
                s_rel += lam * (gp - ev[n])
                a_next = ar
            lam_next = lam
        d_att = torch.tensor(aa * ba * s_att, dtype=DT).reshape(th_att.shape)
        d_rel = torch.tensor(ar * br * s_rel, dtype=DT).reshape(th_rel.shape)
        return torch.tensor(de, dtype=DT), d_att, d_rel


def comp_curve(G, T, W, R):
    """Quadratic-knee compressor curve (Sec. 3.5)."""
    above = T + (G - T) / R
    mid = G + (1.0 / R - 1.0) * (G - T + W) ** 2 / (4.0 * W)
    return torch.where(G >= T + W, above, torch.where(G >= T - W, mid, G))


def gate_curve(G, T, W, R):
    """Noisegate curve (Sec. 3.6): identity above the knee, expansion below."""
    mid = G + (1.0 - R) * (G - T - W) ** 2 / (4.0 * W)
    below = T + R * (G - T)
    return torch.where(G >= T + W, G, torch.where(G >= T - W, mid, below))


def dynamics(u: torch.Tensor, p: torch.Tensor, gate: bool, attack_release: bool = False,
             return_env: bool = False):
    """Compressor (gate=False) or noisegate (gate=True), Sec. 3.5-3.6.

    Raw parameters: [theta_alpha, T, log W, log(R - 1)] (single coefficient) or
    [theta_att, theta_rel, T, log W, log(R - 1)] (attack/release).  T and G are
    natural logs of the energy of the mid signal u_l + u_r."""
    um = u[0] + u[1]
    e = um * um
    if attack_release:
        g = AttackRelease.apply(e, p[0], p[1])
        q = p[2:]
    else:
        g = OnePole.apply(e, p[0])
        q = p[1:]
    T = q[0]
    W = torch.exp(q[1])
    R = 1.0 + torch.exp(q[2])
    G = torch.log(g + COMP_EPS)
    Gy = gate_curve(G, T, W, R) if gate else comp_curve(G, T, W, R)
    ybar = torch.exp(Gy - G).unsqueeze(0) * u
    return (ybar, g) if return_env else ybar


# ---------------------------------------------------------------------------
# Sec. 3.7 multitap delay
# ---------------------------------------------------------------------------
def delay_layout(p: torch.Tensor, M: int, Kc: int):
    """Raw vector -> [2 channels, M taps, 2 + Kc] (Re z, Im z, Kc log-mags)."""
    return p.view(2, M, 2 + Kc)


def delay_index(zr: float, zi: float, D: int) -> int:
    """Integer delay within a tap range from the angle of z:
    z = exp(-j 2 pi d / D)  <=>  d = round(-arg(z) D / (2 pi)) mod D,
    rounding half up."""
    phi = math.atan2(zi, zr)
    return int(math.floor(-phi * D / (2.0 * math.pi) + 0.5)) % D


def delay_fir(p: torch.Tensor, M: int, D: int, taps: int, surrogate: bool = True):
    """Per-channel multitap FIR h_d = sum_m c_m * delta[n - d_m] (Sec. 3.7),
    support [-(taps-1)/2, M*D + (taps-1)/2), returned as ([2, M*D + taps - 1],
    lag0 = -(taps-1)/2).  Tap m (0-based) delays by d_m = m*D + d'_m.

    With surrogate=True the result carries the straight-through gradient of
    Sec. 3.7: its value is the exact integer-delay FIR, its derivative with
    respect to z_m is that of the surrogate in which delta[q - d'_m], q in
    [0, D), is replaced by Re{(1/D) sum_k z_m^k exp(j 2 pi k q / D)} (placed at
    offset m*D and convolved with a detached c_m)."""
    Kc = (taps + 1) // 2
    half = (taps - 1) // 2
    pv = delay_layout(p, M, Kc)
    Lh = M * D + taps - 1
    h_exact = torch.zeros(2, Lh, dtype=DT)
    h_sur = torch.zeros(2, Lh, dtype=DT)
    k = torch.arange(D, dtype=DT)
    for c in range(2):
        for m in range(M):
            cm = zero_phase_fir(pv[c, m, 2:], taps)
            d = m * D + delay_index(pv[c, m, 0].item(), pv[c, m, 1].item(), D)
            # index of tap n is n + half (lag0 = -half)
            h_exact = h_exact.index_put((torch.tensor([c]).repeat(taps),
                                         torch.arange(taps) + d), cm, accumulate=True)
            if surrogate:
                z = torch.complex(pv[c, m, 0], pv[c, m, 1])
                zk = torch.exp(k * torch.log(z))
                dsur = torch.fft.ifft(zk).real                       # [D]
                seg = torch.nn.functional.conv1d(
                    dsur.view(1, 1, -1), cm.detach().flip(0).view(1, 1, -1),
                    padding=taps - 1).view(-1)                      # [D + taps - 1]
                h_sur = h_sur.index_put((torch.tensor([c]).repeat(D + taps - 1),
                                         torch.arange(D + taps - 1) + m * D), seg,
                                        accumulate=True)
    if surrogate:
        h = h_exact + (h_sur - h_sur.detach())
    else:
        h = h_exact
    return h, -half


def delay(u: torch.Tensor, p: torch.Tensor, M: int, D: int, taps: int) -> torch.Tensor:
    h, lag0 = delay_fir(p, M, D, taps)
    return fir_conv(u, h, lag0)


def delay_grad_rule(g_re: float, g_im: float, z_re: float, z_im: float, gamma: float = 0.01):
    """Sec. 3.7 gradient rule for one tap: the surrogate gradient g (as the
    complex number dL/dRe z + j dL/dIm z) is replaced by
    g/|g| + gamma (|z| - 1) z/|z|, with sgn(0) = 0.  Returns (re, im)."""
    ag = math.hypot(g_re, g_im)
    az = math.hypot(z_re, z_im)
    sr, si = (g_re / ag, g_im / ag) if ag > 0 else (0.0, 0.0)
    if az > 0:
        sr += gamma * (az - 1.0) * z_re / az
        si += gamma * (az - 1.0) * z_im / az
    return sr, si
