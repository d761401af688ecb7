"""Pins of the FP64 oracle's processors against facts fixed by the paper's
definitions (Sec. 3) and by mathematics: closed forms, special cases, brute
force and finite differences.  CPU only."""
import math

import numpy as np
import pytest
import torch
from scipy.signal import lfilter

from oracle import processors as P

DT = torch.float64


def _sig(L=700, seed=0, stereo=True):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((2, L)) * 0.3
    if not stereo:
        x[1] = x[0]
    return torch.tensor(x, dtype=DT)


# ---------------------------------------------------------------- gain / imager / tanh
def test_gain_doubles_and_halves():
    u = _sig()
    y = P.gain_pan(u, torch.tensor([math.log(2.0), math.log(0.5)], dtype=DT))
    assert torch.allclose(y[0], 2.0 * u[0], rtol=1e-15, atol=0)
    assert torch.allclose(y[1], 0.5 * u[1], rtol=1e-15, atol=0)


def test_imager_identity_and_mono():
    u = _sig()
    assert torch.allclose(P.imager(u, torch.zeros(1, dtype=DT)), u, rtol=0, atol=1e-15)
    mono = _sig(stereo=False)
    for p in (-2.0, 0.7, 3.0):
        assert torch.allclose(P.imager(mono, torch.tensor([p], dtype=DT)), mono, atol=1e-15)
    # side removed entirely -> both channels carry the mid average
    y = P.imager(u, torch.tensor([-60.0], dtype=DT))
    avg = (u[0] + u[1]) / 2
    assert torch.allclose(y[0], avg, atol=1e-12) and torch.allclose(y[1], avg, atol=1e-12)


def test_tanh_symmetry_small_signal_and_saturation():
    p = torch.tensor([1.3, -0.4], dtype=DT)
    u = _sig()
    assert torch.allclose(P.tanh_dist(-u, p), -P.tanh_dist(u, p), atol=0)
    small = torch.full((2, 4), 1e-7, dtype=DT)
    ratio = P.tanh_dist(small, p) / small
    assert torch.allclose(ratio, torch.full_like(ratio, math.exp(0.9)), rtol=1e-12)
    big = torch.full((2, 4), 1e3, dtype=DT)
    assert torch.allclose(P.tanh_dist(big, p), torch.full_like(big, math.exp(-0.4)), rtol=1e-15)


# ---------------------------------------------------------------- equalizer
@pytest.mark.parametrize("N", [7, 39, 255, 1023])
def test_eq_fir_spectrum_is_hann_smoothed_response(N):
    """The DFT of the Hann-windowed FIR equals 1/2 H[k] + 1/4 H[k-1] + 1/4 H[k+1]
    (window multiplication = circular convolution of the sampled response)."""
    K = (N + 1) // 2
    rng = np.random.default_rng(N)
    p = torch.tensor(rng.normal(0, 0.7, K), dtype=DT)
    h = P.zero_phase_fir(p, N).numpy()
    half = (N - 1) // 2
    circ = np.zeros(N)
    for i, n in enumerate(range(-half, half + 1)):
        circ[n % N] = h[i]
    Hs = np.fft.fft(circ)
    Hk = np.exp(p.numpy())
    Hfull = np.concatenate([Hk, Hk[1:][::-1]])          # Hermitian-even extension
    expect = 0.5 * Hfull + 0.25 * np.roll(Hfull, 1) + 0.25 * np.roll(Hfull, -1)
    assert np.allclose(Hs.imag, 0, atol=1e-12)
    assert np.allclose(Hs.real, expect, rtol=1e-12, atol=1e-13)


def test_eq_flat_response_is_a_gain():
    u = _sig()
    y = P.equalizer(u, torch.full((128,), 0.3, dtype=DT), 255)
    assert torch.allclose(y, math.exp(0.3) * u, rtol=1e-10, atol=1e-12)


def test_eq_impulse_reproduces_centred_fir():
    N = 63
    p = torch.tensor(np.random.default_rng(3).normal(0, 1, 32), dtype=DT)
    u = torch.zeros(2, 300, dtype=DT)
    u[:, 150] = 1.0
    y = P.equalizer(u, p, N)
    h = P.zero_phase_fir(p, N)
    assert torch.allclose(y[0, 150 - 31:150 + 32], h, atol=1e-13)
    assert torch.allclose(y[0, :150 - 31], torch.zeros(150 - 31, dtype=DT), atol=1e-13)


@pytest.mark.parametrize("lag0", [-31, 0, 5])
def test_fir_conv_matches_direct_sum(lag0):
    rng = np.random.default_rng(lag0 + 100)
    x = rng.standard_normal((2, 257))
    h = rng.standard_normal((2, 63))
    y = P.fir_conv(torch.tensor(x), torch.tensor(h), lag0).numpy()
    L = x.shape[1]
    for c in range(2):
        ref = np.zeros(L)
        for n in range(L):
            s = 0.0
            for i in range(h.shape[1]):
                j = n - (i + lag0)
                if 0 <= j < L:
                    s += h[c, i] * x[c, j]
            ref[n] = s
        assert np.allclose(y[c], ref, atol=1e-11)


# ---------------------------------------------------------------- reverb
def test_reverb_unit_mask_reconstructs_noise():
    """With the mask at exp(0) for every bin and frame, the LS-ISTFT of the
    noise STFT is the noise itself (perfect reconstruction, Nyquist aside)."""
    fs, Lr = 16000, 2000
    rng = np.random.default_rng(1)
    noise = torch.tensor(rng.uniform(-1, 1, (2, Lr)), dtype=DT)
    p = torch.zeros(2, 2, 192, dtype=DT)
    p[:, 0] = -P.reverb_gain_bias(fs)
    p[:, 1] = -80.0                 # decay -softplus(-80 + beta) ~ -1e-35 per frame
    h = P.reverb_fir(p.reshape(-1), noise, fs)
    # removing the Nyquist bin removes the (-1)^n component of each frame;
    # compare against the noise with that component projected out per frame
    win = P.hann_periodic(384)
    nf, idx = P.centred_frames(Lr, 384, 192)
    ref = []
    for x in range(2):
        fr = torch.where((idx >= 0) & (idx < Lr), noise[x][idx.clamp(0, Lr - 1)], torch.zeros((), dtype=DT)) * win
        U = torch.fft.rfft(fr)
        U[:, 192] = 0
        s = torch.fft.irfft(U, n=384) * win
        acc = torch.zeros(Lr, dtype=DT)
        ws = torch.zeros(Lr, dtype=DT)
        keep = ((idx >= 0) & (idx < Lr)).reshape(-1)
        acc.index_add_(0, idx.reshape(-1)[keep], s.reshape(-1)[keep])
        ws.index_add_(0, idx.reshape(-1)[keep], (win ** 2).repeat(nf)[keep])
        ref.append(acc / ws)
    # and that projection only removes the alternating component
    assert torch.allclose(h[0], ref[0] + ref[1], atol=1e-12)
    assert torch.allclose(h[1], ref[0] - ref[1], atol=1e-12)
    assert float(torch.linalg.norm(ref[0] - noise[0]) / torch.linalg.norm(noise[0])) < 0.2


def test_reverb_unit_mask_on_bin_sinusoids_is_exact():
    """On-bin sinusoids (bins 3 and 40 of 384) have no Nyquist content in any
    Hann-windowed frame that lies fully inside the signal, so with a unit mask
    the LS-ISTFT returns them exactly wherever both covering frames are inside
    ([hop, Lr - hop) for Lr a multiple of hop)."""
    fs, Lr = 16000, 1536
    n = np.arange(Lr)
    sig = np.stack([np.sin(2 * np.pi * 3 * n / 384) + 0.3 * np.cos(2 * np.pi * 40 * n / 384 + 1),
                    np.cos(2 * np.pi * 7 * n / 384)])
    noise = torch.tensor(sig, dtype=DT)
    p = torch.zeros(2, 2, 192, dtype=DT)
    p[:, 0] = -P.reverb_gain_bias(fs)
    p[:, 1] = -80.0
    h = P.reverb_fir(p.reshape(-1), noise, fs)
    sl = slice(192, Lr - 192)
    assert torch.allclose(h[0, sl], (noise[0] + noise[1])[sl], atol=1e-12)
    assert torch.allclose(h[1, sl], (noise[0] - noise[1])[sl], atol=1e-12)


def test_stft_frames_match_explicit_dft():
    rng = np.random.default_rng(4)
    x = rng.uniform(-1, 1, 384)
    win = P.hann_periodic(384).numpy()
    k = np.arange(193)[:, None]
    t = np.arange(384)[None, :]
    Dm = np.exp(-2j * np.pi * ((k * t) % 384) / 384)
    ref = Dm @ (x * win)
    got = torch.fft.rfft(torch.tensor(x * win)).numpy()
    assert np.allclose(got, ref, atol=1e-11)


def test_reverb_decay_map():
    """theta = 0 gives the 0.5 s RT60 step; the step is always a decay and
    approaches 0 (no decay) for very negative theta."""
    fs, hop = 44100, 192
    d0 = float(P.reverb_decay(torch.tensor(0.0, dtype=DT), fs, hop))
    assert abs(d0 - (-6.91 * hop / (0.5 * fs))) < 1e-15
    th = torch.linspace(-40, 40, 101, dtype=DT)
    d = P.reverb_decay(th, fs, hop)
    assert bool((d < 0).all()) and bool((d[1:] < d[:-1]).all())


def test_reverb_output_is_causal_direct_convolution():
    fs = 8000
    rng = np.random.default_rng(2)
    noise = torch.tensor(rng.uniform(-1, 1, (2, 900)), dtype=DT)
    p = torch.tensor(rng.normal(0, 0.3, 768), dtype=DT)
    u = torch.tensor(rng.standard_normal((2, 400)), dtype=DT)
    y = P.reverb(u, p, noise, fs).numpy()
    h = P.reverb_fir(p, noise, fs).numpy()
    for c in range(2):
        ref = np.convolve(u[c].numpy(), h[c])[:400]
        assert np.allclose(y[c], ref, atol=1e-10)


# ---------------------------------------------------------------- compressor / gate
def _comp_params(alpha, T, W, R):
    return torch.tensor([math.log(alpha / (1 - alpha)), T, math.log(W), math.log(R - 1)], dtype=DT)


def test_compressor_constant_level_closed_form():
    a, alpha, T, W, R = 0.2, 0.97, math.log(0.01), 1.5, 4.0
    L = 400
    u = torch.full((2, L), a, dtype=DT)
    y, g = P.dynamics(u, _comp_params(alpha, T, W, R), gate=False, return_env=True)
    n = np.arange(L)
    g_ref = 4 * a * a * (1 - alpha ** (n + 1))
    assert np.allclose(g.numpy(), g_ref, rtol=1e-12)
    G = np.log(g_ref + P.COMP_EPS)
    Gy = np.where(G >= T + W, T + (G - T) / R,
                  np.where(G >= T - W, G + (1 / R - 1) * (G - T + W) ** 2 / (4 * W), G))
    assert np.allclose(y[0].numpy(), a * np.exp(Gy - G), rtol=1e-12)
    # tends to the static gain far above the knee
    Gs = math.log(4 * a * a + P.COMP_EPS)
    assert abs(float(y[0, -1]) / a - math.exp(T + (Gs - T) / R - Gs)) < 1e-6


def test_compressor_below_knee_is_identity():
    u = _sig() * 1e-3
    y = P.dynamics(u, _comp_params(0.9, math.log(1.0), 0.5, 5.0), gate=False)
    assert torch.allclose(y, u, rtol=1e-15, atol=0)


def test_gate_above_knee_identity_and_below_expansion():
    u = torch.full((2, 300), 0.3, dtype=DT)
    y = P.dynamics(u, _comp_params(0.5, math.log(1e-3), 0.2, 3.0), gate=True)
    assert torch.allclose(y[:, 20:], u[:, 20:], rtol=1e-14)
    q = torch.full((2, 300), 1e-4, dtype=DT)
    T, R = math.log(0.5), 3.0
    y, g = P.dynamics(q, _comp_params(0.5, T, 0.2, R), gate=True, return_env=True)
    G = torch.log(g + P.COMP_EPS)
    assert torch.allclose(y[0], q[0] * torch.exp((R - 1) * (G - T)), rtol=1e-12)


@pytest.mark.parametrize("gate", [False, True])
def test_curves_are_c1_at_knee_edges(gate):
    T, W, R = torch.tensor(-2.0, dtype=DT), torch.tensor(0.7, dtype=DT), torch.tensor(3.5, dtype=DT)
    f = P.gate_curve if gate else P.comp_curve
    for edge in (float(T - W), float(T + W)):
        for d in (1e-7,):
            lo = torch.tensor(edge - d, dtype=DT)
            hi = torch.tensor(edge + d, dtype=DT)
            assert abs(float(f(hi, T, W, R) - f(lo, T, W, R))) < 1e-6
            s_lo = (f(lo, T, W, R) - f(lo - 1e-5, T, W, R)) / 1e-5
            s_hi = (f(hi + 1e-5, T, W, R) - f(hi, T, W, R)) / 1e-5
            assert abs(float(s_hi - s_lo)) < 1e-4


def test_onepole_matches_loop_and_lfilter():
    rng = np.random.default_rng(5)
    e = rng.uniform(0, 1, 500)
    th = torch.tensor(1.7, dtype=DT)
    g = P.OnePole.apply(torch.tensor(e), th).numpy()
    a = 1 / (1 + math.exp(-1.7))
    ref = np.zeros_like(e)
    prev = 0.0
    for n in range(e.size):
        prev = a * prev + (1 - a) * e[n]
        ref[n] = prev
    assert np.allclose(g, ref, rtol=1e-13)
    assert np.allclose(lfilter([1 - a], [1, -a], e), ref, rtol=1e-13)


def test_attack_release_constant_input_uses_attack():
    a = 0.3
    u = torch.full((2, 200), a, dtype=DT)
    p = torch.tensor([math.log(0.8 / 0.2), math.log(0.99 / 0.01), 0.0, 0.0, 0.0], dtype=DT)
    _, g = P.dynamics(u, p, gate=False, attack_release=True, return_env=True)
    n = np.arange(200)
    assert np.allclose(g.numpy(), 4 * a * a * (1 - 0.8 ** (n + 1)), rtol=1e-12)


def test_attack_release_decay_uses_release():
    e_val = 0.25
    u = torch.zeros(2, 100, dtype=DT)
    u[:, 0] = e_val ** 0.5 / 2
    p = torch.tensor([math.log(0.5), math.log(0.9 / 0.1), 0.0, 0.0, 0.0], dtype=DT)
    _, g = P.dynamics(u, p, gate=False, attack_release=True, return_env=True)
    aa = 1 / (1 + 2.0)
    g0 = (1 - aa) * e_val
    assert abs(float(g[0]) - g0) < 1e-15
    assert np.allclose(g.numpy()[1:], g0 * 0.9 ** np.arange(1, 100), rtol=1e-12)


def test_recursion_adjoints_match_finite_differences():
    rng = np.random.default_rng(7)
    e = torch.tensor(rng.uniform(0, 1, 60), dtype=DT, requires_grad=True)
    th = torch.tensor(0.8, dtype=DT, requires_grad=True)
    assert torch.autograd.gradcheck(P.OnePole.apply, (e, th), eps=1e-6, atol=1e-8)
    # attack/release: away from ties the branch pattern is stable under the probe
    e2 = torch.tensor(np.abs(np.sin(np.arange(60) * 0.7)) + 0.05, dtype=DT, requires_grad=True)
    ta = torch.tensor(0.3, dtype=DT, requires_grad=True)
    tr = torch.tensor(2.0, dtype=DT, requires_grad=True)
    assert torch.autograd.gradcheck(P.AttackRelease.apply, (e2, ta, tr), eps=1e-7, atol=1e-7)


# ---------------------------------------------------------------- multitap delay
def test_delay_index_of_on_bin_angles():
    D = 400
    for d in (0, 1, 17, 199, 200, 399):
        z = complex(math.cos(-2 * math.pi * d / D), math.sin(-2 * math.pi * d / D))
        assert P.delay_index(z.real, z.imag, D) == d


def test_single_flat_tap_is_a_pure_shift():
    M, D, taps = 3, 200, 39
    Kc = 20
    p = np.zeros((2, M, 2 + Kc))
    p[:, :, 2:] = -800.0                    # taps switched off
    d = [(1, 37), (2, 150)]                 # (tap, in-range delay) per channel
    for c, (m, dd) in enumerate(d):
        ang = -2 * math.pi * dd / D
        p[c, :, 0], p[c, :, 1] = 1.0, 0.0
        p[c, m, 0], p[c, m, 1] = math.cos(ang), math.sin(ang)
        p[c, m, 2:] = 0.0                   # flat 39-tap FIR = unit impulse
    u = _sig(L=900)
    y = P.delay(u, torch.tensor(p.reshape(-1)), M, D, taps)
    for c, (m, dd) in enumerate(d):
        s = m * D + dd
        assert torch.allclose(y[c, s:], u[c, :900 - s], atol=1e-12)
        assert torch.allclose(y[c, :s], torch.zeros(s, dtype=DT), atol=1e-12)


def test_surrogate_on_bin_is_exact_delta():
    D = 128
    for d in (0, 5, 64, 127):
        z = complex(math.cos(-2 * math.pi * d / D), math.sin(-2 * math.pi * d / D))
        zk = np.exp(np.arange(D) * np.log(z))
        s = np.fft.ifft(zk).real
        ref = np.zeros(D)
        ref[d] = 1.0
        assert np.allclose(s, ref, atol=1e-12)


def test_surrogate_gradient_matches_finite_difference_of_surrogate():
    """The z-gradient the oracle produces is the derivative of the surrogate
    FIR (value path replaced by the surrogate), checked by central FD."""
    M, D, taps = 2, 64, 7
    Kc = 4
    rng = np.random.default_rng(9)
    p0 = rng.normal(0, 0.5, (2, M, 2 + Kc))
    p0[:, :, 0:2] *= 0.6
    u = _sig(L=300, seed=3)
    gw = torch.tensor(rng.standard_normal((2, 300)), dtype=DT)

    def sur_loss(pv):
        # surrogate-only FIR: h_sur built exactly as delay_fir does
        h, lag0 = P.delay_fir(pv, M, D, taps, surrogate=True)
        return h

    p = torch.tensor(p0.reshape(-1), dtype=DT, requires_grad=True)
    h, lag0 = P.delay_fir(p, M, D, taps, surrogate=True)
    y = P.fir_conv(u, h, lag0)
    (y * gw).sum().backward()
    g = p.grad.view(2, M, 2 + Kc)

    def value(pp):
        # evaluate the surrogate FIR value directly (the ST value is the exact
        # FIR, so rebuild the surrogate part by hand for the FD probe)
        pv = pp.view(2, M, 2 + Kc)
        out = torch.zeros(2, M * D + taps - 1, dtype=DT)
        k = torch.arange(D, dtype=DT)
        for c in range(2):
            for m in range(M):
                cm = P.zero_phase_fir(torch.tensor(p0[c, m, 2:]), taps)
                z = complex(float(pv[c, m, 0]), float(pv[c, m, 1]))
                dsur = np.fft.ifft(np.exp(np.arange(D) * np.log(z))).real
                seg = np.convolve(dsur, cm.numpy())
                out[c, m * D:m * D + D + taps - 1] += torch.tensor(seg)
        return float((P.fir_conv(u, out, lag0) * gw).sum())

    for c in range(2):
        for m in range(M):
            for j in range(2):
                pp = torch.tensor(p0.reshape(-1), dtype=DT)
                idx = (c * M + m) * (2 + Kc) + j
                e = 1e-6
                pp[idx] += e
                fp = value(pp)
                pp[idx] -= 2 * e
                fm = value(pp)
                fd = (fp - fm) / (2 * e)
                assert abs(fd - float(g[c, m, j])) <= 1e-6 * max(1.0, abs(fd)), (c, m, j, fd, float(g[c, m, j]))


def test_delay_grad_rule_properties():
    r, i = P.delay_grad_rule(3.0, 4.0, 0.0, 0.0)
    assert (r, i) == (0.6, 0.8)
    r, i = P.delay_grad_rule(0.0, 0.0, 0.5, 0.0, gamma=0.01)
    assert abs(r - 0.01 * (0.5 - 1.0)) < 1e-15 and i == 0.0


def test_reverb_frame_decay_closed_form():
    """An on-bin sinusoid with a per-frame log-decay delta: frame m carries
    exp(c + m*delta) x, so the LS overlap-add gives, at n = q*hop + r,
    x[n] e^c (w2[r+hop] e^{q delta} + w2[r] e^{(q+1) delta}) / (w2[r+hop] + w2[r])."""
    fs, Lr, hop = 16000, 1536, 192
    c0, delta = 0.4, -0.05
    n = np.arange(Lr)
    x = np.sin(2 * np.pi * 5 * n / 384)
    noise = torch.tensor(np.stack([x, np.zeros(Lr)]), dtype=DT)
    p = torch.zeros(2, 2, 192, dtype=DT)
    p[:, 0] = c0 - P.reverb_gain_bias(fs)
    # raw decay that maps to delta: softplus(theta + beta) = -delta
    p[:, 1] = math.log(math.expm1(-delta)) - P.reverb_decay_offset(fs, hop)
    h = P.reverb_fir(p.reshape(-1), noise, fs).numpy()
    w2 = P.hann_periodic(384).numpy() ** 2
    q, r = n // hop, n % hop
    ref = x * np.exp(c0) * (w2[r + hop] * np.exp(q * delta) + w2[r] * np.exp((q + 1) * delta)) / (w2[r + hop] + w2[r])
    sl = slice(hop, Lr - hop)
    assert np.allclose(h[0, sl], ref[sl], atol=1e-12)
    assert np.allclose(h[1, sl], ref[sl], atol=1e-12)


def test_reverb_gain_bias_gives_unit_energy_at_zero_parameters():
    """At raw parameters 0 the mid and side FIRs of the reverb (Sec. 3.4) have
    unit energy on average: U(-1, 1) noise has variance 1/3, the decay at 0 is
    6.91 nepers per 0.5 s, so the energy sums to (1/3) e^{2 g0} 0.5 fs / 13.82,
    which the gain bias g0 sets to 1.  Statistical pin over 6 noise draws at
    44.1 kHz (about 1 % standard error on the mean); the Nyquist bin and the
    frame-wise gain interpolation move it by well under 1 %."""
    fs = 44100
    Lr = int(1.5 * fs)
    p = torch.zeros(768, dtype=DT)
    energies = []
    for seed in range(6):
        rng = np.random.default_rng(100 + seed)
        noise = torch.tensor(rng.uniform(-1, 1, (2, Lr)), dtype=DT)
        h = P.reverb_fir(p, noise, fs)
        hm, hs = 0.5 * (h[0] + h[1]), 0.5 * (h[0] - h[1])
        energies += [float(torch.sum(hm * hm)), float(torch.sum(hs * hs))]
    mean = float(np.mean(energies))
    assert abs(mean - 1.0) < 0.04, energies
    # a bias of the other sign (or none) is far off
    assert abs(math.exp(-2 * P.reverb_gain_bias(fs)) - 1.0) > 10
