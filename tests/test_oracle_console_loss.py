"""Pins of the oracle's console evaluation, MRSTFT loss, gradients and Adam
(Sec. 3 preamble, Sec. 4.1, Sec. 5.1, Sec. 6): closed forms, brute force and
central finite differences.  CPU only."""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import console as C
from oracle import loss as LS
from oracle import processors as P
from oracle import train as TR

DT = torch.float64


def _small(chain="ecxsgdr", seconds=0.3, **kw):
    cfg = synth.small_config(seconds=seconds, chain=chain, **kw)
    g, dry, noise = synth.song(3, cfg)
    return cfg, g, dry, noise


# ---------------------------------------------------------------- console
def test_all_dry_weights_zero_gives_sum_of_sources():
    """w = 0 everywhere is the 'base graph' that sums the inputs (Sec. 5.3)."""
    cfg, g, dry, noise = _small()
    th, we = synth.random_params(3, g, cfg)
    mask = {v: 0.0 for v in g.processors()}
    mix = TR.render(g, cfg, dry, noise, th, we, mask)
    ref = dry.astype(np.float64).sum(0)
    assert np.array_equal(mix, ref) or np.allclose(mix, ref, rtol=0, atol=1e-15)


def test_mono_tracks_are_duplicated():
    cfg = synth.small_config(seconds=0.2, chain="g", stereo_tracks=False)
    g, dry, noise = synth.song(4, cfg)
    assert dry.shape[1] == 1
    mix = TR.render(g, cfg, dry, noise, {v: np.zeros(2) for v in g.processors()},
                    {v: 0.0 for v in g.processors()})
    assert np.allclose(mix[0], mix[1], rtol=0, atol=0)
    assert np.allclose(mix[0], dry[:, 0].astype(np.float64).sum(0), atol=1e-15)


def test_gain_only_console_by_hand():
    """A two-level console of gain/pan processors computed by hand."""
    cfg = synth.small_config(seconds=0.1, chain="g", n_tracks=3, n_subgroups=2)
    g, dry, noise = synth.song(8, cfg)
    rng = np.random.default_rng(0)
    th = {v: rng.normal(0, 0.5, 2) for v in g.processors()}
    we = {v: float(rng.normal()) for v in g.processors()}
    mix = TR.render(g, cfg, dry, noise, th, we)
    labels = synth.subgroup_labels(3, cfg.n_tracks, cfg.n_subgroups)
    # nodes: track k -> i at 2k, g at 2k+1; subgroup s -> m at 2K + 2s, g at 2K + 2s + 1
    K = cfg.n_tracks
    sig = lambda x: 1 / (1 + math.exp(-x))
    ref = np.zeros((2, dry.shape[-1]))
    labels = [None] * K
    for s_, d_ in g.edges:
        if g.types[d_] == "m":
            labels[(s_ - 1) // 2] = d_
    for m_node in sorted(set(labels)):
        acc = np.zeros_like(ref)
        for k in range(K):
            if labels[k] != m_node:
                continue
            v = 2 * k + 1
            u = dry[k].astype(np.float64)
            w = sig(we[v])
            acc += w * np.exp(th[v])[:, None] * u + (1 - w) * u
        v = m_node + 1
        w = sig(we[v])
        ref += w * np.exp(th[v])[:, None] * acc + (1 - w) * acc
    assert np.allclose(mix, ref, rtol=1e-13, atol=1e-15)


def test_cycle_is_rejected():
    with pytest.raises(ValueError):
        C.topo_order(3, [(0, 1), (1, 2), (2, 0)])


def test_console_type_string_matches_paper():
    g = synth.make_console(3, [0, 1, 1], "ecnsgdr")
    # every track chain and every subgroup chain is the paper's order
    assert "".join(g.types[0:8]) == "iecnsgdr"
    m_nodes = [v for v, t in enumerate(g.types) if t == "m"]
    assert len(m_nodes) == 2 and g.types[-1] == "o"
    assert "".join(g.types[m_nodes[0]:m_nodes[0] + 8]) == "mecnsgdr"


# ---------------------------------------------------------------- loss
def test_a_weighting_published_values():
    """IEC 61672 A-weighting table at the exact base-ten mid-band frequencies
    1000 * 10^(n/10): 0 dB at 1 kHz, -19.1 dB at 100 Hz, -2.5 dB at 10 kHz,
    -39.4 dB at 31.5 Hz (n = -15), +1.3 dB at 2.5 kHz (n = 4); the table
    rounds to 0.1 dB."""
    db = lambda f: 20 * math.log10(float(LS.a_weighting_mag(f)))
    assert abs(db(1000.0)) < 1e-12
    for n, ref in ((-10, -19.1), (10, -2.5), (-15, -39.4), (4, 1.3), (-20, -70.4)):
        f = 1000.0 * 10.0 ** (n / 10.0)
        assert abs(db(f) - ref) < 0.051, (f, db(f))


def test_mel_filterbank_partition_of_unity_and_htk_scale():
    assert abs(float(LS.hz_to_mel(700.0)) - 2595 * math.log10(2)) < 1e-9
    fb = LS.mel_filterbank(2048, 44100, 96)
    pts = LS.mel_to_hz(np.linspace(0, LS.hz_to_mel(22050), 98))
    f = np.arange(1025) * 44100 / 2048
    inner = (f >= pts[1]) & (f <= pts[96])
    assert np.allclose(fb[:, inner].sum(0), 1.0, atol=1e-12)
    assert fb.max() <= 1.0 + 1e-15


def test_loss_zero_at_target_and_scale_law():
    cfg, g, dry, noise = _small(seconds=0.5)
    rng = np.random.default_rng(1)
    y = torch.tensor(rng.standard_normal((2, cfg.length)), dtype=DT)
    assert float(LS.mrstft(y, y, cfg.loss_ffts, cfg.fs)["La"]) == 0.0
    c = 2.0
    out = LS.mrstft(c * y, y, cfg.loss_ffts, cfg.fs)
    # every non-empty Mel cell moves by log c (eps negligible for this level);
    # the spectral-convergence term is exactly |1 - c| per resolution and combo
    nres = len(cfg.loss_ffts)
    frac = []
    for n_fft in cfg.loss_ffts:
        fb = LS.mel_filterbank(n_fft, cfg.fs)
        aw = LS.a_weighting_mag(np.arange(n_fft // 2 + 1) * cfg.fs / n_fft)
        frac.append(np.mean((fb * aw).sum(1) > 0))
    expect = sum(math.log(c) * fr + abs(1 - c) for fr in frac)
    for k in ("Llr", "Lm", "Ls"):
        assert abs(float(out[k]) - expect) < 1e-5, (k, float(out[k]), expect)
    assert abs(float(out["La"]) - expect) < 1e-5


def test_stft_frame_against_explicit_dft_matrix():
    rng = np.random.default_rng(2)
    x = torch.tensor(rng.standard_normal((2, 3000)), dtype=DT)
    n_fft, fs = 512, 16000
    Y = LS.mel_spectra(x, n_fft, fs)
    hop = n_fft // 4
    f = 3
    seg = x[:, f * hop:f * hop + n_fft].numpy()
    win = 0.5 - 0.5 * np.cos(2 * np.pi * np.arange(n_fft) / n_fft)
    k = np.arange(n_fft // 2 + 1)[:, None]
    t = np.arange(n_fft)[None, :]
    Dm = np.exp(-2j * np.pi * ((k * t) % n_fft) / n_fft)
    Xl, Xr = Dm @ (seg[0] * win), Dm @ (seg[1] * win)
    aw = LS.a_weighting_mag(np.arange(n_fft // 2 + 1) * fs / n_fft)
    fb = LS.mel_filterbank(n_fft, fs)
    for key, X in (("l", Xl), ("r", Xr), ("m", Xl + Xr), ("s", Xl - Xr)):
        assert np.allclose(Y[key][f].numpy(), fb @ (np.abs(X) * aw), rtol=1e-11, atol=1e-12)


# ---------------------------------------------------------------- gradients
def test_gradients_match_central_differences():
    """dL/dtheta from the oracle against central differences of L for a sample
    of entries of every processor type and of the dry/wet logits (delay z
    entries excluded: their rule is a surrogate, pinned separately)."""
    cfg, g, dry, noise = _small(seconds=0.12, fs=8000, loss_ffts=(128, 256), eq_taps=31,
                                delay_range_s=0.04, reverb_seconds=0.05)
    th, we = synth.random_params(5, g, cfg, std=0.2)
    gt, gw = synth.ground_truth_params(6, g, cfg)
    target = TR.render(g, cfg, dry, noise, gt, gw)
    vals, gth, gwe, _ = TR.loss_and_grad(g, cfg, dry, noise, target, th, we, alpha_p=1e-2,
                                         delay_rule=False)
    rng = np.random.default_rng(0)
    Kc = (cfg.delay_fir_taps + 1) // 2

    def L_at(th2, we2):
        return TR.losses(g, cfg, dry, noise, target, th2, we2, alpha_p=1e-2)["L"]

    checked = 0
    for v in g.processors():
        t = g.types[v]
        n = th[v].size
        cand = list(range(n))
        if t == "d":
            cand = [i for i in cand if (i % (2 + Kc)) >= 2]
        for i in rng.choice(cand, size=min(3, len(cand)), replace=False):
            h = 1e-6 * max(1.0, abs(th[v][i]))
            tp = {k: x.copy() for k, x in th.items()}
            tp[v][i] += h
            lp = L_at(tp, we)
            tp[v][i] -= 2 * h
            lm = L_at(tp, we)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - gth[v][i]) <= 2e-5 * max(1e-3, abs(fd)) + 1e-8, (t, v, i, fd, gth[v][i])
            checked += 1
        h = 1e-6
        wp = dict(we)
        wp[v] += h
        lp = L_at(th, wp)
        wp[v] -= 2 * h
        lm = L_at(th, wp)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - gwe[v]) <= 2e-5 * max(1e-3, abs(fd)) + 1e-8, (t, v, "w", fd, gwe[v])
    assert checked > 20


def test_attack_release_console_gradients_match_central_differences():
    cfg = synth.small_config(seconds=0.1, fs=8000, chain="ecg", eq_taps=31,
                             comp_mode="attack_release", stereo_tracks=False,
                             loss_ffts=(128, 256), n_tracks=2, n_subgroups=1)
    g, dry, noise = synth.song(2, cfg)
    th, we = synth.random_params(7, g, cfg, std=0.2)
    gt, gw = synth.ground_truth_params(8, g, cfg)
    target = TR.render(g, cfg, dry, noise, gt, gw)
    vals, gth, gwe, _ = TR.loss_and_grad(g, cfg, dry, noise, target, th, we)
    for v in g.processors():
        if g.types[v] != "c":
            continue
        for i in range(5):
            h = 1e-6 * max(1.0, abs(th[v][i]))
            tp = {k: x.copy() for k, x in th.items()}
            tp[v][i] += h
            lp = TR.losses(g, cfg, dry, noise, target, tp, we)["L"]
            tp[v][i] -= 2 * h
            lm = TR.losses(g, cfg, dry, noise, target, tp, we)["L"]
            fd = (lp - lm) / (2 * h)
            assert abs(fd - gth[v][i]) <= 1e-4 * max(1e-3, abs(fd)) + 1e-8, (v, i, fd, gth[v][i])


# ---------------------------------------------------------------- Adam
def test_adam_first_step_moves_by_lr_times_sign():
    g = np.array([3.0, -1e-3, 0.5, -40.0])
    th = np.zeros(4)
    m = np.zeros(4)
    v = np.zeros(4)
    TR.adam_step(th, m, v, g, 1, lr=1e-2)
    assert np.allclose(th, -1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    # second step with the same gradient: m_hat = g, v_hat = g^2 again
    TR.adam_step(th, m, v, g, 2, lr=1e-2)
    assert np.allclose(th, -2e-2 * g / (np.abs(g) + 1e-8), rtol=1e-10)


def test_adamw_matches_the_library_optimizer_and_its_closed_form():
    """AdamW (decoupled weight decay): against torch.optim.AdamW in FP64 over
    several steps, and with a zero gradient the parameters only decay,
    theta_t = (1 - lr wd)^t theta_0."""
    rng = np.random.default_rng(9)
    th0 = rng.normal(size=7)
    th = th0.copy()
    m = np.zeros(7)
    v = np.zeros(7)
    p = torch.nn.Parameter(torch.tensor(th0, dtype=DT))
    opt = torch.optim.AdamW([p], lr=1e-2, betas=(0.9, 0.999), eps=1e-8, weight_decay=0.05)
    for step in range(1, 6):
        g = rng.normal(size=7)
        TR.adamw_step(th, m, v, g, step, lr=1e-2, weight_decay=0.05)
        p.grad = torch.tensor(g, dtype=DT)
        opt.step()
    assert np.allclose(th, p.detach().numpy(), rtol=1e-13, atol=1e-15)
    th = th0.copy()
    m = np.zeros(7)
    v = np.zeros(7)
    for step in range(1, 4):
        TR.adamw_step(th, m, v, np.zeros(7), step, lr=1e-2, weight_decay=0.1)
    assert np.allclose(th, (1 - 1e-3) ** 3 * th0, rtol=1e-14)


def test_channel_swap_isolates_the_left_right_term():
    """Swapping l and r leaves |mid| and |side| spectra unchanged, so
    L_m = L_s = 0 and L_a = 0.5 L_lr exactly."""
    rng = np.random.default_rng(5)
    y = torch.tensor(rng.standard_normal((2, 5000)), dtype=DT)
    out = LS.mrstft(y.flip(0), y, (256, 512), 16000)
    assert float(out["Lm"]) == 0.0
    assert float(out["Ls"]) < 1e-12
    assert float(out["Llr"]) > 0.1
    assert abs(float(out["La"]) - 0.5 * float(out["Llr"])) < 1e-12


def test_gain_staging_term_of_a_constant_eq_is_its_log_gain():
    """Sec. 5.1 gain-staging regulariser, pinned by a closed form: an EQ whose
    log-magnitudes all equal c has the FIR e^c delta (the Dirichlet sum of an
    odd-length cosine series), so its wet output is e^c u and its term is
    exactly |c| at any dry/wet weight.  A term on the squared norm would give
    2|c|; one on the dry/wet-mixed output would give |log(w e^c + 1 - w)|.
    Gain/pan nodes contribute nothing (the sum runs over e, r and d only)."""
    cfg = synth.small_config(seconds=1.0, chain="eg", n_tracks=3, n_subgroups=2, eq_taps=63)
    g, dry, noise = synth.song(5, cfg)
    # every node carries signal, so the 1e-12 inside the norms is negligible
    assert np.sum(dry.astype(np.float64) ** 2, axis=(1, 2)).min() > 1e-2
    rng = np.random.default_rng(11)
    K = (cfg.eq_taps + 1) // 2
    th, we, cs = {}, {}, []
    for v in g.processors():
        if g.types[v] == "e":
            c = float(rng.uniform(-1.5, 1.5))
            cs.append(c)
            th[v] = torch.full((K,), c, dtype=DT)
        else:
            th[v] = torch.tensor(rng.normal(0, 0.7, 2), dtype=DT)
        we[v] = torch.tensor(float(rng.normal()), dtype=DT)
    out = C.evaluate(g, cfg, dry, noise, th, we)
    assert len(cs) == cfg.n_tracks + cfg.n_subgroups
    assert abs(float(out["Lg"]) - sum(abs(c) for c in cs)) < 1e-9
    # and the eq's wet output is the scaled input, sample for sample
    v = next(v for v in g.processors() if g.types[v] == "e")
    u = torch.tensor(rng.standard_normal((2, 500)), dtype=DT)
    ybar = C.process("e", u, th[v], cfg)
    assert torch.allclose(ybar, math.exp(float(th[v][0])) * u, rtol=0, atol=1e-12)
