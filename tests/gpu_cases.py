"""Shared setup for the GPU parity tests: one seeded synthetic song, its
target rendered by the FP64 oracle, the HIP session, and the oracle's
results on exactly the FP32 values the GPU sees."""
import numpy as np
import torch

import synth
from oracle import train as TR
from paper_2509_15948_amd import mixgraph as MG
from paper_2509_15948_amd import workloads as W


def f32(x):
    return np.asarray(x, np.float32).astype(np.float64)


class Case:
    def __init__(self, cfg, seed=3, params="random", alpha_g=1e-3, alpha_p=0.0, mode=1, std=0.3, max_trials=0,
                 trial_slots=0, unfused=False):
        self.cfg = cfg
        self.g, self.dry, self.noise = synth.song(seed, cfg)
        gt, gw = synth.ground_truth_params(seed + 100, self.g, cfg)
        self.target = TR.render(self.g, cfg, self.dry, self.noise, gt, gw).astype(np.float32)
        if params == "random":
            th, we = synth.random_params(seed, self.g, cfg, std=std)
        else:
            th, we = synth.init_params(seed, self.g, cfg)
        self.th = {v: f32(p) for v, p in th.items()}
        self.we = {v: float(np.float32(w)) for v, w in we.items()}
        self.alpha_g, self.alpha_p = alpha_g, alpha_p
        self.bg = W.binding_graph(self.g, cfg, alpha_g, alpha_p, max_trials=max_trials, trial_slots=trial_slots,
                                  unfused=unfused)
        dev = "cuda"
        self.noise_d = torch.from_numpy(W.noise_rows(self.bg, self.noise, cfg.reverb_length)).to(dev)
        self.target_d = torch.from_numpy(self.target).to(dev)
        self.dry_d = torch.from_numpy(self.dry).to(dev)
        self.sess = MG.Session(self.bg, self.noise_d, self.target_d, mode=mode)
        th_f, we_f = self.bg.flatten(self.th, self.we)
        self.theta_d = torch.from_numpy(th_f).to(dev)
        self.wet_d = torch.from_numpy(we_f).to(dev)
        self.sizes = {v: len(p) for v, p in self.th.items()}

    def mask_d(self, mask):
        return None if mask is None else torch.from_numpy(self.bg.mask_vector(mask)).cuda()

    def gpu_forward(self, mask=None):
        mix = torch.empty(2, self.cfg.length, dtype=torch.float32, device="cuda")
        losses = torch.zeros(7, dtype=torch.float64, device="cuda")
        self.sess.forward(self.dry_d, self.theta_d, self.wet_d, self.mask_d(mask), mix, losses)
        torch.cuda.synchronize()
        return mix.cpu().numpy().astype(np.float64), dict(zip(MG.LOSS_KEYS, losses.cpu().numpy().tolist()))

    def gpu_backward(self):
        gth = torch.empty(self.bg.n_theta, dtype=torch.float32, device="cuda")
        gwe = torch.empty(self.bg.n_proc, dtype=torch.float32, device="cuda")
        self.sess.backward(gth, gwe)
        torch.cuda.synchronize()
        return self.bg.unflatten(gth.cpu().numpy(), gwe.cpu().numpy(), self.sizes)

    def oracle(self, mask=None, grads=True):
        tgt = self.target.astype(np.float64)
        if grads:
            vals, gth, gwe, mix = TR.loss_and_grad(self.g, self.cfg, self.dry, self.noise, tgt, self.th, self.we,
                                                   mask, self.alpha_g, self.alpha_p)
            return mix, vals, gth, gwe
        vals = TR.losses(self.g, self.cfg, self.dry, self.noise, tgt, self.th, self.we, mask, self.alpha_g,
                         self.alpha_p)
        mix = TR.render(self.g, self.cfg, self.dry, self.noise, self.th, self.we, mask)
        return mix, vals, None, None


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


# Relative RMS error of one FP32 FFT convolution (a library FP32 FFT measures
# 2.7e-7 at 2^14 points); the loss is evaluated in FP64 on the FP32 mix.
FP32_CONV_REL = 3e-7


# Noise-derived bounds never exceed CAP x the stated tolerance.
CAP = 10.0
AUDIO_TERMS = ("L", "La", "Llr", "Lm", "Ls")


def _noisy_process(rng):
    """OC.process with FP32-level white noise (FP32_CONV_REL * RMS) added to
    every processor's wet output."""
    from oracle import console as OC
    orig = OC.process

    def noisy(t, u, p, cfg, noise=None):
        y = orig(t, u, p, cfg, noise)
        rms = float(y.detach().pow(2).mean().sqrt())
        return y + torch.from_numpy(rng.standard_normal(tuple(y.shape))) * (FP32_CONV_REL * rms)

    return orig, noisy


def _f32_storage_process():
    """OC.process with every processor's wet output rounded to FP32, the
    rounding every FP32 implementation makes when it stores a node output."""
    from oracle import console as OC
    orig = OC.process

    def rounded(t, u, p, cfg, noise=None):
        return orig(t, u, p, cfg, noise).to(torch.float32).to(torch.float64)

    return orig, rounded


# The storage-rounding shift is a floor: the GPU also rounds inside every
# processor, so its loss error may be a few times that shift.
FLOOR_MULT = 3.0


def loss_tolerances(case, omix=None, mask=None, draws=4, rel=1e-5, k=5.0):
    """Per loss term: max(rel * |L|, min(k * sigma, CAP * rel * scale),
    FLOOR_MULT * floor).

    sigma is the RMS change of the oracle's losses over `draws` draws of
    FP32-level white noise (FP32_CONV_REL * RMS) added to every processor's
    wet output: the GPU rounds at every processor, not only at the mix, and
    the errors of a chain of FFT convolutions accumulate; its loss error is
    one such draw, so the bound sits k standard deviations out.  That bound is
    capped at CAP x the stated tolerance.

    floor is the change of the oracle's losses when every processor output is
    rounded to FP32 and nothing else changes.  No FP32 implementation avoids
    that rounding; where the log-Mel term sits on quiet cells (a noisegate
    closing on a quiet mix) it alone exceeds the stated tolerance, and the
    bound follows it.  Everything is computed from the oracle only (omix is
    not used)."""
    from oracle import console as OC
    tgt = case.target.astype(np.float64)
    base = TR.losses(case.g, case.cfg, case.dry, case.noise, tgt, case.th, case.we, mask, case.alpha_g,
                     case.alpha_p)
    orig, noisy = _noisy_process(np.random.default_rng(4242))
    ss = {key: 0.0 for key in base}
    try:
        OC.process = noisy
        for _ in range(draws):
            out = TR.losses(case.g, case.cfg, case.dry, case.noise, tgt, case.th, case.we, mask, case.alpha_g,
                            case.alpha_p)
            for key in base:
                ss[key] += (float(out[key]) - float(base[key])) ** 2
        OC.process = _f32_storage_process()[1]
        rounded = TR.losses(case.g, case.cfg, case.dry, case.noise, tgt, case.th, case.we, mask, case.alpha_g,
                            case.alpha_p)
    finally:
        OC.process = orig
    la = abs(float(base["La"]))
    out = {}
    for key in base:
        noise = k * float(np.sqrt(ss[key] / draws))
        floor = abs(float(rounded[key]) - float(base[key]))
        # the noise-derived bound is capped at CAP x the stated tolerance; the
        # audio terms take it relative to L_a (a term that is zero in exact
        # arithmetic, such as the mid term of a chain that leaves the mid
        # signal alone, has no relative scale of its own)
        scale = max(abs(float(base[key])), la) if key in AUDIO_TERMS else abs(float(base[key]))
        out[key] = max(rel * abs(float(base[key])), min(noise, CAP * rel * scale), FLOOR_MULT * floor)
        print("loss bound", key, "stated", rel * abs(float(base[key])), "oracle noise", noise, "cap",
              CAP * rel * scale, "FP32 storage floor", floor, "->", out[key], flush=True)
    return out


def grad_tolerances(case, oth, owe, mask=None, draws=2, rel=1e-3):
    """Per processor type (and 'w' for the dry/wet logits): max(rel,
    min(CAP * rel, 3 * the relative change of the oracle's own gradient when FP32-level white noise
    (FP32_CONV_REL * RMS) is added to every processor's wet output).  The
    log-Mel term makes some gradients (the delay's normalised z direction, the
    noisegate near its threshold) sensitive to rounding in quiet cells; this
    measures that sensitivity with the oracle alone."""
    from oracle import console as OC
    tgt = case.target.astype(np.float64)
    orig, noisy = _noisy_process(np.random.default_rng(777))
    worst = {}
    types = sorted({case.g.types[v] for v in case.g.processors()})
    try:
        OC.process = noisy
        for _ in range(draws):
            _, gth, gwe, _ = TR.loss_and_grad(case.g, case.cfg, case.dry, case.noise, tgt, case.th, case.we,
                                              mask, case.alpha_g, case.alpha_p)
            for t in types:
                vs = [v for v in case.g.processors() if case.g.types[v] == t]
                e = rel_l2(np.concatenate([gth[v] for v in vs]), np.concatenate([oth[v] for v in vs]))
                worst[t] = max(worst.get(t, 0.0), e)
            procs = case.g.processors()
            e = rel_l2([gwe[v] for v in procs], [owe[v] for v in procs])
            worst["w"] = max(worst.get("w", 0.0), e)
    finally:
        OC.process = orig
    return {k: max(rel, min(3.0 * s, CAP * rel)) for k, s in worst.items()}, worst
