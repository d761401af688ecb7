"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module holds NO arithmetic of the mixing-graph method itself: it draws
dry multitrack songs, mixing-console graphs (node types and cables), raw
parameter vectors (ground truth and initial), the fixed reverb noise, and
pruning masks.  Everything a processor, the console, the loss or an adjoint
computes lives in ``oracle/`` (the FP64 reference) or in the HIP library, and
the two never share code.

Stand-in for the paper's datasets (MedleyDB, MixingSecrets, Internal; Sec. 5.3),
which are not available: songs are sums of harmonic tones gated by ADSR notes
plus pink-noise bursts, shaped like multitrack stems (17.6-28.8 tracks per
song in the paper's data, Sec. 7.6).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Sequence, Tuple

import numpy as np

# ---------------------------------------------------------------------------
# node types (Sec. 1.1: processors e c n s g d r; auxiliary i m o).  'x' is
# the tanh waveshaper of the benchmark configurations.
# ---------------------------------------------------------------------------
TYPE_CODES = {"i": 0, "m": 1, "o": 2, "e": 3, "c": 4, "n": 5, "x": 6,
              "s": 7, "g": 8, "d": 9, "r": 10}
CODE_TYPES = {v: k for k, v in TYPE_CODES.items()}
PROCESSOR_TYPES = "ecnxsgdr"


@dataclasses.dataclass(frozen=True)
class ConsoleConfig:
    """Sizes of one workload.  All lengths in samples unless stated."""
    name: str
    n_tracks: int
    n_subgroups: int
    seconds: float
    fs: int
    stereo_tracks: bool
    chain: str = "ecxsgdr"
    eq_taps: int = 2047            # N of the zero-phase EQ FIR (odd)
    comp_mode: str = "single"      # "single" or "attack_release"
    delay_taps: int = 4            # M taps per channel
    delay_range_s: float = 0.5     # all taps together span this many seconds
    delay_fir_taps: int = 39       # zero-phase FIR per tap (odd)
    reverb_seconds: float = 1.5
    reverb_nfft: int = 384
    reverb_hop: int = 192
    loss_ffts: Tuple[int, ...] = (512, 1024, 2048)
    n_mels: int = 96
    steps: int = 20
    lr: float = 1e-2

    @property
    def length(self) -> int:
        return int(round(self.seconds * self.fs))

    @property
    def reverb_length(self) -> int:
        return int(round(self.reverb_seconds * self.fs))

    @property
    def delay_range(self) -> int:
        """D: width of each tap's delay range in samples."""
        return int(math.floor(self.delay_range_s * self.fs / self.delay_taps))

    def n_params(self, t: str) -> int:
        """N_t: raw parameters of one node of type t (dry/wet excluded)."""
        if t == "g":
            return 2
        if t == "s":
            return 1
        if t == "x":
            return 2
        if t == "e":
            return (self.eq_taps + 1) // 2
        if t in "cn":
            return 5 if (t == "c" and self.comp_mode == "attack_release") else 4
        if t == "d":
            return 2 * self.delay_taps * (2 + (self.delay_fir_taps + 1) // 2)
        if t == "r":
            return 2 * 2 * (self.reverb_nfft // 2)
        return 0


CONFIGS: Dict[str, ConsoleConfig] = {
    # 4 mono tracks, 2 s, one subgroup; gain/pan + 1024-tap EQ + attack/release compressor
    "tiny": ConsoleConfig("tiny", 4, 1, 2.0, 44100, False, chain="ecg",
                          eq_taps=1023, comp_mode="attack_release",
                          loss_ffts=(512, 1024, 2048), steps=20),
    # 16 stereo tracks, 4 subgroups, 10 s, full processor set
    "full": ConsoleConfig("full", 16, 4, 10.0, 44100, True, steps=500),
    # 64 tracks, 8 subgroups, 60 s at 48 kHz, 2 s reverb, 5 loss resolutions
    "large": ConsoleConfig("large", 64, 8, 60.0, 48000, True, reverb_seconds=2.0,
                           loss_ffts=(256, 512, 1024, 2048, 4096), steps=200),
}


def small_config(name: str = "small", n_tracks: int = 3, n_subgroups: int = 2,
                 seconds: float = 0.75, fs: int = 16000, chain: str = "ecxsgdr",
                 **kw) -> ConsoleConfig:
    """A reduced console for parity tests: same structure, short signals."""
    base = dict(eq_taps=255, delay_range_s=0.1, reverb_seconds=0.2,
                loss_ffts=(256, 512, 1024), stereo_tracks=True)
    base.update(kw)
    stereo = base.pop("stereo_tracks")
    return ConsoleConfig(name, n_tracks, n_subgroups, seconds, fs, stereo,
                         chain=chain, **base)


# ---------------------------------------------------------------------------
# graphs
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Graph:
    types: List[str]              # per node, one of TYPE_CODES
    edges: List[Tuple[int, int]]  # (src, dst) cables
    track_of_input: Dict[int, int]  # input node -> dry track index

    @property
    def n_nodes(self) -> int:
        return len(self.types)

    def type_codes(self) -> np.ndarray:
        return np.array([TYPE_CODES[t] for t in self.types], dtype=np.int32)

    def edge_array(self) -> np.ndarray:
        if not self.edges:
            return np.zeros((2, 0), dtype=np.int32)
        return np.array(self.edges, dtype=np.int32).T.copy()

    def processors(self) -> List[int]:
        return [v for v, t in enumerate(self.types) if t in PROCESSOR_TYPES]


def subgroup_labels(seed: int, n_tracks: int, n_subgroups: int) -> List[int]:
    """A random surjection of tracks onto subgroups (subgrouping is known a priori)."""
    s = min(n_subgroups, n_tracks)
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 101])))
    labels = list(range(s)) + list(rng.integers(0, s, size=n_tracks - s))
    rng.shuffle(labels)
    return [int(x) for x in labels]


def make_console(n_tracks: int, labels: Sequence[int], chain: str) -> Graph:
    """Mixing console: every track gets the chain, tracks are summed per subgroup
    by an 'm' node, every subgroup gets the chain again, and subgroup chains are
    summed by the single output node 'o' (Sec. 1.2)."""
    types: List[str] = []
    edges: List[Tuple[int, int]] = []
    track_of_input: Dict[int, int] = {}

    def add(t: str) -> int:
        types.append(t)
        return len(types) - 1

    n_sub = max(labels) + 1 if len(labels) else 0
    track_ends = []
    for k in range(n_tracks):
        v = add("i")
        track_of_input[v] = k
        for t in chain:
            w = add(t)
            edges.append((v, w))
            v = w
        track_ends.append(v)
    sub_ends = []
    for s in range(n_sub):
        m = add("m")
        for k in range(n_tracks):
            if labels[k] == s:
                edges.append((track_ends[k], m))
        v = m
        for t in chain:
            w = add(t)
            edges.append((v, w))
            v = w
        sub_ends.append(v)
    o = add("o")
    for v in sub_ends:
        edges.append((v, o))
    return Graph(types, edges, track_of_input)


# ---------------------------------------------------------------------------
# dry tracks
# ---------------------------------------------------------------------------
def _rng(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(key))))


def _adsr_notes(rng, L, fs) -> np.ndarray:
    env = np.zeros(L)
    T = L / fs
    n_notes = rng.poisson(1.5 * T)
    for _ in range(n_notes):
        t0 = rng.uniform(0.0, T)
        dur = rng.uniform(0.2, 1.5)
        a = rng.uniform(0.005, 0.05)
        d = rng.uniform(0.05, 0.3)
        s = rng.uniform(0.3, 0.9)
        r = rng.uniform(0.05, 0.5)
        n0 = int(t0 * fs)
        n1 = min(L, int((t0 + dur + r) * fs) + 1)
        if n1 <= n0:
            continue
        t = np.arange(n1 - n0) / fs
        gate = np.where(t < a, t / a,
                        np.where(t < a + d, 1.0 - (1.0 - s) * (t - a) / d, s))
        rel_level = (dur / a) if dur < a else (1.0 - (1.0 - s) * (dur - a) / d if dur < a + d else s)
        rel = rel_level * np.clip(1.0 - (t - dur) / r, 0.0, 1.0)
        e = np.where(t < dur, gate, rel)
        env[n0:n1] = np.maximum(env[n0:n1], e)
    return env


def _pink_bursts(rng, L, fs, level) -> np.ndarray:
    out = np.zeros(L)
    T = L / fs
    fade = max(1, int(0.005 * fs))
    for _ in range(rng.poisson(0.5 * T)):
        n0 = int(rng.uniform(0.0, T) * fs)
        n = int(rng.uniform(0.05, 0.3) * fs)
        n = min(n, L - n0)
        if n < 4:
            continue
        white = rng.standard_normal(n)
        spec = np.fft.rfft(white)
        f = np.arange(spec.size, dtype=np.float64)
        f[0] = 1.0
        spec = spec / np.sqrt(f)
        spec[0] = 0.0
        pink = np.fft.irfft(spec, n)
        pink /= (np.sqrt(np.mean(pink ** 2)) + 1e-12)
        w = np.ones(n)
        k = min(fade, n // 2)
        ramp = 0.5 - 0.5 * np.cos(np.pi * np.arange(k) / k)
        w[:k] = ramp
        w[n - k:] = ramp[::-1]
        out[n0:n0 + n] += level * pink * w
    return out


def dry_track(seed: int, k: int, L: int, fs: int, stereo: bool) -> np.ndarray:
    """One dry source, shape [C][L] (C = 2 if stereo else 1), float64."""
    rng = _rng(seed, 11, k)
    t = np.arange(L) / fs
    tones = np.zeros(L)
    for _ in range(3):
        f0 = math.exp(rng.uniform(math.log(55.0), math.log(880.0)))
        phases = rng.uniform(0.0, 2.0 * math.pi, size=6)
        sig = np.zeros(L)
        for h in range(1, 7):
            if h * f0 < 0.45 * fs:
                sig += np.sin(2.0 * math.pi * h * f0 * t + phases[h - 1]) / h
        tones += sig * _adsr_notes(rng, L, fs)
    tone_rms = float(np.sqrt(np.mean(tones ** 2)))
    if tone_rms == 0.0:
        tone_rms = 0.1
    level = tone_rms * 10.0 ** (-12.0 / 20.0)
    chans = 2 if stereo else 1
    out = np.zeros((chans, L))
    for c in range(chans):
        out[c] = tones + _pink_bursts(rng, L, fs, level)
    if stereo:
        off = rng.uniform(-3.0, 3.0)
        out[0] *= 10.0 ** (off / 40.0)
        out[1] *= 10.0 ** (-off / 40.0)
    peak = float(np.max(np.abs(out))) or 1.0
    out *= 10.0 ** (rng.uniform(-24.0, -6.0) / 20.0) / peak
    # a recording noise floor near -100 dBFS, so no stem is digitally silent
    out += 1e-5 * rng.uniform(-1.0, 1.0, size=out.shape)
    return out


def dry_tracks(seed: int, cfg: ConsoleConfig) -> np.ndarray:
    """All dry sources, shape [K][C][L], float32 (tracks drawn in parallel
    threads for long songs; each track has its own generator, so the values
    do not depend on the threading)."""
    L = cfg.length
    if cfg.n_tracks * L > 20_000_000:
        from concurrent.futures import ThreadPoolExecutor
        import os
        with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
            tracks = list(ex.map(lambda k: dry_track(seed, k, L, cfg.fs, cfg.stereo_tracks), range(cfg.n_tracks)))
    else:
        tracks = [dry_track(seed, k, L, cfg.fs, cfg.stereo_tracks) for k in range(cfg.n_tracks)]
    return np.stack(tracks).astype(np.float32)


def reverb_noise(seed: int, node: int, cfg: ConsoleConfig) -> np.ndarray:
    """Fixed uniform noise of one reverb node: [2 (mid, side)][L_r], float32."""
    rng = _rng(seed, 7919, node)
    return rng.uniform(-1.0, 1.0, size=(2, cfg.reverb_length)).astype(np.float32)


def reverb_noise_all(seed: int, graph: Graph, cfg: ConsoleConfig) -> Dict[int, np.ndarray]:
    return {v: reverb_noise(seed, v, cfg) for v, t in enumerate(graph.types) if t == "r"}


# ---------------------------------------------------------------------------
# parameters (raw, unconstrained vectors; the maps to physical values belong
# to the method and are implemented on each side separately)
# ---------------------------------------------------------------------------
_LN10 = math.log(10.0)


def _db_to_ln_amp(db):
    return np.asarray(db) * _LN10 / 20.0


def _db_to_ln_energy(db):
    return np.asarray(db) * _LN10 / 10.0


def _logit(p):
    p = np.asarray(p, dtype=np.float64)
    return np.log(p) - np.log1p(-p)


def _rbj_mag(kind: str, f0: float, gain_db: float, q: float, fs: float, f: np.ndarray) -> np.ndarray:
    """|H(e^{jw})| of one audio-EQ-cookbook biquad (public RBJ formulas)."""
    A = 10.0 ** (gain_db / 40.0)
    w0 = 2.0 * math.pi * f0 / fs
    cw, sw = math.cos(w0), math.sin(w0)
    if kind == "peak":
        alpha = sw / (2.0 * q)
        b = [1 + alpha * A, -2 * cw, 1 - alpha * A]
        a = [1 + alpha / A, -2 * cw, 1 - alpha / A]
    else:
        alpha = sw / 2.0 * math.sqrt(2.0)  # shelf slope S = 1
        sa = 2.0 * math.sqrt(A) * alpha
        if kind == "low":
            b = [A * ((A + 1) - (A - 1) * cw + sa), 2 * A * ((A - 1) - (A + 1) * cw),
                 A * ((A + 1) - (A - 1) * cw - sa)]
            a = [(A + 1) + (A - 1) * cw + sa, -2 * ((A - 1) + (A + 1) * cw),
                 (A + 1) + (A - 1) * cw - sa]
        else:
            b = [A * ((A + 1) + (A - 1) * cw + sa), -2 * A * ((A - 1) + (A + 1) * cw),
                 A * ((A + 1) + (A - 1) * cw - sa)]
            a = [(A + 1) - (A - 1) * cw + sa, 2 * ((A - 1) - (A + 1) * cw),
                 (A + 1) - (A - 1) * cw - sa]
    z = np.exp(-1j * 2.0 * math.pi * f / fs)
    num = b[0] + b[1] * z + b[2] * z * z
    den = a[0] + a[1] * z + a[2] * z * z
    return np.abs(num / den)


def ground_truth_params(seed: int, graph: Graph, cfg: ConsoleConfig):
    """Raw parameters of a plausible target mix.  Returns (theta, wet_logit):
    theta[v] is the raw vector of processor v, wet_logit[v] its dry/wet logit."""
    theta: Dict[int, np.ndarray] = {}
    wet: Dict[int, float] = {}
    fs = cfg.fs
    for v, t in enumerate(graph.types):
        if t not in PROCESSOR_TYPES:
            continue
        rng = _rng(seed, 23, v)
        if t == "g":
            p = _db_to_ln_amp(rng.uniform(-12.0, 6.0, size=2))
        elif t == "s":
            p = _db_to_ln_amp(rng.uniform(-6.0, 6.0, size=1))
        elif t == "x":
            drive = rng.uniform(0.0, 18.0)
            p = np.array([_db_to_ln_amp(drive), _db_to_ln_amp(-0.8 * drive)])
        elif t == "e":
            K = cfg.n_params("e")
            N = cfg.eq_taps
            f = np.arange(K) * fs / N
            mag = (_rbj_mag("low", math.exp(rng.uniform(math.log(60), math.log(250))),
                            rng.uniform(-9, 9), 0.707, fs, f)
                   * _rbj_mag("peak", math.exp(rng.uniform(math.log(250), math.log(4000))),
                              rng.uniform(-9, 9), rng.uniform(0.5, 2.0), fs, f)
                   * _rbj_mag("high", math.exp(rng.uniform(math.log(4000), math.log(12000))),
                              rng.uniform(-9, 9), 0.707, fs, f))
            p = np.log(mag)
        elif t in "cn":
            if t == "c":
                T_db = rng.uniform(-30.0, -10.0)
                R = rng.uniform(1.0, 8.0)
            else:
                T_db = rng.uniform(-70.0, -40.0)
                R = rng.uniform(1.5, 4.0)
            knee_db = rng.uniform(2.0, 12.0)
            tail = [float(_db_to_ln_energy(T_db)),
                    math.log(float(_db_to_ln_energy(knee_db / 2.0))),
                    math.log(max(R - 1.0, 0.05))]
            if t == "c" and cfg.comp_mode == "attack_release":
                ta = rng.uniform(0.001, 0.030)
                tr = rng.uniform(0.050, 0.300)
                aa, ar = math.exp(-1.0 / (ta * fs)), math.exp(-1.0 / (tr * fs))
                p = np.array([_logit(aa), _logit(ar)] + tail)
            else:
                tau = rng.uniform(0.005, 0.100)
                al = math.exp(-1.0 / (tau * fs))
                p = np.array([_logit(al)] + tail)
        elif t == "d":
            M = cfg.delay_taps
            Kc = (cfg.delay_fir_taps + 1) // 2
            p = np.zeros((2, M, 2 + Kc))
            for c in range(2):
                for m in range(M):
                    phi = rng.uniform(-math.pi, math.pi)
                    p[c, m, 0] = math.cos(phi)
                    p[c, m, 1] = math.sin(phi)
                    p[c, m, 2:] = rng.normal(-1.5, 0.5, size=Kc)
            p = p.reshape(-1)
        elif t == "r":
            nb = cfg.reverb_nfft // 2
            hop = cfg.reverb_hop
            p = np.zeros((2, 2, nb))
            fk = np.arange(nb) * fs / cfg.reverb_nfft
            # raw values that the console maps to the drawn colouration and
            # decay (inverse of the documented input conventions: gain offset
            # -0.5 log(0.5 fs / (6 * 6.91)), decay -softplus(raw + beta))
            beta = math.log(math.expm1(6.91 * hop / (0.5 * fs)))
            gbias = -0.5 * math.log(0.5 * fs / (6.0 * 6.91))
            for x in range(2):
                rt60 = rng.uniform(0.3, 1.5)
                dec = -6.91 * hop / (rt60 * fs) * np.where(fk > 4000.0, 1.5, 1.0)
                p[x, 0] = rng.normal(-3.0, 0.3, size=nb) - gbias
                p[x, 1] = np.log(np.expm1(-dec)) - beta
            p = p.reshape(-1)
        else:
            raise ValueError(t)
        theta[v] = np.asarray(p, dtype=np.float64).reshape(-1)
        wet[v] = float(_logit(rng.uniform(0.3, 0.95)))
    return theta, wet


def init_params(seed: int, graph: Graph, cfg: ConsoleConfig, std: float = 0.1):
    """Initial raw parameters: N(0, 10^-2) on every entry (Sec. 5.1)."""
    rng = _rng(seed + 1, 31)
    theta: Dict[int, np.ndarray] = {}
    wet: Dict[int, float] = {}
    for v, t in enumerate(graph.types):
        if t not in PROCESSOR_TYPES:
            continue
        theta[v] = rng.normal(0.0, std, size=cfg.n_params(t))
        wet[v] = float(rng.normal(0.0, std))
    return theta, wet


def random_params(seed: int, graph: Graph, cfg: ConsoleConfig, std: float = 0.3):
    """Random raw parameters around the ground-truth draw (for parity tests that
    need every processor away from its trivial point)."""
    gt, gw = ground_truth_params(seed, graph, cfg)
    rng = _rng(seed, 977)
    th = {v: gt[v] + rng.normal(0.0, std, size=gt[v].shape) for v in gt}
    we = {v: gw[v] + float(rng.normal(0.0, std)) for v in gw}
    # delay angular frequencies stay inside the unit disk, where the
    # surrogate of Sec. 3.7 is defined: radius drawn in [0.5, 0.95]
    Kc = (cfg.delay_fir_taps + 1) // 2
    for v, t in enumerate(graph.types):
        if t == "d":
            p = th[v].reshape(2, cfg.delay_taps, 2 + Kc)
            r = rng.uniform(0.5, 0.95, size=(2, cfg.delay_taps))
            ang = np.arctan2(p[:, :, 1], p[:, :, 0])
            p[:, :, 0] = r * np.cos(ang)
            p[:, :, 1] = r * np.sin(ang)
            th[v] = p.reshape(-1)
    return th, we


def song(seed: int, cfg: ConsoleConfig):
    """Everything one search needs: graph, dry tracks, reverb noise."""
    labels = subgroup_labels(seed, cfg.n_tracks, cfg.n_subgroups)
    graph = make_console(cfg.n_tracks, labels, cfg.chain)
    dry = dry_tracks(seed, cfg)
    noise = reverb_noise_all(seed, graph, cfg)
    return graph, dry, noise


# ---------------------------------------------------------------------------
# serving workload: whole-song searches arriving over time
# ---------------------------------------------------------------------------
def serving_requests(seed: int, n: int, rate: float, tracks=(4, 32), subgroups=(2, 8), seconds=(5.0, 30.0),
                     fs: int = 44100, chain: str = "ecxsgdr", **kw) -> List[Tuple[float, ConsoleConfig, int]]:
    """n requests: (arrival time in s, console sizes, song seed).  Arrivals
    form a Poisson process of the given rate (exponential gaps); tracks and
    subgroups are uniform integers in the closed ranges (subgroups capped at
    the track count), lengths uniform in seconds."""
    rng = _rng(seed, 4099)
    t = 0.0
    out = []
    for i in range(n):
        t += float(rng.exponential(1.0 / rate)) if rate > 0 else 0.0
        k = int(rng.integers(tracks[0], tracks[1] + 1))
        s = min(k, int(rng.integers(subgroups[0], subgroups[1] + 1)))
        sec = round(float(rng.uniform(seconds[0], seconds[1])), 3)
        cfg = ConsoleConfig(f"request{i}", k, s, sec, fs, True, chain=chain, **kw)
        out.append((t, cfg, int(seed * 1000 + i)))
    return out
