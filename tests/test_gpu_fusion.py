"""Fused pointwise chains (one launch for consecutive gain/pan, imager and
waveshaper stages, forward and backward) against one launch per stage: the
same bits for the mix, the losses and every gradient."""
import numpy as np
import pytest

import synth

from gpu_cases import Case

pytestmark = pytest.mark.gpu


def _pair(cfg, **kw):
    return Case(cfg, unfused=False, **kw), Case(cfg, unfused=True, **kw)


def _same(fused, plain, mask=None):
    mf, lf = fused.gpu_forward(mask)
    mp, lp = plain.gpu_forward(mask)
    assert np.array_equal(mf, mp)
    assert lf == lp
    gf, wf = fused.gpu_backward()
    gp, wp = plain.gpu_backward()
    for v in gp:
        assert np.array_equal(gf[v], gp[v]), v
    assert wf == wp


@pytest.mark.parametrize("chain", ["ecxsgdr", "sxg", "gx", "xg"])
def test_fused_chains_match_per_stage_launches(chain):
    cfg = synth.small_config(seconds=0.5, fs=16000, n_tracks=3, n_subgroups=2, chain=chain)
    fused, plain = _pair(cfg, seed=5)
    print("chain", chain, flush=True)
    _same(fused, plain)


def test_fused_chains_odd_length():
    """A length that is not a multiple of 4 takes the single-sample path of
    the pointwise kernels (and every kernel's ragged tails)."""
    cfg = synth.small_config(seconds=8001 / 16000, fs=16000, n_tracks=3, n_subgroups=2, chain="ecxsgdr")
    assert cfg.length == 8001
    fused, plain = _pair(cfg, seed=7)
    _same(fused, plain)


def test_fused_chains_with_a_mask():
    cfg = synth.small_config(seconds=0.5, fs=16000, n_tracks=3, n_subgroups=2, chain="ecxsgdr")
    fused, plain = _pair(cfg, seed=6)
    procs = fused.g.processors()
    mask = {v: 1.0 for v in procs}
    for v in procs[::4]:
        mask[v] = 0.0
    mask[procs[1]] = 0.5
    _same(fused, plain, mask)


def test_fused_chains_full_console():
    fused, plain = _pair(synth.CONFIGS["full"], seed=2)
    _same(fused, plain)
