"""A step captured as a HIP graph (mixgraph.StepGraph: mg_forward and
mg_backward of a session) against the same step run eagerly: every replay,
with eager work and synchronisations between replays, gives the eager step's
losses and gradients bit for bit, and a replay after the parameters change
in place follows the new values."""
import pytest
import torch

import synth
from paper_2509_15948_amd import mixgraph as MG

from gpu_cases import Case

pytestmark = pytest.mark.gpu


def _eager(case, theta):
    losses = torch.zeros(7, dtype=torch.float64, device="cuda")
    gth = torch.empty_like(theta)
    gwe = torch.empty_like(case.wet_d)
    case.sess.forward(case.dry_d, theta, case.wet_d, None, None, losses)
    case.sess.backward(gth, gwe)
    torch.cuda.synchronize()
    return losses.clone(), gth.clone(), gwe.clone()


@pytest.mark.parametrize("name", ["small", "48k"])
def test_captured_step_replays_the_eager_step(name):
    if name == "small":
        cfg = synth.small_config(seconds=0.75, fs=16000, n_tracks=3, n_subgroups=2, chain="ecxsgdr")
    else:
        # 3072-point engine rows, the 4096-point loss group on the side stream
        cfg = synth.small_config(seconds=0.75, fs=48000, n_tracks=3, n_subgroups=2, chain="ecxsgdr",
                                 loss_ffts=(256, 512, 1024, 2048, 4096))
    case = Case(cfg, alpha_p=1e-2)
    theta = case.theta_d.clone()
    ref = _eager(case, theta)
    losses = torch.zeros(7, dtype=torch.float64, device="cuda")
    gth = torch.empty_like(theta)
    gwe = torch.empty_like(case.wet_d)
    step = MG.StepGraph(case.sess, case.dry_d, theta, case.wet_d, None, losses, gth, gwe)
    for rep in range(4):
        losses.fill_(float("nan"))
        gth.fill_(float("nan"))
        gwe.fill_(float("nan"))
        step.replay()
        torch.cuda.synchronize()
        print(name, "replay", rep, "L", float(losses[0]), flush=True)
        assert torch.equal(losses, ref[0]), rep
        assert torch.equal(gth, ref[1]), rep
        assert torch.equal(gwe, ref[2]), rep
        # eager work of the program between replays
        other = _eager(case, theta)
        assert torch.equal(other[0], ref[0])
    # the graph reads the parameters at replay time
    theta.mul_(0.97)
    ref2 = _eager(case, theta)
    assert not torch.equal(ref2[0], ref[0])
    step.replay()
    torch.cuda.synchronize()
    assert torch.equal(losses, ref2[0])
    assert torch.equal(gth, ref2[1])
    assert torch.equal(gwe, ref2[2])
