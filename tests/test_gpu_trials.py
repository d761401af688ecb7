"""Pruning trials by suffix recomputation (mg_forward_trials) against complete
masked forwards (mg_forward_masked) and the oracle, and the pruning round
driver against the oracle's rule."""
import numpy as np
import pytest
import torch

import synth
from oracle import prune as OP
from paper_2509_15948_amd import mixgraph as MG

from gpu_cases import Case, loss_tolerances

pytestmark = pytest.mark.gpu


def _small(chain="ecxsgdr", **kw):
    base = dict(seconds=0.75, fs=16000, n_tracks=3, n_subgroups=2, chain=chain)
    base.update(kw)
    return synth.small_config(**base)


def _trial_case(max_trials, trial_slots=0, mode=1, chain="ecxsgdr", seed=3):
    case = Case(_small(chain), seed=seed, mode=mode, max_trials=max_trials, trial_slots=trial_slots)
    return case


def _keeps(case, rng, B):
    """Single bypasses, pairs on one path (one downstream of the other) and
    random multi-bypass masks."""
    P = case.bg.n_proc
    procs = case.g.processors()
    keep = np.ones((B, P), np.uint8)
    for b in range(B):
        kind = b % 3
        if kind == 0:
            keep[b, rng.integers(P)] = 0
        elif kind == 1:
            v = procs[rng.integers(len(procs))]
            path = [v]
            while case.g.types[path[-1]] != "o":
                path.append(next(d for s, d in case.g.edges if s == path[-1]))
            chain = [u for u in path if u in procs]
            for u in chain[:2]:
                keep[b, int(case.bg.proc_index[u])] = 0
        else:
            keep[b, rng.choice(P, size=4, replace=False)] = 0
    return keep


def _masked_reference(case, keep):
    masks = torch.from_numpy(keep.astype(np.float32)).cuda()
    out = torch.zeros(keep.shape[0], 7, dtype=torch.float64, device="cuda")
    case.sess.forward_masked(case.dry_d, case.theta_d, case.wet_d, masks, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _trials(case, keep):
    out = torch.zeros(keep.shape[0], 7, dtype=torch.float64, device="cuda")
    case.sess.forward_trials(keep, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("slots", [0, 40])
def test_trials_equal_complete_masked_forwards_bitwise(slots):
    """Suffix recomputation gives the very bits of a complete forward with the
    same mask (40 slots hold any one trial of this 41-node console but not all
    twelve, so they run in several batches)."""
    case = _trial_case(12, trial_slots=slots, mode=0)
    keep = _keeps(case, np.random.default_rng(0), 12)
    case.gpu_forward()
    got = _trials(case, keep)
    ref = _masked_reference(case, keep)
    for b in range(len(keep)):
        print("trial", b, "dropped", np.flatnonzero(keep[b] == 0).tolist(), "L", got[b][0], "ref", ref[b][0],
              flush=True)
    assert np.array_equal(got, ref)


def test_trials_against_the_oracle():
    case = _trial_case(4, mode=0)
    keep = _keeps(case, np.random.default_rng(1), 4)
    case.gpu_forward()
    got = _trials(case, keep)
    procs = case.g.processors()
    for b in range(len(keep)):
        mask = {v: float(keep[b, int(case.bg.proc_index[v])]) for v in procs}
        omix, ol, _, _ = case.oracle(mask, grads=False)
        tol = loss_tolerances(case, omix, mask)
        for i, k in enumerate(MG.LOSS_KEYS):
            bound = max(1e-5 * abs(ol[k]), tol.get(k, 0.0))
            print("trial", b, k, got[b][i], ol[k], flush=True)
            assert abs(got[b][i] - ol[k]) <= bound or abs(got[b][i] - ol[k]) < 1e-9, (b, k)


def test_trials_with_a_base_mask():
    """Trial masks multiply the mask of the cached forward."""
    case = _trial_case(3, mode=0)
    P = case.bg.n_proc
    base = np.ones(P, np.float32)
    base[[0, 5]] = 0.0
    base[7] = 0.5
    base_d = torch.from_numpy(base).cuda()   # must stay alive: the trials read it
    case.sess.forward(case.dry_d, case.theta_d, case.wet_d, base_d, None,
                      torch.zeros(7, dtype=torch.float64, device="cuda"))
    keep = np.ones((3, P), np.uint8)
    keep[0, 2] = 0
    keep[1, [3, 9]] = 0
    keep[2, 7] = 0
    got = _trials(case, keep)
    masks = torch.from_numpy((keep * base[None, :]).astype(np.float32)).cuda()
    out = torch.zeros(3, 7, dtype=torch.float64, device="cuda")
    case.sess.forward_masked(case.dry_d, case.theta_d, case.wet_d, masks, out)
    torch.cuda.synchronize()
    assert np.array_equal(got, out.cpu().numpy())


def test_trials_leave_a_pending_backward_intact():
    case = _trial_case(6, mode=1)
    case.gpu_forward()
    g_ref, w_ref = case.gpu_backward()
    case.gpu_forward()
    _trials(case, _keeps(case, np.random.default_rng(2), 6))
    g, w = case.gpu_backward()
    for v in g:
        assert np.array_equal(g[v], g_ref[v]), v
    assert w == w_ref


def test_trials_need_a_cached_forward():
    case = _trial_case(2, mode=0)
    keep = np.ones((1, case.bg.n_proc), np.uint8)
    with pytest.raises(MG.MixgraphError):
        _trials(case, keep)


def test_full_console_64_single_bypass_trials():
    """16 tracks, 4 subgroups, 10 s: 64 single-processor trials in one batch;
    a sample of them against complete masked forwards, bit for bit."""
    cfg = synth.CONFIGS["full"]
    case = Case(cfg, seed=1, params="init", mode=0, max_trials=64)
    P = case.bg.n_proc
    keep = np.ones((64, P), np.uint8)
    for b in range(64):
        keep[b, (b * 37) % P] = 0
    case.gpu_forward()
    got = _trials(case, keep)
    pick = [0, 17, 40, 63]
    ref = _masked_reference(case, keep[pick])
    assert np.array_equal(got[pick], ref)


def test_pruning_round_matches_the_oracle_rule():
    """One round on the GPU (binding driver over the C-ABI rule) against the
    oracle's rule applied to the GPU's own trial losses, and the decisions
    against the oracle's losses where they are not within 1e-5 L of a
    threshold."""
    case = _trial_case(16, mode=0, seed=4)
    res = MG.prune_round(case.sess, case.dry_d, case.theta_d, case.wet_d, None, tau=1e-2, max_candidates=16)
    print("round", res, flush=True)
    alive = [True] * case.bg.n_proc
    # oracle rule on the GPU's trial losses
    lookup = {}
    for keepv, L in res["evaluated"]:
        lookup[tuple(bool(x) for x in keepv)] = L
    we = case.wet_d.cpu().numpy().astype(np.float64)
    w = (1.0 / (1.0 + np.exp(-we))).tolist()
    new, L_new, info = OP.prune_round(lambda a: lookup[tuple(bool(x) for x in a)], alive, w, res["L_start"],
                                      tau=1e-2, max_candidates=16)
    assert info["candidates"] == res["candidates"]
    assert info["order"] == res["order"]
    assert info["k"] == res["k"]
    assert new == [bool(x) for x in res["alive"]]
    assert L_new == res["L_min"]
    # the oracle's own losses: same decisions unless one sits within 1e-5 L of
    # its threshold (several outcomes are then correct)
    procs = case.g.processors()
    node_of = {int(case.bg.proc_index[v]): v for v in procs}

    def oracle_La(alive_mask):
        mask = {node_of[p]: (1.0 if a else 0.0) for p, a in enumerate(alive_mask)}
        return case.oracle(mask, grads=False)[1]["La"]

    L0 = oracle_La(alive)
    onew, _, oinfo = OP.prune_round(oracle_La, alive, w, L0, tau=1e-2, max_candidates=16)
    print("oracle round", oinfo, flush=True)
    margin = 1e-5 * L0
    near = any(abs(L - L0 - 1e-2 * L0) < margin for L in oinfo["L_cand"])
    near = near or any(abs(L - L0 * (1 + 1e-2)) < margin for L in oinfo["L_prefix"])
    if not near:
        assert onew == new


def test_compacted_graph_gives_the_masked_audio_loss():
    """Sec. 1.2: removing the bypassed processors (graph surgery, parameters
    remapped) leaves the mix, and so L_a, bit for bit as under the mask."""
    case = _trial_case(4, mode=1, seed=6)
    P = case.bg.n_proc
    alive = np.ones(P, np.uint8)
    alive[[1, 4, 9, 17, 30]] = 0
    mask_d = torch.from_numpy(alive.astype(np.float32)).cuda()
    mix_m = torch.empty(2, case.cfg.length, device="cuda")
    lm = torch.zeros(7, dtype=torch.float64, device="cuda")
    case.sess.forward(case.dry_d, case.theta_d, case.wet_d, mask_d, mix_m, lm)
    new, o2n, sess, noise_d, (th,), (we,) = MG.compact(case.bg, alive, case.noise, case.cfg.reverb_length,
                                                       case.target_d, (case.theta_d,), (case.wet_d,))
    assert new.n_proc == P - 5
    mix_c = torch.empty(2, case.cfg.length, device="cuda")
    lc = torch.zeros(7, dtype=torch.float64, device="cuda")
    sess.forward(case.dry_d, th, we, None, mix_c, lc)
    torch.cuda.synchronize()
    assert torch.equal(mix_m, mix_c)
    assert lm[1].item() == lc[1].item()
    gth = torch.empty(new.n_theta, device="cuda")
    gwe = torch.empty(new.n_proc, device="cuda")
    sess.backward(gth, gwe)
    torch.cuda.synchronize()
    assert torch.isfinite(gth).all() and torch.isfinite(gwe).all()


def test_drywet_round_matches_the_oracle_rule():
    """One iteration of the dry/wet method (Alg. 3) on the GPU (the binding's
    driver: one suffix-recomputed trial at a time, the library's rule)
    against the oracle's rule applied to the GPU's own trial losses, with the
    paper's absolute tolerance; every trial loss against the oracle's loss of
    the same mask."""
    case = _trial_case(16, mode=0, seed=5)
    rng = np.random.default_rng(11)
    u = rng.random(4 * case.bg.n_proc + 64)
    res = MG.drywet_round(case.sess, case.dry_d, case.theta_d, case.wet_d, u, tau=0.05, relative=False)
    print("dry/wet round: trials", res["trials"], "pruned", int((res["alive"] == 0).sum()), "L_min", res["L_min"],
          flush=True)
    lookup = {tuple(bool(x) for x in k): L for k, L in res["evaluated"]}
    wet = case.wet_d.cpu().numpy()
    w32 = (np.float32(1.0) / (np.float32(1.0) + np.exp(-wet))).astype(np.float32).tolist()
    procs = case.g.processors()
    node_of = {int(case.bg.proc_index[v]): v for v in procs}
    types = [case.g.types[node_of[p]] for p in range(case.bg.n_proc)]
    new, L_new, info = OP.drywet_round(lambda a: lookup[tuple(bool(x) for x in a)], [True] * case.bg.n_proc, w32,
                                       types, res["L_start"], 0.05, u.tolist(), relative=False)
    assert len(info["trials"]) == res["trials"]
    assert new == [bool(x) for x in res["alive"]]
    assert L_new == res["L_min"]
    # the trial losses themselves against the oracle
    worst = 0.0
    for keep, L in res["evaluated"][:6]:
        mask = {node_of[p]: float(k) for p, k in enumerate(keep)}
        ref = case.oracle(mask, grads=False)[1]["La"]
        tol = loss_tolerances(case, mask=mask)
        worst = max(worst, abs(L - ref) / abs(ref))
        assert abs(L - ref) <= max(tol["La"], 1e-5 * abs(ref)), (L, ref)
    print("worst trial loss rel err", worst, flush=True)
