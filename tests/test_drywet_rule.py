"""The library's dry/wet method (mg_drywet_*, host only) against the
oracle's (oracle/prune.py drywet_round, Alg. 3) on random loss tables: the
same trials in the same order, the same final mask and threshold, for the
relative and the absolute tolerance, with ties in the weights."""
import numpy as np
import pytest

from oracle import prune as OP
from paper_2509_15948_amd import mixgraph as MG

TYPES = "ecnxsgdr"


def _run_library(proc_type, wet, mask, alive, L_min, tau, relative, u, loss):
    dw = MG.DryWet(proc_type, wet, mask, alive, L_min, tau, relative, u)
    trials = []
    while True:
        keep = dw.next()
        if keep is None:
            break
        L = loss(keep.astype(bool).tolist())
        dw.report(L)
        trials.append(keep.tolist())
    keep, L_new, n = dw.end()
    return keep, L_new, trials


@pytest.mark.parametrize("seed", range(40))
def test_library_rule_equals_the_oracle_rule(seed):
    rng = np.random.default_rng(seed)
    P = int(rng.integers(1, 60))
    codes = rng.choice([3, 4, 5, 6, 7, 8, 9, 10], size=P).astype(np.int32)
    types = [TYPES[[3, 4, 5, 6, 7, 8, 9, 10].index(c)] for c in codes]
    wet = rng.normal(size=P).astype(np.float32)
    if seed % 4 == 0:
        wet[: P // 2] = wet[0]                              # ties in w
    mask = (rng.random(P) < 0.9).astype(np.float32) if seed % 3 == 0 else None
    alive = (rng.random(P) < 0.85).astype(np.uint8)
    w32 = (np.float32(1.0) / (np.float32(1.0) + np.exp(-wet))).astype(np.float32)
    if mask is not None:
        w32 = w32 * mask
    relative = bool(seed % 2)
    tau = float(rng.choice([1e-3, 1e-2, 0.1]))
    base = rng.normal(scale=0.4 * tau, size=P)
    pair = rng.normal(scale=0.1 * tau, size=(P, P))

    def loss(alive_mask):
        off = np.array([not a for a in alive_mask])
        return float(1.0 + base[off].sum() + pair[np.ix_(off, off)].sum() / 2)

    u = rng.random(4 * P + 64)
    k_lib, L_lib, trials = _run_library(codes, wet, mask, alive, 1.0, tau, relative, u, loss)
    m_or, L_or, info = OP.drywet_round(loss, alive.astype(bool).tolist(), w32.tolist(), types, 1.0, tau,
                                       u.tolist(), relative=relative)
    assert len(trials) == len(info["trials"])
    m = alive.astype(bool).tolist()
    for keep, tr in zip(trials, info["trials"]):
        expect = [a and p not in tr["candidates"] for p, a in enumerate(m)]
        assert [bool(k) for k in keep] == expect
        if tr["accepted"]:
            m = expect
    assert k_lib.astype(bool).tolist() == m_or
    assert L_lib == L_or


def test_out_of_draws_and_call_order_are_errors():
    dw = MG.DryWet(np.array([3, 3], np.int32), np.zeros(2, np.float32), None, np.ones(2, np.uint8), 1.0, 0.01,
                   False, np.zeros(0))
    with pytest.raises(MG.MixgraphError):
        dw.next()
    dw = MG.DryWet(np.array([3], np.int32), np.zeros(1, np.float32), None, np.ones(1, np.uint8), 1.0, 0.01,
                   False, np.zeros(4))
    assert dw.next() is not None
    with pytest.raises(MG.MixgraphError):
        dw.next()                                           # the loss was not reported
    dw.report(float("nan"))                                 # a NaN loss fails the test
    assert dw.next() is None                                # count 1 failed: the type left
    keep, L, n = dw.end()
    assert keep.tolist() == [1] and L == 1.0 and n == 1
