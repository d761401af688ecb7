"""Serving loop on the GPU: several searches admitted as they arrive, their
work overlapping on separate streams; each result equals the same search
run alone, bit for bit."""
import numpy as np
import pytest

import synth
from paper_2509_15948_amd import serve as SV

pytestmark = pytest.mark.gpu

SPEC = SV.SearchSpec(steps=6, rounds=2, finetune=2, tau=5e-2, candidates=8, quantum=2)
SMALL = dict(eq_taps=255, delay_range_s=0.1, reverb_seconds=0.2, loss_ffts=(256, 512, 1024))


def _requests():
    return synth.serving_requests(5, 4, rate=200.0, tracks=(2, 5), subgroups=(1, 3), seconds=(0.4, 0.9),
                                  fs=16000, **SMALL)


def _make(i, cfg, seed):
    return SV.Search(i, cfg, seed, SPEC)


def test_each_search_is_the_same_alone_and_in_the_mix():
    reqs = _requests()
    alone = [SV.run_alone(_make(i, cfg, seed)) for i, (_, cfg, seed) in enumerate(reqs)]
    server = SV.Server(budget_bytes=1 << 40, max_active=4)
    out = server.run(reqs, _make)
    print("p50", out["p50_s"], "p99", out["p99_s"], "peak active", out["peak_active"], flush=True)
    assert out["peak_active"] >= 2, "the searches did not overlap"
    for a, m in zip(alone, out["results"]):
        print("trace", m["trace"], flush=True)
        assert np.array_equal(a["losses"], m["losses"])
        assert np.array_equal(a["theta"], m["theta"])
        assert np.array_equal(a["wet"], m["wet"])
        assert a["types"] == m["types"] and a["processors"] == m["processors"]


def test_memory_budget_serialises_admission():
    reqs = _requests()
    size = max(_make(i, cfg, seed).bytes for i, (_, cfg, seed) in enumerate(reqs))
    server = SV.Server(budget_bytes=size, max_active=4)
    out = server.run(reqs, _make)
    assert out["peak_active"] == 1
    assert out["peak_bytes"] <= size
