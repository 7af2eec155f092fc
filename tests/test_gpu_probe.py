"""The FMA probe behind the single-wave bound of small builds: one wave's time
per FMA, with 1 (dependent) and 2 or 4 (independent) chains per lane."""
import sys

import pytest

from paper_1304_6514_amd import nv

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-test]", *a, file=sys.__stderr__, flush=True)


@pytest.fixture(scope="module")
def torch():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    nv.load()
    return torch


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_probe_reports_a_plausible_time_per_fma(torch, precision):
    times = {}
    for chains in (1, 2, 4):
        ns, cyc = nv.nv_probe_fma_chains(precision, 1 << 20, chains)
        say(precision, chains, "chains:", round(ns, 3), "ns,", round(cyc, 3), "ticks per FMA")
        # one wave64 FMA takes a few clock ticks to issue; at 1-3 GHz that is
        # between a fraction of a nanosecond and a few tens of them
        assert 0.1 < ns < 50.0 and 1.0 < cyc < 100.0
        times[chains] = ns
    # more independent chains never make one FMA slower by more than the noise
    assert times[4] < 1.5 * times[1]
    # the single-chain call is the latency probe
    ns1, _ = nv.nv_probe_fma_latency(precision, 1 << 20)
    assert 0.5 * times[1] < ns1 < 2.0 * times[1]
