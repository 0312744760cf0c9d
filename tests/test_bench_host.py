"""Host-side arithmetic of bench.py: algorithmic flop counts per Gray term,
the repeated-row flop model, and the traffic gate (no GPU)."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.abspath(os.path.join(os.path.dirname(__file__), ".."))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_flops_per_term_unit_multiplicities():
    # n complex adds, n - 1 complex multiplies and one accumulate: 8n - 4
    assert [bench.flops_per_term(n) for n in (24, 28, 30, 32)] == [188, 220, 236, 252]


def test_traffic_gate():
    # other sizes have no counters; at n = 30 the figure is either the
    # calibrated one (sources unchanged since the counters) or None
    assert bench.sweep_traffic_bytes(28) is None
    v = bench.sweep_traffic_bytes(30)
    t = bench.SWEEP_TRAFFIC
    want = 1024.0 * (t["fetch_kib"] * t["fetch_factor"] + t["write_kib"] * t["write_factor"])
    assert v is None or v == pytest.approx(want)
    assert want == pytest.approx(545_113, abs=1)


def test_repeated_flops_model():
    pytest.importorskip("torch")
    # unit multiplicities on both sides: n - 1 joins nominally; the grouped
    # product runs c - 1 + max kappa = n multiplies (its first one is by 1)
    n = 6
    S = [1] * n
    nominal, executed = bench.repeated_flops(S, S)
    terms = 2 ** (n - 1)
    assert nominal == terms * (2 * n + 6 * (n - 1) + 4)
    assert executed == terms * (2 * n + 6 * n + 4)
    # powers (1, 2, 4) on the power side: nominal multiplies 0 + 1 + 2 per
    # column (squaring) plus 2 joins; the grouped product c - 1 + max kappa
    # = 2 + 4 (one multiply per unit of rise, so more than squaring here)
    S = [1, 2, 4]
    T = [7, 0, 0]
    nominal, executed = bench.repeated_flops(S, T)
    import paper_2403_04006_amd as pq
    info = pq.plan_describe(S, T)
    pw = np.asarray(T if info["transposed"] else S)
    kap = sorted(int(k) for k in pw[pw > 0])
    c = len(kap)
    pm = {1: 0, 2: 1, 3: 2, 4: 2}
    assert nominal == info["terms"] * (2 * c + 6 * (sum(pm[k] for k in kap) + c - 1) + 4)
    assert executed == info["terms"] * (2 * c + 6 * (c - 1 + max(kap)) + 4)
    # many columns of one power: grouping needs fewer multiplies than
    # squaring each column (10 columns of power 2: 9 + 2 against 10 + 9)
    S = [2] * 10
    T = [20] + [0] * 9
    nominal, executed = bench.repeated_flops(S, T)
    assert not pq.plan_describe(S, T)["transposed"]     # the powers are S's
    assert executed < nominal
