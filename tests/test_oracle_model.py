"""Pins of the performance-model fit (Section 4) against the paper's numbers."""

import json
import os

import numpy as np

from oracle import model

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table2_fischer_brown.json")


def test_fit_recovers_parameters_exactly():
    t0, w = 7.5e-6, 5.2e12
    B = np.geomspace(1e4, 4e10, 60)
    T = t0 + B / w
    f0, fw = model.fit(B, T)
    assert abs(f0 - t0) <= 1e-9 * t0 + 1e-15
    assert abs(fw - w) <= 1e-9 * w


def test_effective_bandwidth_reaches_80_percent_at_fischer_brown_point():
    t0, w = 3e-6, 8e12
    b08 = model.fischer_brown(t0, w)
    assert abs(model.effective_bandwidth(b08, t0, w) - 0.8 * w) <= 1e-6 * w
    assert model.effective_bandwidth(1e15, t0, w) > 0.999 * w
    # at B = T0 * W the device runs at exactly half speed
    assert abs(model.effective_bandwidth(t0 * w, t0, w) - 0.5 * w) <= 1e-6 * w


def test_fischer_brown_reproduces_paper_worked_example():
    # The paper's BS3 example quotes B_0.8 for the V100 and MI60 in MB and in
    # millions of doubles.  4*T0*W_max from Table 2 gives those numbers when
    # microsecond*GB/s is read as KiB (factor 1.024); in SI bytes it is
    # 24.66e6 and 57.29e6.
    g = json.load(open(GOLDEN))
    cols = g["table2"]["columns"]
    for gpu in ("V100", "MI60"):
        t0_us, w_gbs = g["table2"]["BS3"][cols.index(gpu)]
        b = model.fischer_brown(t0_us * 1e-6, w_gbs * 1e9)
        printed = g["fischer_brown_BS3"][gpu]
        assert round(b * 1.024 / 2**20, 1) == round(printed["MB"], 1) or round(b * 1.024 / 2**20) == printed["MB"]
        assert round(b * 1.024 / 8 / 1e6, 2) == printed["M_doubles"]
    v100 = g["table2"]["BS3"][cols.index("V100")]
    assert round(model.fischer_brown(v100[0] * 1e-6, v100[1] * 1e9) / 1e6, 2) == 24.66


def test_fit_on_table2_model_curves_returns_table2():
    g = json.load(open(GOLDEN))
    for test, rows in g["table2"].items():
        if test == "columns":
            continue
        for t0_us, w_gbs in rows:
            B = np.linspace(1e6, 2e9, 40)
            T = t0_us * 1e-6 + B / (w_gbs * 1e9)
            f0, fw = model.fit(B, T)
            assert abs(f0 * 1e6 - t0_us) < 1e-6 and abs(fw / 1e9 - w_gbs) < 1e-6
