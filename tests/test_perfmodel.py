"""The library's model fit agrees with the oracle's (and so with Table 2)."""

import json
import os

import numpy as np

from oracle import model
from paper_2009_10917_amd import perfmodel

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table2_fischer_brown.json")


def test_fit_matches_oracle_on_noisy_data():
    rng = np.random.default_rng(1)
    B = np.geomspace(1e5, 3e10, 80)
    T = 6.1e-6 + B / 6.4e12
    T = T * (1 + 0.02 * rng.standard_normal(B.size))
    a0, aw = perfmodel.fit_time_model(B, T)
    b0, bw = model.fit(B, T)
    assert abs(a0 - b0) <= 1e-9 * abs(b0) + 1e-18 and abs(aw - bw) <= 1e-9 * bw


def test_fischer_brown_and_table2():
    g = json.load(open(GOLDEN))
    cols = g["table2"]["columns"]
    t0, w = g["table2"]["BS3"][cols.index("MI60")]
    assert abs(perfmodel.fischer_brown_bytes(t0 * 1e-6, w * 1e9) - model.fischer_brown(t0 * 1e-6, w * 1e9)) < 1e-3
    assert abs(perfmodel.effective_bandwidth(4 * 2e-6 * 5e12, 2e-6, 5e12) - 4e12) < 1e-3
