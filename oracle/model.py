"""Launch-latency + bandwidth model of Section 4.

T(B) = T0 + B / W_max                (eq. time_model)
W_eff(B) = B / (T0 + B / W_max)      (eq. perf_model)
B_0.8 = 4 T0 W_max                   (eq. Fischer-Brown)

T0 and W_max come from an ordinary least-squares straight-line fit of the
measured times against bytes moved (Section 6).

TEST INFRASTRUCTURE ONLY: not part of the library path.
"""

import numpy as np


def fit(bytes_moved, seconds):
    """Least-squares fit of T = T0 + B/W.  Returns (T0 [s], W_max [B/s])."""
    B = np.asarray(bytes_moved, dtype=np.float64)
    T = np.asarray(seconds, dtype=np.float64)
    A = np.stack([np.ones_like(B), B], axis=1)
    (t0, slope), *_ = np.linalg.lstsq(A, T, rcond=None)
    return float(t0), float(1.0 / slope)


def effective_bandwidth(B, t0, w_max):
    """W_eff(B) of eq. perf_model, in the units of w_max."""
    B = np.asarray(B, dtype=np.float64)
    return B / (t0 + B / w_max)


def fischer_brown(t0, w_max):
    """Bytes needed to reach 80 % of W_max: 4 T0 W_max."""
    return 4.0 * t0 * w_max
