"""Launch-latency + bandwidth model of the streaming operations (Section 4).

A call that moves B bytes takes T(B) = T0 + B / W_max (eq. time_model), so
its effective bandwidth is B / T(B) (eq. perf_model), and 80 % of W_max is
reached at B_0.8 = 4 T0 W_max bytes (eq. Fischer-Brown).  T0 and W_max come
from a least-squares straight line through measured (bytes, seconds) pairs
(Section 6), computed here from the closed-form normal equations.
"""


def fit_time_model(bytes_moved, seconds):
    """Least-squares T = T0 + B/W over the points; returns (T0 [s], W [B/s])."""
    B = [float(b) for b in bytes_moved]
    T = [float(t) for t in seconds]
    n = len(B)
    if n < 2 or n != len(T):
        raise ValueError("need at least two (bytes, seconds) points of equal count")
    mb = sum(B) / n
    mt = sum(T) / n
    sbb = sum((b - mb) * (b - mb) for b in B)
    sbt = sum((b - mb) * (t - mt) for b, t in zip(B, T))
    if sbb == 0.0:
        raise ValueError("all points move the same number of bytes")
    slope = sbt / sbb
    t0 = mt - slope * mb
    return t0, (1.0 / slope if slope > 0 else float("inf"))


def effective_bandwidth(B, t0, w_max):
    """B / (T0 + B / W_max), in the units of w_max."""
    return B / (t0 + B / w_max)


def fischer_brown_bytes(t0, w_max):
    """Bytes at which the model reaches 80 % of W_max: 4 T0 W_max."""
    return 4.0 * t0 * w_max
