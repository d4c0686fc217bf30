"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module holds no arithmetic of the streaming operations themselves: it
only produces input values (vectors, scalars, element permutations and
orientation choices) from a seed.  Both sides of every parity check draw from
it; the oracle uses the numpy form below and the GPU tests may use the device
form in ``bsgen/csrc/bsgen.hip``, which implements the same published
generator and is checked bit-for-bit against this one.

Generator: the SplitMix64 output function F and its odd "golden gamma"
increment (Steele, Lea & Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014).  Value ``i`` of stream ``k`` under seed ``S`` is

    x[k, i] = F(key(S, k) + (i + 1) * GAMMA)   (mod 2**64)
    key(S, k) = F(S xor F(k))

so any index range of any stream can be regenerated independently, on the
host or on the device.

Derived draws:
  * uniform [0, 1):   (x >> 11) * 2**-53
  * uniform [-1, 1):  2u - 1 (exact in binary64)
  * integer [0, m):   ((x >> 32) * m) >> 32, for 0 < m < 2**32
  * permutation of E items: Fisher-Yates from s = E-1 down to 1, swapping
    slot s with slot j = integer(draw s, s + 1)
  * orientation of element slot s: integer(draw s, 24)
"""

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK64 = (1 << 64) - 1

DEFAULT_SEED = 10917

# Stream ids: one per input role.
STREAM = {
    "x": 1, "y": 2, "p": 3, "r": 4, "Ap": 5, "w": 6, "scalars": 7,
    "perm": 8, "orient": 9, "b": 10, "xL": 11, "xG": 12,
    "inst_E": 13, "inst_N": 14,
}


def _mix_int(z: int) -> int:
    """SplitMix64 output function on a Python int (mod 2**64)."""
    z &= _MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def _mix(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function on a uint64 array (wrapping arithmetic)."""
    z = z ^ (z >> np.uint64(30))
    z = z * _M1
    z = z ^ (z >> np.uint64(27))
    z = z * _M2
    return z ^ (z >> np.uint64(31))


def stream_key(seed: int, stream: int) -> int:
    """key(S, k) = F(S xor F(k))."""
    return _mix_int((seed & _MASK64) ^ _mix_int(stream))


def raw(seed: int, stream: int, start: int, count: int) -> np.ndarray:
    """Raw 64-bit draws i = start .. start+count-1 of one stream."""
    key = np.uint64(stream_key(seed, stream))
    i = np.arange(start + 1, start + 1 + count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix(key + i * GAMMA)


def raw_at(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    """Raw draws at arbitrary indices (for sampled checks of huge vectors)."""
    key = np.uint64(stream_key(seed, stream))
    i = np.asarray(idx, dtype=np.uint64) + np.uint64(1)
    with np.errstate(over="ignore"):
        return _mix(key + i * GAMMA)


def to_unit(x: np.ndarray) -> np.ndarray:
    """uniform [0, 1) from raw draws: top 53 bits times 2**-53."""
    return (x >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def to_sym(x: np.ndarray) -> np.ndarray:
    """uniform [-1, 1) from raw draws: 2u - 1."""
    return 2.0 * to_unit(x) - 1.0


def to_int(x: np.ndarray, m: int) -> np.ndarray:
    """integer in [0, m) from raw draws (multiply-shift on the top 32 bits)."""
    if not (0 < m < (1 << 32)):
        raise ValueError("m must lie in (0, 2**32)")
    hi = x >> np.uint64(32)
    return ((hi * np.uint64(m)) >> np.uint64(32)).astype(np.int64)


_CHUNK = 1 << 22


def uniform(seed: int, stream: int, n: int, lo: float = -1.0, start: int = 0) -> np.ndarray:
    """n float64 draws, uniform [-1,1) when lo == -1 else uniform [0,1)."""
    if lo not in (-1.0, 0.0):
        raise ValueError("lo must be -1.0 or 0.0")
    out = np.empty(n, dtype=np.float64)
    conv = to_sym if lo == -1.0 else to_unit
    for a in range(0, n, _CHUNK):
        b = min(n, a + _CHUNK)
        out[a:b] = conv(raw(seed, stream, start + a, b - a))
    return out


def uniform_at(seed: int, stream: int, idx: np.ndarray, lo: float = -1.0) -> np.ndarray:
    conv = to_sym if lo == -1.0 else to_unit
    return conv(raw_at(seed, stream, idx))


def scalars(seed: int, tag: int, count: int = 2) -> np.ndarray:
    """uniform [0,1) scalars (alpha, beta, ...) for one size tag."""
    return to_unit(raw(seed, STREAM["scalars"], tag * 16, count))


def permutation(seed: int, n: int) -> np.ndarray:
    """Fisher-Yates permutation of range(n) from the 'perm' stream."""
    perm = np.arange(n, dtype=np.int64)
    if n <= 1:
        return perm
    draws = raw(seed, STREAM["perm"], 0, n)
    # partner for slot s uses draw s; integers computed up front, swaps in order
    hi = (draws >> np.uint64(32)).astype(np.uint64)
    bound = np.arange(n, dtype=np.uint64) + np.uint64(1)
    with np.errstate(over="ignore"):
        partner = ((hi * bound) >> np.uint64(32)).astype(np.int64)
    p = perm.tolist()
    part = partner.tolist()
    for s in range(n - 1, 0, -1):
        j = part[s]
        p[s], p[j] = p[j], p[s]
    return np.asarray(p, dtype=np.int64)


def orientations(seed: int, n: int) -> np.ndarray:
    """Orientation index in [0, 24) for each of n element slots."""
    return to_int(raw(seed, STREAM["orient"], 0, n), 24)


def batch_instances(seed: int, n: int):
    """Descriptors of n independent instances: element counts E_i and degrees N_i.

    E_i = round(2**(12 u)) with u uniform [0, 1) (log-uniform on [1, 4096]),
    N_i uniform in {2, ..., 8}.  Returns two int64 arrays.
    """
    u = to_unit(raw(seed, STREAM["inst_E"], 0, n))
    E = np.rint(np.exp2(12.0 * u)).astype(np.int64)
    N = 2 + to_int(raw(seed, STREAM["inst_N"], 0, n), 7)
    return E, N


def round_f32(x: np.ndarray) -> np.ndarray:
    """binary64 -> binary32, round to nearest even (numpy's cast)."""
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def round_bf16_bits(x: np.ndarray) -> np.ndarray:
    """binary64 -> binary32 (RNE) -> bfloat16 (RNE); returns uint16 bit patterns.

    NaN inputs are not produced by this generator and are not handled.
    """
    f = round_f32(x).view(np.uint32).astype(np.uint64)
    lsb = (f >> np.uint64(16)) & np.uint64(1)
    r = (f + np.uint64(0x7FFF) + lsb) >> np.uint64(16)
    return r.astype(np.uint16)


def bf16_bits_to_f64(b: np.ndarray) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------- device form

_DEVLIB = None


def _devlib():
    global _DEVLIB
    if _DEVLIB is None:
        import ctypes
        import os

        import torch  # noqa: F401  (bind to torch's HIP runtime, loaded first)
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libbsgen.so")
        if not os.path.exists(path):
            raise ImportError(f"{path} is not built (python paper_2009_10917_amd/build.py)")
        lib = ctypes.CDLL(path)
        lib.bsgen_uniform.restype = ctypes.c_int
        lib.bsgen_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64,
                                      ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
        _DEVLIB = lib
    return _DEVLIB


def device_uniform(out, seed, stream, lo=-1.0, start=0, hip_stream=None):
    """Fill a contiguous device tensor with values start.. of one stream.

    float64 tensors get the binary64 draws; float32 and bfloat16 tensors get
    them rounded (binary64 -> binary32 -> bfloat16, nearest even), exactly
    as ``round_f32`` / ``round_bf16_bits`` do on the host.
    """
    import torch
    codes = {torch.float64: 0, torch.float32: 1, torch.bfloat16: 2}
    if out.dtype not in codes or not out.is_contiguous() or not out.is_cuda:
        raise ValueError("device_uniform needs a contiguous float64/float32/bfloat16 device tensor")
    if lo not in (-1.0, 0.0):
        raise ValueError("lo must be -1.0 or 0.0")
    hs = torch.cuda.current_stream().cuda_stream if hip_stream is None else hip_stream
    rc = _devlib().bsgen_uniform(seed & _MASK64, stream, start, out.numel(), 1 if lo == -1.0 else 0,
                                 codes[out.dtype], out.data_ptr(), hs)
    if rc != 0:
        raise RuntimeError(f"bsgen_uniform failed with HIP error {rc}")
    return out
