"""Conjugate gradients (Algorithm 1) on a 7-point finite-difference operator.

The paper's CG iteration (Algorithm 1) is what the seven streaming
operations serve.  A CG solve needs an operator; this oracle uses the
7-point Laplacian with unit spacing plus a diagonal shift, on an m^3 grid of
unknowns with homogeneous Dirichlet ghost values (the operator the benchmark
configuration for mixed precision names: 6 + shift on the diagonal, -1 for
each of the six neighbours).  Unknown (i, j, k) has index i + m(j + m k).

stencil7 fixes the order of the additions so that a device kernel can match
it bit for bit: y = fl(c x_c), then subtract the neighbours at i-1, i+1,
j-1, j+1, k-1, k+1 in that order (absent neighbours skipped), with the
diagonal c = 6 + shift computed in binary64 and rounded once to the working
precision.

cg follows Algorithm 1 with x0 given, alpha = r.r / p.Ap, beta = r'.r'/r.r,
and stops on the true relative residual ||b - Ax|| / ||b|| <= tol (the
paper's test on r.r is replaced by this, recomputed from x at the end;
iteration stops on the recursive residual first).

ir_cg is the mixed-precision iterative refinement the benchmark
configuration describes: binary64 outer residual, correction and update;
inner CG on A d = r / ||r|| with vectors stored in binary32 or bfloat16 and
binary32 arithmetic, stopped at a fixed relative residual inner_tol (or
after max_inner iterations).  The scaled residual r / ||r|| is rounded once,
to nearest with ties to even, from binary64 to the storage type.  Inner
reductions are the correctly rounded exact sums of their terms.

round_storage rounds binary64 values to the nearest value of a storage
format given by its significand bits and exponent range (ties to even,
overflow to infinity), as the definition of round-to-nearest says: the
nearest multiple of the quantum of the value's binade.

TEST INFRASTRUCTURE ONLY: not part of the library path.
"""

import math

import numpy as np

__all__ = ["stencil7", "eigenvalue", "sine_mode", "cg", "ir_cg", "round_storage", "FORMATS"]


def stencil7(x, m, shift, dtype=np.float64):
    """y = (L + shift I) x with the fixed order of additions (see above)."""
    x = np.asarray(x, dtype=dtype).reshape(m, m, m)  # axes (k, j, i)
    c = dtype(6.0 + shift)  # diagonal, rounded once from binary64
    y = c * x
    for axis, side in ((2, -1), (2, 1), (1, -1), (1, 1), (0, -1), (0, 1)):
        nb = np.zeros_like(x)
        src = [slice(None)] * 3
        dst = [slice(None)] * 3
        if side == -1:   # neighbour at index - 1
            dst[axis] = slice(1, None)
            src[axis] = slice(None, -1)
        else:            # neighbour at index + 1
            dst[axis] = slice(None, -1)
            src[axis] = slice(1, None)
        nb[tuple(dst)] = x[tuple(src)]
        y = y - nb  # an absent neighbour subtracts +0.0, which leaves y unchanged
    return y.ravel()


def eigenvalue(m, shift, a, b, c):
    """Eigenvalue of the sine mode (a, b, c) in 1..m of the shifted operator."""
    th = lambda q: 2.0 - 2.0 * math.cos(q * math.pi / (m + 1))
    return th(a) + th(b) + th(c) + shift


def sine_mode(m, a, b, c):
    s = lambda q: np.sin(q * np.pi * np.arange(1, m + 1) / (m + 1))
    return np.einsum("k,j,i->kji", s(c), s(b), s(a)).ravel()


def cg_operator(apply, b, x0=None, tol=1e-10, max_iter=10000):
    """Algorithm 1 in binary64 for the symmetric positive definite operator
    `apply` (a function of a vector).  Returns (x, iterations, true relative
    residual)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    nb = math.sqrt(float(np.dot(b, b)))
    r = b - apply(x)
    p = r.copy()
    rr = float(np.dot(r, r))
    j = 0
    while j < max_iter and math.sqrt(rr) > tol * nb:
        Ap = apply(p)
        alpha = rr / float(np.dot(p, Ap))
        x = x + alpha * p
        r = r - alpha * Ap
        rr_new = float(np.dot(r, r))
        p = r + (rr_new / rr) * p
        rr = rr_new
        j += 1
    res = b - apply(x)
    return x, j, math.sqrt(float(np.dot(res, res))) / nb


def cg(b, m, shift, x0=None, tol=1e-10, max_iter=10000):
    """Algorithm 1 in binary64 on the shifted 7-point operator.  Returns (x,
    iterations, true relative residual)."""
    return cg_operator(lambda v: stencil7(v, m, shift), b, x0, tol, max_iter)


# significand bits (with the hidden bit), smallest normal exponent, largest finite value
FORMATS = {
    "f32": (24, -126, (2.0 - 2.0 ** -23) * 2.0 ** 127),
    "bf16": (8, -126, (2.0 - 2.0 ** -7) * 2.0 ** 127),
}


def round_storage(x, fmt):
    """Round binary64 values once to the nearest value of format fmt (ties to even).

    For |x| in the binade [2^e, 2^(e+1)) (e clamped below at the smallest
    normal exponent, where subnormals share its quantum) the representable
    values are the multiples of q = 2^(e + 1 - p); x / q is exact in
    binary64 and np.rint rounds it to the nearest integer, ties to even.
    Results above the largest finite value become infinities.  Returned as
    binary64 holding the rounded values.
    """
    p, emin, vmax = FORMATS[fmt]
    x = np.asarray(x, dtype=np.float64)
    _, ex = np.frexp(x)                     # |x| = m 2^ex, m in [0.5, 1)
    e = np.maximum(ex.astype(np.int64) - 1, emin)
    q_exp = e + 1 - p
    y = np.ldexp(np.rint(np.ldexp(x, -q_exp)), q_exp)
    y = np.where(np.abs(y) > vmax, np.copysign(np.inf, x), y)
    return np.where(np.isfinite(x), y, x)


def _store(x, fmt):
    """Rounded storage value of binary32 arithmetic results (held as binary32)."""
    x32 = np.asarray(x, dtype=np.float32)
    if fmt == "f32":
        return x32
    return round_storage(x32.astype(np.float64), fmt).astype(np.float32)


def _exact_dot(a, b):
    """Correctly rounded sum of the exact products a_i b_i (binary32 inputs)."""
    prod = np.asarray(a, dtype=np.float64) * np.asarray(b, dtype=np.float64)  # exact: 24 + 24 <= 53 bits
    return math.fsum(prod.tolist())


def ir_cg(b, m, shift, tol=1e-10, inner_tol=1e-4, max_inner=400, max_outer=50, inner="f32"):
    """Iterative refinement with an inner CG stored in `inner` ("f32" or "bf16").

    Returns (x, outer, inner iterations, true relative residual).  Steps:
    x = 0; repeat: r = b - A x and ||r|| in binary64; stop when
    ||r|| <= tol ||b|| (or after max_outer steps); r^ = r / ||r|| rounded to
    the storage type; CG on A d = r^ from d = 0 with every vector stored in
    that type, each vector operation computed in binary32 and rounded once
    to storage, alpha and beta from correctly rounded reductions, until
    ||r_j|| <= inner_tol ||r_0|| or max_inner iterations; x += ||r|| d in
    binary64.
    """
    if inner not in FORMATS:
        raise ValueError("inner must be 'f32' or 'bf16'")
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    nb = math.sqrt(float(np.dot(b, b)))
    outer = inner_its = 0
    while outer < max_outer:
        r = b - stencil7(x, m, shift)
        nr = math.sqrt(float(np.dot(r, r)))
        if nr <= tol * nb:
            break
        rl = round_storage(r / nr, inner).astype(np.float32)
        d = np.zeros_like(rl)
        p = rl.copy()
        rr = _exact_dot(rl, rl)
        stop = inner_tol * inner_tol * rr
        j = 0
        while j < max_inner and rr > stop:
            Ap = _store(stencil7(p, m, shift, dtype=np.float32), inner)
            alpha = np.float32(rr / _exact_dot(p, Ap))
            d = _store(d + alpha * p, inner)
            rl = _store(rl - alpha * Ap, inner)
            rr_new = _exact_dot(rl, rl)
            beta = np.float32(rr_new / rr)
            p = _store(np.float32(1.0) * rl + beta * p, inner)
            rr = rr_new
            j += 1
        inner_its += j
        x = x + nr * d.astype(np.float64)
        outer += 1
    res = b - stencil7(x, m, shift)
    return x, outer, inner_its, math.sqrt(float(np.dot(res, res))) / nb
