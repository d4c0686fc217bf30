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
inner CG on A d = r / ||r|| with vectors stored in binary32, stopped at a
relative residual theta = max(inner_tol, 0.5 tol ||b|| / ||r||): the looser
value applies when it already meets the outer target, so the last step is
not solved further than needed.

TEST INFRASTRUCTURE ONLY: not part of the library path.
"""

import math

import numpy as np

__all__ = ["stencil7", "eigenvalue", "sine_mode", "cg", "ir_cg"]


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


def cg(b, m, shift, x0=None, tol=1e-10, max_iter=10000):
    """Algorithm 1 in binary64.  Returns (x, iterations, true relative residual)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    nb = math.sqrt(float(np.dot(b, b)))
    r = b - stencil7(x, m, shift)
    p = r.copy()
    rr = float(np.dot(r, r))
    j = 0
    while j < max_iter and math.sqrt(rr) > tol * nb:
        Ap = stencil7(p, m, shift)
        alpha = rr / float(np.dot(p, Ap))
        x = x + alpha * p
        r = r - alpha * Ap
        rr_new = float(np.dot(r, r))
        p = r + (rr_new / rr) * p
        rr = rr_new
        j += 1
    res = b - stencil7(x, m, shift)
    return x, j, math.sqrt(float(np.dot(res, res))) / nb


def ir_cg(b, m, shift, tol=1e-10, inner_tol=1e-4, max_inner=400, max_outer=50):
    """Iterative refinement with binary32 inner CG.  Returns (x, outer, inner, relres)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    nb = math.sqrt(float(np.dot(b, b)))
    outer = inner = 0
    while outer < max_outer:
        r = b - stencil7(x, m, shift)
        nr = math.sqrt(float(np.dot(r, r)))
        if nr <= tol * nb:
            break
        theta = max(inner_tol, 0.5 * tol * nb / nr)
        rh = (r / nr).astype(np.float32)
        d = np.zeros_like(rh)
        rl = rh.copy()
        p = rl.copy()
        rr = np.float32(np.dot(rl.astype(np.float64), rl.astype(np.float64)))
        rr0 = rr
        j = 0
        while j < max_inner and math.sqrt(float(rr)) > theta * math.sqrt(float(rr0)):
            Ap = stencil7(p, m, shift, dtype=np.float32)
            alpha = np.float32(rr / np.float32(np.dot(p.astype(np.float64), Ap.astype(np.float64))))
            d = (d + alpha * p).astype(np.float32)
            rl = (rl - alpha * Ap).astype(np.float32)
            rr_new = np.float32(np.dot(rl.astype(np.float64), rl.astype(np.float64)))
            p = (rl + np.float32(rr_new / rr) * p).astype(np.float32)
            rr = rr_new
            j += 1
        inner += j
        x = x + nr * d.astype(np.float64)
        outer += 1
    res = b - stencil7(x, m, shift)
    return x, outer, inner, math.sqrt(float(np.dot(res, res))) / nb
