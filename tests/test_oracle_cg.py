"""Pins of the oracle's stencil operator and CG solvers."""

import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import bsgen
from oracle import cg


def kron_laplacian(m, shift):
    T = sp.diags([-np.ones(m - 1), 2 * np.ones(m), -np.ones(m - 1)], [-1, 0, 1])
    I = sp.identity(m)
    return (sp.kron(I, sp.kron(I, T)) + sp.kron(I, sp.kron(T, I)) + sp.kron(T, sp.kron(I, I))
            + shift * sp.identity(m ** 3)).tocsr()


@pytest.mark.parametrize("m", [1, 2, 3, 8, 13])
def test_stencil_is_the_kronecker_sum_laplacian(m):
    A = kron_laplacian(m, 0.01)
    # integer data with a dyadic shift: every sum is exact, so bits must agree
    x = bsgen.to_int(bsgen.raw(1, 1, 0, m ** 3), 200).astype(np.float64) - 100.0
    A2 = kron_laplacian(m, 0.5)
    assert np.array_equal(cg.stencil7(x, m, 0.5), A2 @ x)
    xr = bsgen.uniform(2, 1, m ** 3)
    assert np.allclose(cg.stencil7(xr, m, 0.01), A @ xr, rtol=0, atol=1e-13)


def test_stencil_order_of_additions():
    # centre term first, then neighbours in a fixed order: with a huge centre
    # value and tiny neighbours the rounding reveals the order
    m = 3
    x = np.zeros(27)
    centre = 1 + 3 + 9
    x[centre] = 2.0 ** 52 / 6.0
    for nb in (centre - 1, centre + 1, centre - 3, centre + 3, centre - 9, centre + 9):
        x[nb] = 0.75
    y = cg.stencil7(x, m, 0.0)
    acc = 6.0 * x[centre]
    for nb in (centre - 1, centre + 1, centre - 3, centre + 3, centre - 9, centre + 9):
        acc = acc - x[nb]
    assert y[centre] == acc
    assert y[centre] != 6.0 * x[centre] - 4.5


def test_sine_modes_are_eigenvectors_and_cg_converges_in_one_step():
    m = 9
    for a, b, c in ((1, 1, 1), (2, 5, 3), (9, 9, 9)):
        v = cg.sine_mode(m, a, b, c)
        lam = cg.eigenvalue(m, 0.01, a, b, c)
        assert np.allclose(cg.stencil7(v, m, 0.01), lam * v, rtol=0, atol=1e-12)
        x, it, res = cg.cg(v, m, 0.01, tol=1e-12)
        assert it == 1 and np.allclose(x, v / lam, rtol=0, atol=1e-13)


@pytest.mark.parametrize("m", [8, 16, 24])
def test_cg_agrees_with_direct_and_scipy_cg(m):
    A = kron_laplacian(m, 0.01)
    b = bsgen.uniform(10917, 10, m ** 3)
    x, it, res = cg.cg(b, m, 0.01, tol=1e-10)
    assert res <= 1e-10
    xd = spla.spsolve(A.tocsc(), b)
    assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)
    xs, info = spla.cg(A, b, rtol=1e-10, maxiter=10000)
    assert info == 0 and np.linalg.norm(x - xs) <= 1e-7 * np.linalg.norm(xd)


def test_cg_iteration_count_near_theory():
    m, shift = 48, 0.01
    kappa = cg.eigenvalue(m, shift, m, m, m) / cg.eigenvalue(m, shift, 1, 1, 1)
    b = bsgen.uniform(10917, 10, m ** 3)
    x, it, res = cg.cg(b, m, shift, tol=1e-10)
    bound = math.sqrt(kappa) * math.log(2 / 1e-10) / 2
    assert res <= 1e-10 and 0.4 * bound <= it <= 1.05 * bound


def test_ir_cg_reaches_binary64_accuracy():
    m = 20
    b = bsgen.uniform(10917, 10, m ** 3)
    x, outer, inner, res = cg.ir_cg(b, m, 0.01, tol=1e-10, inner_tol=1e-4)
    assert res <= 1e-10 and 2 <= outer <= 6
    xr, it, _ = cg.cg(b, m, 0.01, tol=1e-12)
    assert np.linalg.norm(x - xr) <= 1e-8 * np.linalg.norm(xr)


# ---------------------------------------------------------------- storage rounding of the refinement

def _nearest_exact(v, fmt):
    """Nearest value of the format by exact rational comparison (ties to the even significand)."""
    from fractions import Fraction
    p, emin, vmax = cg.FORMATS[fmt]
    if v == 0.0:
        return v
    a = Fraction(abs(v))
    e = max(math.frexp(abs(v))[1] - 1, emin)
    q = Fraction(2) ** (e + 1 - p)
    k = a / q
    lo = k.numerator // k.denominator
    rem = k - lo
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and lo % 2 == 1):
        lo += 1
    out = float(lo * q)
    if out > vmax:
        out = math.inf
    return math.copysign(out, v)


@pytest.mark.parametrize("fmt", ["f32", "bf16"])
def test_round_storage_is_nearest_ties_to_even(fmt):
    p = cg.FORMATS[fmt][0]
    rng = np.random.default_rng(7)
    vals = list(rng.standard_normal(400) * np.exp2(rng.integers(-140, 126, 400)))
    one = [1.0 + k * 2.0 ** -p for k in range(-4, 9)]          # ties and near-ties around 1
    vals += one + [-v for v in one] + [2.0 ** -130, 3 * 2.0 ** -135, 0.0, -0.0, 3.0e38, 3.4e38, 2.0 ** 128]
    got = cg.round_storage(np.array(vals), fmt)
    want = [_nearest_exact(v, fmt) for v in vals]
    assert np.array_equal(got, np.array(want))


def test_round_storage_f32_matches_the_hardware_conversion():
    x = bsgen.uniform(3, 1, 5000) * np.exp2(bsgen.to_int(bsgen.raw(3, 2, 0, 5000), 200).astype(np.float64) - 100)
    assert np.array_equal(cg.round_storage(x, "f32"), x.astype(np.float32).astype(np.float64))


def test_round_storage_bf16_of_binary32_matches_torch():
    # for binary32 inputs the library routine's bfloat16 conversion is the same single rounding
    import torch
    x32 = (bsgen.uniform(4, 1, 5000) * 3.0).astype(np.float32)
    ref = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(cg.round_storage(x32.astype(np.float64), "bf16"), ref)


def test_round_storage_bf16_rounds_binary64_once():
    # 1 + 2^-8 + 2^-30 lies above the tie between 1 and 1 + 2^-7; going through
    # binary32 first would drop 2^-30, land on the tie and round down to 1
    x = 1.0 + 2.0 ** -8 + 2.0 ** -30
    assert cg.round_storage(np.array([x]), "bf16")[0] == 1.0 + 2.0 ** -7
    twice = cg.round_storage(cg.round_storage(np.array([x]), "f32"), "bf16")[0]
    assert twice == 1.0


@pytest.mark.parametrize("inner,tau", [("f32", 1e-4), ("bf16", 0.1)])
def test_ir_cg_eigenvector_rhs(inner, tau):
    # b a sine mode: every inner CG ends after one iteration with d = b^/lambda
    # (up to storage rounding), and refinement drives the binary64 error down
    m = 11
    v = cg.sine_mode(m, 3, 1, 4)
    lam = cg.eigenvalue(m, 0.01, 3, 1, 4)
    x, outer, inner_its, res = cg.ir_cg(v, m, 0.01, tol=1e-12, inner_tol=tau, inner=inner)
    assert res <= 1e-12
    assert np.allclose(x, v / lam, rtol=0, atol=1e-12 * np.abs(v / lam).max())
    # the inner solve of the first step is a single iteration (modes stay modes up to rounding)
    x1, o1, i1, _ = cg.ir_cg(v, m, 0.01, tol=1e-12, inner_tol=tau, inner=inner, max_outer=1)
    assert o1 == 1 and i1 <= 3


def test_ir_cg_bfloat16_inner_reaches_binary64_accuracy():
    m = 20
    b = bsgen.uniform(10917, 10, m ** 3)
    x, outer, inner, res = cg.ir_cg(b, m, 0.01, tol=1e-10, inner_tol=0.1, inner="bf16")
    assert res <= 1e-10 and outer >= 3
    xr, _, _ = cg.cg(b, m, 0.01, tol=1e-12)
    kappa = cg.eigenvalue(m, 0.01, m, m, m) / cg.eigenvalue(m, 0.01, 1, 1, 1)
    assert np.linalg.norm(x - xr) <= kappa * 1e-10 * np.linalg.norm(xr)


def test_ir_cg_fixed_inner_tolerance_sets_the_contraction():
    # each refinement step solves to a fixed relative residual tau, so the outer
    # residual falls by roughly tau per step (binary32 storage adds u32 kappa)
    m = 16
    b = bsgen.uniform(10917, 10, m ** 3)
    res = [cg.ir_cg(b, m, 0.01, tol=1e-14, inner_tol=1e-3, max_outer=k)[3] for k in (1, 2, 3)]
    kappa = cg.eigenvalue(m, 0.01, m, m, m) / cg.eigenvalue(m, 0.01, 1, 1, 1)
    for k in range(3):
        assert res[k] <= (1e-3 + kappa * 2.0 ** -24) ** (k + 1) * 3
