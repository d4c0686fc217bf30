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
