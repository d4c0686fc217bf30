"""Pins of the oracle's seven operations against what mathematics fixes.

None of these retypes the oracle's own formula: each compares it with exact
rational arithmetic, a closed form, an invariant or a hand-made case whose
answer is known in advance.
"""

from fractions import Fraction

import numpy as np
import pytest

import bsgen
from oracle import mesh, ops

U = 2.0 ** -53


def _exact(vals):
    return sum((Fraction(float(v)) for v in vals), Fraction(0))


# ---------------------------------------------------------------- copy (BS1)

def test_copy_bits_including_signed_zero_and_nan_payload():
    x = np.array([0.0, -0.0, 1.5, np.inf, -np.inf], dtype=np.float64)
    nan_bits = np.array([0x7FF8000000000ABC, 0xFFF0000000000001], dtype=np.uint64)
    x = np.concatenate([x, nan_bits.view(np.float64)])
    y = ops.copy(x)
    assert np.array_equal(x.view(np.uint64), y.view(np.uint64))
    assert y is not x


# ---------------------------------------------------------------- axpy (BS2)

def test_axpy_exact_on_dyadic_data():
    # few-bit dyadic values: every product and sum is exact, so the result is
    # the exact rational alpha*x + beta*y
    rng = np.random.default_rng(0)
    x = rng.integers(-64, 64, 1000) / 8.0
    y = rng.integers(-64, 64, 1000) / 16.0
    out = ops.axpy(0.375, x, -1.25, y)
    ref = [float(Fraction(3, 8) * Fraction(a) + Fraction(-5, 4) * Fraction(b)) for a, b in zip(x, y)]
    assert np.array_equal(out, np.array(ref))


def test_axpy_within_rounding_bound_and_operand_order():
    x = bsgen.uniform(5, 1, 2000)
    y = bsgen.uniform(5, 2, 2000)
    a, b = 0.37, 1.0
    out = ops.axpy(a, x, b, y)
    for xi, yi, oi in zip(x, y, out):
        exact = Fraction(a) * Fraction(xi) + Fraction(b) * Fraction(yi)
        bound = (2 * U + U * U) * (abs(a * xi) + abs(b * yi))
        assert abs(Fraction(oi) - exact) <= Fraction(bound)
    # swapping the roles of x and y (or of alpha and beta) must change it
    assert not np.array_equal(out, ops.axpy(a, y, b, x))
    assert not np.array_equal(out, ops.axpy(b, x, a, y))


def test_axpy_is_two_products_and_one_sum():
    # alpha*x = (1 + 2^-30)^2 = 1 + 2^-29 + 2^-60 rounds to 1 + 2^-29, which
    # beta*y cancels exactly: separately rounded products give 0, whereas a
    # fused multiply-add keeps the 2^-60 term
    a = 1.0 + 2.0**-30
    out = ops.axpy(a, np.array([a]), -1.0, np.array([1.0 + 2.0**-29]))
    assert out[0] == 0.0
    exact = Fraction(a) * Fraction(a) - Fraction(1.0 + 2.0**-29)
    assert exact == Fraction(1, 2**60)


# ---------------------------------------------------------------- norm (BS3)

def test_norm_matches_exact_rational_sum():
    for n in (1, 7, 1000, 10000):
        x = bsgen.uniform(9, 1, n)
        terms = x * x
        assert ops.norm(x) == float(_exact(terms))
        w = bsgen.uniform(9, 6, n, lo=0.0)
        assert ops.norm(x, w) == float(_exact(w * terms))


def test_norm_constant_vector_closed_form():
    for n in (1, 3, 1000, 123457):
        for c in (1.0, 0.5, -3.0, 2.0 ** -20):
            assert ops.norm(np.full(n, c)) == n * c * c


def test_norm_is_squared_not_sqrt():
    assert ops.norm(np.array([3.0, 4.0])) == 25.0


def test_empty_reductions_are_zero():
    e = np.zeros(0)
    assert ops.norm(e) == 0.0 and ops.dot(e, e) == 0.0


def test_weighted_norm_of_ones_is_global_node_count():
    # weights 1/deg are dyadic on a structured mesh, so the sum is exact
    for K, N in ((8, 3), (3, 1), (2, 7), (4, 5)):
        E, NL, NG = mesh.sizes(K, N)
        ids = mesh.hex_map(K, N)
        w = mesh.weights(ids, NG)
        assert ops.norm(np.ones(NL), w) == float(NG)
    E, NL, NG = mesh.sizes(8, 3)
    assert NG == 15625 and NL == 32768


def test_weighted_local_norm_equals_global_norm():
    K, N = 5, 3
    E, NL, NG = mesh.sizes(K, N)
    perm = bsgen.permutation(2, E)
    orient = bsgen.orientations(2, E)
    ids = mesh.hex_map(K, N, perm, orient)
    w = mesh.weights(ids, NG)
    xG = bsgen.uniform(2, 12, NG)
    xL = ops.scatter(ids, xG, np.zeros(NL))
    assert abs(ops.norm(xL, w) - ops.norm(xG)) <= 1e-14 * ops.norm(xG)


# ---------------------------------------------------------------- dot (BS4)

def test_two_product_is_exact():
    a = bsgen.uniform(4, 1, 3000)
    b = bsgen.uniform(4, 2, 3000) * 1e3
    p, e = ops.two_product(a, b)
    for ai, bi, pi, ei in zip(a, b, p, e):
        assert Fraction(pi) + Fraction(ei) == Fraction(ai) * Fraction(bi)


def test_dot_matches_exact_rational_sum():
    for n in (1, 2, 10, 5000):
        x = bsgen.uniform(13, 1, n)
        y = bsgen.uniform(13, 2, n)
        ref = sum((Fraction(a) * Fraction(b) for a, b in zip(x, y)), Fraction(0))
        assert ops.dot(x, y) == float(ref)


def test_dot_under_cancellation():
    # x.y = 1 exactly although the terms are ~1e16: a naive float sum fails
    x = np.array([1e16, 1.0, -1e16, 1.0])
    y = np.array([1.0, 0.5, 1.0, 0.5])
    assert ops.dot(x, y) == 1.0
    assert sum(x * y) != 1.0


def test_dot_self_equals_norm():
    x = bsgen.uniform(21, 1, 50000)
    d, nrm = ops.dot(x, x), ops.norm(x)
    assert abs(d - nrm) <= 1e-14 * nrm


def test_dot_ones_with_coordinate_is_half_node_count():
    # the GLL lattice is symmetric about 1/2 on [0, 1], so the coordinates
    # of all global nodes sum to N_G / 2
    K, N = 6, 5
    E, NL, NG = mesh.sizes(K, N)
    M = K * N + 1
    r = _gll(N)
    one_d = np.concatenate([(q + (1.0 + r[:-1]) / 2.0) / K for q in range(K)] + [np.array([1.0])])
    assert one_d.size == M
    X = np.tile(one_d, M * M)
    assert abs(ops.dot(np.ones(NG), X) - NG / 2.0) <= 1e-14 * NG / 2.0


def _gll(N):
    from numpy.polynomial import legendre
    inner = legendre.Legendre.basis(N).deriv().roots() if N > 1 else np.zeros(0)
    return np.concatenate([[-1.0], np.sort(inner.real), [1.0]])


# ---------------------------------------------------------------- fused CG update (BS5)

def test_cg_update_alpha_zero_leaves_vectors_bit_unchanged():
    n = 4097
    x, p, r, Ap = (bsgen.uniform(3, s, n) for s in (1, 3, 4, 5))
    w = bsgen.uniform(3, 6, n, lo=0.0)
    xn, rn, rho = ops.cg_update(0.0, x, p, r, Ap, w)
    assert np.array_equal(xn, x) and np.array_equal(rn, r)
    assert rho == float(_exact(w * (r * r)))


def test_cg_update_constant_closed_form():
    n = 1000
    xn, rn, rho = ops.cg_update(0.5, np.ones(n), np.full(n, 2.0), np.full(n, 3.0), np.full(n, 4.0))
    assert np.all(xn == 2.0) and np.all(rn == 1.0) and rho == float(n)
    w = np.full(n, 0.25)
    assert ops.cg_update(0.5, np.ones(n), np.full(n, 2.0), np.full(n, 3.0), np.full(n, 4.0), w)[2] == n / 4.0


def test_cg_update_against_exact_and_sign():
    n = 3000
    a = 0.37
    x, p, r, Ap = (bsgen.uniform(8, s, n) for s in (1, 3, 4, 5))
    xn, rn, rho = ops.cg_update(a, x, p, r, Ap)
    for i in range(0, n, 7):
        ex = Fraction(x[i]) + Fraction(a) * Fraction(p[i])
        er = Fraction(r[i]) - Fraction(a) * Fraction(Ap[i])
        assert abs(Fraction(xn[i]) - ex) <= Fraction((2 * U) * (abs(x[i]) + abs(a * p[i])))
        assert abs(Fraction(rn[i]) - er) <= Fraction((2 * U) * (abs(r[i]) + abs(a * Ap[i])))
    # rho is taken over the stored new residual
    assert rho == float(_exact(rn * rn))
    assert rho != ops.norm(r)


# ---------------------------------------------------------------- gather / scatter (BS6, BS7)

def test_scatter_masked_entries_untouched():
    ids = np.array([2, -1, 0, 2, -5, 1])
    xG = np.array([10.0, 11.0, 12.0])
    old = np.array([-1.0, -2.0, -3.0, -4.0, -5.0, -6.0])
    out = ops.scatter(ids, xG, old)
    assert list(out) == [12.0, -2.0, 10.0, 12.0, -5.0, 11.0]


def test_gather_order_and_initial_value():
    # row 0 copies (ascending l): 1, 2^-53, 2^-53 -> ((0+1)+u)+u = 1 exactly,
    # whereas summing the small terms first gives 1 + 2^-52.
    # row 1: all -0.0 -> +0.0 (the sum starts from +0.0).  row 2: no copies.
    ids = np.array([0, 1, 0, -1, 0, 1])
    xL = np.array([1.0, -0.0, 2.0**-53, 7.0, 2.0**-53, -0.0])
    rs, ci = mesh.csr_inverse(ids, 3)
    assert list(rs) == [0, 3, 5, 5] and list(ci) == [0, 2, 4, 1, 5]
    g = ops.gather(rs, ci, xL)
    assert g[0] == 1.0
    assert g[1] == 0.0 and not np.signbit(g[1])
    assert g[2] == 0.0 and not np.signbit(g[2])
    # reversed local order changes the result: the order is part of the definition
    xL_rev = np.array([2.0**-53, -0.0, 2.0**-53, 7.0, 1.0, -0.0])
    assert ops.gather(rs, ci, xL_rev)[0] == 1.0 + 2.0**-52


@pytest.mark.parametrize("K,N", [(2, 1), (3, 2), (2, 3), (3, 3)])
def test_gather_dense_bruteforce(K, N):
    E, NL, NG = mesh.sizes(K, N)
    perm = bsgen.permutation(K * 10 + N, E)
    orient = bsgen.orientations(K * 10 + N, E)
    ids = mesh.hex_map(K, N, perm, orient)
    Z = np.zeros((NL, NG))
    Z[np.arange(NL), ids] = 1.0
    assert np.all(Z.sum(axis=1) == 1.0)
    deg = mesh.degree(ids, NG)
    assert np.array_equal(Z.T @ Z, np.diag(deg.astype(np.float64)))
    xL = bsgen.to_int(bsgen.raw(1, 11, 0, NL), 2000).astype(np.float64) - 1000.0
    rs, ci = mesh.csr_inverse(ids, NG)
    assert np.array_equal(ops.gather(rs, ci, xL), Z.T @ xL)
    xG = bsgen.uniform(1, 12, NG)
    assert np.array_equal(ops.scatter(ids, xG, np.zeros(NL)), Z @ xG)


def test_gather_of_scatter_is_degree_times_field():
    K, N = 6, 4
    E, NL, NG = mesh.sizes(K, N)
    ids = mesh.hex_map(K, N, bsgen.permutation(4, E), bsgen.orientations(4, E))
    rs, ci = mesh.csr_inverse(ids, NG)
    deg = mesh.degree(ids, NG)
    ones = ops.scatter(ids, np.ones(NG), np.zeros(NL))
    assert np.array_equal(ops.gather(rs, ci, ones), deg.astype(np.float64))
    f = bsgen.to_int(bsgen.raw(4, 12, 0, NG), 512).astype(np.float64) / 64.0 - 4.0
    fl = ops.scatter(ids, f, np.zeros(NL))
    assert np.array_equal(ops.gather(rs, ci, fl), deg * f)


def test_gather_invariant_under_element_permutation_and_orientation():
    K, N = 4, 3
    E, NL, NG = mesh.sizes(K, N)
    f = bsgen.to_int(bsgen.raw(6, 12, 0, NG), 100).astype(np.float64)
    results = []
    for seed in (0, 1, 2):
        perm = np.arange(E) if seed == 0 else bsgen.permutation(seed, E)
        orient = np.zeros(E, dtype=np.int64) if seed == 0 else bsgen.orientations(seed, E)
        ids = mesh.hex_map(K, N, perm, orient)
        rs, ci = mesh.csr_inverse(ids, NG)
        xL = ops.scatter(ids, f, np.zeros(NL)) * 3.0
        results.append(ops.gather(rs, ci, xL))
    assert np.array_equal(results[0], results[1]) and np.array_equal(results[0], results[2])


def test_exact_sum_helper_is_correctly_rounded():
    vals = [1e100, 1.0, -1e100, 2.0**-60]
    assert ops.exact_sum(vals) == float(_exact(vals)) == 1.0
    assert ops.exact_sum([0.1] * 10) == float(_exact([0.1] * 10))
