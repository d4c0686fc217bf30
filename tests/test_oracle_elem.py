"""Pins of the element-operator oracle (Section 2: GLL Lagrange basis, the
mass and stiffness blocks and their assembly Z^T A_L Z).

Every pin is a value the mathematics fixes: closed-form GLL rules, exactness
of the quadrature, the cardinal and partition-of-unity properties of the
basis, and integrals of polynomial fields over the unit cube that the
assembled matrices must reproduce (the field is in the finite element space,
so u^T M u and u^T S u are exact integrals).
"""

import math
from fractions import Fraction

import numpy as np
import pytest

import bsgen
from oracle import elem, mesh, ops


def test_gll_closed_forms():
    x, w = elem.gll(1)
    assert np.allclose(x, [-1, 1]) and np.allclose(w, [1, 1])
    x, w = elem.gll(2)
    assert np.allclose(x, [-1, 0, 1], atol=1e-15) and np.allclose(w, [1 / 3, 4 / 3, 1 / 3], atol=1e-15)
    x, w = elem.gll(3)
    s = 1 / math.sqrt(5)
    assert np.allclose(x, [-1, -s, s, 1], atol=1e-15) and np.allclose(w, [1 / 6, 5 / 6, 5 / 6, 1 / 6], atol=1e-15)


def _legendre_q(n, x):
    """P_n(x) and P_n'(x) at a rational x, exactly (the explicit sum
    P_n(x) = 2^-n sum_k (-1)^k C(n,k) C(2n-2k,n) x^(n-2k), not the
    recurrence the oracle uses)."""
    p = sum((-1) ** k * math.comb(n, k) * math.comb(2 * n - 2 * k, n) * x ** (n - 2 * k) for k in range(n // 2 + 1))
    dp = sum((-1) ** k * math.comb(n, k) * math.comb(2 * n - 2 * k, n) * (n - 2 * k) * x ** (n - 2 * k - 1)
             for k in range(n // 2 + 1) if n - 2 * k > 0)
    return p / Fraction(2) ** n, dp / Fraction(2) ** n


def _brackets_a_root(f, x):
    """f changes sign between the midpoints from x to its binary64
    neighbours, so x is the root rounded to nearest (or f(x) = 0)."""
    lo = (Fraction(x) + Fraction(np.nextafter(x, -np.inf))) / 2
    hi = (Fraction(x) + Fraction(np.nextafter(x, np.inf))) / 2
    return f(Fraction(x)) == 0 or (f(lo) > 0) != (f(hi) > 0)


@pytest.mark.parametrize("N", [2, 3, 5, 7, 10, 15])
def test_rule_nodes_are_correctly_rounded_roots(N):
    # interior GLL nodes are the roots of P_N', Gauss nodes those of P_{N+1}
    x, _ = elem.gll(N)
    for a in range(1, N):
        assert _brackets_a_root(lambda t: _legendre_q(N, t)[1], x[a]), (N, a)
    xq, _ = elem.gauss(N + 1)
    for a in range(N + 1):
        assert _brackets_a_root(lambda t: _legendre_q(N + 1, t)[0], xq[a]), (N, a)


@pytest.mark.parametrize("N", [3, 7, 15])
def test_rule_weights_within_an_ulp(N):
    # GLL: w = 2 / (N (N+1) P_N(x)^2), evaluated exactly at the rounded node
    # (P_N is stationary at the GLL nodes, so the rounding of the node moves
    # it by far less than an ulp).  Gauss: w = 2 / ((1 - x^2) P_q'(x)^2) is
    # monotone over the half-ulp interval around the rounded node that holds
    # the exact root, so the exact weight lies between its values at the two
    # ends; the oracle's weight is within one ulp of that interval.
    x, w = elem.gll(N)
    for a in range(N + 1):
        ref = float(Fraction(2) / (N * (N + 1) * _legendre_q(N, Fraction(x[a]))[0] ** 2))
        assert abs(w[a] - ref) <= np.spacing(ref), (N, a)
    xq, wq = elem.gauss(N + 1)

    def wg(t):
        return Fraction(2) / ((1 - t * t) * _legendre_q(N + 1, t)[1] ** 2)

    for a in range(N + 1):
        lo = (Fraction(xq[a]) + Fraction(np.nextafter(xq[a], -np.inf))) / 2
        hi = (Fraction(xq[a]) + Fraction(np.nextafter(xq[a], np.inf))) / 2
        w_lo, w_hi = sorted((wg(lo), wg(hi)))
        u = Fraction(float(np.spacing(wq[a])))
        assert w_lo - u <= Fraction(wq[a]) <= w_hi + u, (N, a)


@pytest.mark.parametrize("N", [1, 2, 3, 5, 7, 11, 15])
def test_gll_rule_exact_to_degree_2N_minus_1(N):
    x, w = elem.gll(N)
    assert abs(w.sum() - 2.0) <= 1e-14
    for k in range(2 * N):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) <= 1e-13, k
    # and not beyond: x^(2N) is where the Lobatto rule stops being exact
    assert abs(np.dot(w, x ** (2 * N)) - 2.0 / (2 * N + 1)) > 1e-10


@pytest.mark.parametrize("N", [1, 2, 4, 7, 10])
def test_lagrange_basis_properties(N):
    x, _ = elem.gll(N)
    B, D = elem.lagrange_basis(x, x)
    assert np.allclose(B, np.eye(N + 1), atol=1e-13)          # cardinal: l_j(x_i) = delta_ij
    pts = np.linspace(-1, 1, 13)
    B, D = elem.lagrange_basis(x, pts)
    assert np.allclose(B.sum(1), 1.0, atol=1e-12) and np.allclose(D.sum(1), 0.0, atol=1e-10)
    for k in range(N + 1):                                  # polynomials of degree <= N are reproduced
        assert np.allclose(B @ x ** k, pts ** k, atol=1e-12)
        if k:
            assert np.allclose(D @ x ** k, k * pts ** (k - 1), atol=1e-9)


@pytest.mark.parametrize("N", [1, 2, 3, 7])
def test_mass_row_sums_are_the_gll_weights(N):
    # sum_j M1_ij = integral of l_i = w_i: the GLL rule is exact for degree N
    B, D, wq = elem.element_1d(N)
    M1 = B.T @ np.diag(wq) @ B
    _, w = elem.gll(N)
    assert np.allclose(M1.sum(1), w, atol=1e-14)
    K1 = D.T @ np.diag(wq) @ D
    assert np.allclose(K1 @ np.ones(N + 1), 0.0, atol=1e-11)   # constants have no gradient
    assert np.allclose(M1, M1.T) and np.all(np.linalg.eigvalsh(M1) > 0)


def _mesh(K, N, seed):
    E = K ** 3
    perm = None if seed is None else bsgen.permutation(seed, E)
    orient = None if seed is None else bsgen.orientations(seed, E)
    return mesh.hex_map(K, N, perm, orient)


@pytest.mark.parametrize("K,N,seed", [(1, 2, None), (2, 3, 1), (3, 2, 2), (2, 5, 3)])
def test_assembled_operators_integrate_polynomial_fields(K, N, seed):
    ids = _mesh(K, N, seed)
    geo = elem.geometry_cube(K)
    X, Y, Z = elem.node_coordinates(K, N)
    one = np.ones_like(X)

    def mass(u):
        return float(u @ elem.apply_assembled(N, geo, 1.0, ids, u) - u @ elem.apply_assembled(N, geo, 0.0, ids, u))

    def stiff(u):
        return float(u @ elem.apply_assembled(N, geo, 0.0, ids, u))

    assert abs(mass(one) - 1.0) <= 1e-13                    # volume of the unit cube
    assert abs(mass(X) - 1 / 3) <= 1e-13                    # int x^2
    assert abs(mass(X * Y * Z) - 1 / 27) <= 1e-13           # int x^2 y^2 z^2
    assert np.allclose(elem.apply_assembled(N, geo, 0.0, ids, one), 0.0, atol=1e-12)  # S 1 = 0
    assert abs(stiff(X + 2 * Y - Z) - 6.0) <= 1e-12         # |grad u|^2 = 1 + 4 + 1
    if N >= 2:
        assert abs(stiff(X * Y) - 2 / 3) <= 1e-12           # int y^2 + x^2


@pytest.mark.parametrize("N", [1, 3, 7])
def test_element_block_symmetric_positive(N):
    A = elem.element_blocks(N, elem.geometry_cube(2)[0], 0.5)
    assert np.allclose(A, A.T, atol=1e-14)
    assert np.linalg.eigvalsh(A).min() > 0


def test_assembly_independent_of_element_order_and_orientation():
    K, N = 3, 3
    geo = elem.geometry_cube(K)
    x = bsgen.uniform(5, 12, (K * N + 1) ** 3)
    a = elem.apply_assembled(N, geo, 0.7, _mesh(K, N, None), x)
    b = elem.apply_assembled(N, geo, 0.7, _mesh(K, N, 9), x)
    assert np.allclose(a, b, rtol=0, atol=1e-13 * np.abs(a).max())


@pytest.mark.parametrize("K,N,seed", [(2, 2, None), (3, 3, 4), (2, 7, 5)])
def test_lumped_mass(K, N, seed):
    ids = _mesh(K, N, seed)
    NG = (K * N + 1) ** 3
    rs, ci = mesh.csr_inverse(ids, NG)
    geo = elem.geometry_cube(K)
    X, Y, Z = elem.node_coordinates(K, N)
    one = np.ones(NG)
    m1 = elem.apply_lumped(N, geo, rs, ci, one)
    assert abs(m1.sum() - 1.0) <= 1e-13                     # volume
    assert abs(float(X @ elem.apply_lumped(N, geo, rs, ci, X)) - 1 / 3) <= 1e-13  # GLL exact for x^2 (N >= 2)
    # one node's row is the sum of its copies' weights: deg * the weight for equal weights
    d = elem.lumped_weights(N, geo)
    g = int(ids[0])
    assert m1[g] == sum(d[l] for l in np.nonzero(ids == g)[0])
    # the lumped mass is the row sum of the exact mass (GLL exact to degree 2N - 1 >= N)
    exact_rows = elem.apply_assembled(N, geo, 1.0, ids, one) - elem.apply_assembled(N, geo, 0.0, ids, one)
    assert np.allclose(m1, exact_rows, rtol=0, atol=1e-14)
    # the fixed order: terms added one copy at a time from +0.0 in ascending l
    x = bsgen.uniform(7, 12, NG)
    y = elem.apply_lumped(N, geo, rs, ci, x)
    ref = np.zeros(NG)
    for g in range(NG):
        acc = 0.0
        for l in ci[rs[g]:rs[g + 1]]:
            acc = acc + d[l] * x[g]
        ref[g] = acc
    assert np.array_equal(y, ref)
    assert np.array_equal(ops.gather(rs, ci, d * x[ids]), y)   # = gather(scatter(x) * d), bit for bit


def test_masked_assembly_is_the_dense_product():
    # Z as a 0/1 matrix (no entry in a masked copy's row), A_L block diagonal
    K, N = 2, 2
    ids = _mesh(K, N, 6).copy()
    ids[::5] = -1
    E, NL, NG = mesh.sizes(K, N)
    P = (N + 1) ** 3
    geo = elem.geometry_cube(K)
    Zm = np.zeros((NL, NG))
    live = np.flatnonzero(ids >= 0)
    Zm[live, ids[live]] = 1.0
    AL = np.zeros((NL, NL))
    for e in range(E):
        AL[e * P:(e + 1) * P, e * P:(e + 1) * P] = elem.element_blocks(N, geo[e], 0.4)
    x = bsgen.uniform(7, 12, NG)
    ref = Zm.T @ (AL @ (Zm @ x))
    got = elem.apply_assembled(N, geo, 0.4, ids, x)
    assert np.allclose(got, ref, rtol=0, atol=1e-13 * np.abs(ref).max())
    # a global node whose copies are all masked has an empty row
    dead = np.setdiff1d(np.arange(NG), ids[live])
    assert dead.size > 0 and np.all(got[dead] == 0.0)


def _interior_problem(K, N, seed):
    """-Lap u = f on the unit cube, u = 0 on its boundary, with u =
    x(1-x) y(1-y) z(1-z): every copy of a boundary node masked, b the
    consistent mass of f against the interior test functions."""
    ids = _mesh(K, N, seed)
    X, Y, Z = elem.node_coordinates(K, N)
    on_bnd = np.zeros(X.size, dtype=bool)
    for c in (X, Y, Z):
        on_bnd |= (np.abs(c) < 1e-14) | (np.abs(c - 1.0) < 1e-14)
    masked = np.where(on_bnd[ids], -1, ids)
    geo = elem.geometry_cube(K)
    geo_mass = geo.copy()
    geo_mass[:, :6] = 0.0  # no stiffness: the block is the consistent mass
    q = lambda t: t * (1.0 - t)  # noqa: E731
    u = q(X) * q(Y) * q(Z)
    f = 2.0 * (q(Y) * q(Z) + q(X) * q(Z) + q(X) * q(Y))
    b = np.where(on_bnd, 0.0, elem.apply_assembled(N, geo_mass, 1.0, ids, f))
    return masked, geo, u, b, on_bnd


@pytest.mark.parametrize("K,N,seed", [(2, 2, None), (2, 3, 3)])
def test_helmholtz_cg_recovers_a_polynomial_solution(K, N, seed):
    # u has degree 2 along each axis, so for N >= 2 it lies in the discrete
    # space and the Galerkin solution is its interpolant (exact quadrature)
    masked, geo, u, b, on_bnd = _interior_problem(K, N, seed)
    x, it, res = elem.helmholtz_cg(N, geo, 0.0, masked, b, tol=1e-13)
    assert res <= 1e-13
    assert np.all(x[on_bnd] == 0.0)
    assert np.max(np.abs(x - u)) <= 1e-12
    assert it <= int((~on_bnd).sum())  # within the number of unknowns


def test_helmholtz_cg_matches_a_dense_solve():
    K, N, lam = 2, 3, 0.5
    ids = _mesh(K, N, 2)
    NG = (K * N + 1) ** 3
    geo = elem.geometry_cube(K)
    A = np.column_stack([elem.apply_assembled(N, geo, lam, ids, np.eye(NG)[:, j]) for j in range(NG)])
    b = bsgen.uniform(9, 12, NG)
    ref = np.linalg.solve(A, b)
    x, it, res = elem.helmholtz_cg(N, geo, lam, ids, b, tol=1e-12)
    assert res <= 1e-12
    kappa = np.linalg.cond(A)
    assert np.linalg.norm(x - ref) <= 4 * kappa * 1e-12 * np.linalg.norm(ref)
