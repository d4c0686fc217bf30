"""Element operators of the Helmholtz problem (Section 2, eqs. helm_var,
global_system, assembled_stiff, assembled_mass), binary64.

Section 2 discretises  int grad v . grad u + lambda v u  on hexahedra with
the tensor-product Lagrange basis through the (N+1) Gauss-Lobatto-Legendre
(GLL) points of each axis, and writes the global operators as
S_G = Z^T S_L Z and M_G = Z^T M_L Z with block-diagonal S_L, M_L.  This
module builds those blocks as dense matrices and applies them literally.

Readings (the paper gives the forms, not the quadrature or the geometry):

* element e is an affine image of the reference cube [-1, 1]^3 with
  Jacobian J_e; its blocks are
      M^e = |J_e| (M1 x M1 x M1)
      S^e = sum_{d,d'} G_{dd'} (A_d)^T W (A_d')     with G = |J_e| J_e^-1 J_e^-T
  where, for the 1D basis l_0..l_N through the GLL points, M1 = B^T W1 B,
  B[a, j] = l_j(xi_a), D[a, j] = l_j'(xi_a) at the q = N + 1 Gauss-Legendre
  points xi_a with weights W1 = diag(w_a); A_1 = B x B x D (derivative along
  the first local axis), A_2 = B x D x B, A_3 = D x B x B and W = W1 x W1 x W1
  (x: Kronecker product, the last factor running fastest, matching local
  index i + (N+1)(j + (N+1) k)).  q = N + 1 Gauss points integrate every
  product of two degree-N polynomials exactly, so on affine elements these
  are the exact Galerkin matrices;
* geometric factors are passed per element as (G11, G12, G13, G22, G23,
  G33, |J|); on the structured meshes of the unit cube (element side
  h = 1/K, any of the 24 orientations) J_e = (h/2) times a signed
  permutation matrix, so G = (h/2) I and |J| = (h/2)^3;
* the Helmholtz block is A^e = S^e + lambda M^e, and the global operator
  y_G = Z^T A_L Z x_G: scatter, apply every block, gather (eq.
  assembled_stiff, assembled_mass); a negative scatter id masks its local
  copy (the scatter's convention, Listing 5): Z has no entry in that row,
  so the copy reads 0 and its result is dropped (a Dirichlet node);
* helmholtz_cg solves Z^T A_L Z x = b with Algorithm 1 in binary64 (the
  conjugate gradients of the cg module, this operator in place of the
  finite-difference one);
* the lumped mass puts the GLL rule on the nodes themselves: the block is
  diagonal, d_l = |J_e| w_i w_j w_k (GLL weights, rounded as
  fl(fl(fl(w_i w_j) w_k) |J_e|)), and y_G[g] adds d_l x_G[g] over the local
  copies l of g in ascending l from +0.0, like the gather (Listing 4).

TEST INFRASTRUCTURE ONLY: not part of the library path.
"""

from fractions import Fraction

import numpy as np
from numpy.polynomial import legendre as L

__all__ = ["gll", "gauss", "lagrange_basis", "element_1d", "element_blocks", "geometry_cube",
           "apply_local", "apply_assembled", "helmholtz_cg", "lumped_weights", "apply_lumped", "node_coordinates"]


def _legendre_exact(n, x):
    """(P_n(x), P_{n-1}(x)) at a rational x by the three-term recurrence
    (k P_k = (2k - 1) x P_{k-1} - (k - 1) P_{k-2}), in exact arithmetic."""
    p0, p1 = Fraction(1), x
    if n == 0:
        return p0, Fraction(0)
    for k in range(2, n + 1):
        p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
    return p1, p0


def _dlegendre_exact(n, x):
    """P_n'(x) from (1 - x^2) P_n' = n (P_{n-1} - x P_n), x != +-1."""
    pn, pm = _legendre_exact(n, x)
    return n * (pm - x * pn) / (1 - x * x)


_ONE = 1 << 256


def _polish(x0, f, df, steps=3):
    """Newton steps on f from the double x0, each evaluated in exact rational
    arithmetic and its result rounded to a multiple of 2^-256 (so the
    numbers stay small); from a start within 1e-13 the second step is
    already below 1e-50."""
    x = Fraction(float(x0))
    for _ in range(steps):
        x = x - f(x) / df(x)
        x = Fraction(round(x * _ONE), _ONE)
    return x


def gll(N):
    """GLL nodes and weights on [-1, 1]: the ends and the roots of P_N',
    weights 2 / (N (N+1) P_N(x)^2), each rounded once to binary64.  numpy's
    companion-matrix roots are only a starting point (they miss the roots by
    up to tens of units in the last place); Newton steps on P_N' in exact
    rational arithmetic, with P_N'' from the Legendre equation
    (1 - x^2) P_N'' = 2 x P_N' - N (N+1) P_N, take each root far below
    binary64 resolution before it is rounded."""
    if N < 1:
        raise ValueError("degree N >= 1")
    cN = np.zeros(N + 1)
    cN[N] = 1.0
    guess = np.sort(np.real(L.legroots(L.legder(cN)))) if N >= 2 else np.zeros(0)

    def f(x):
        return _dlegendre_exact(N, x)

    def df(x):
        pn, _ = _legendre_exact(N, x)
        return (2 * x * f(x) - N * (N + 1) * pn) / (1 - x * x)

    roots = [Fraction(-1)] + [_polish(g, f, df) for g in guess] + [Fraction(1)]
    x = np.array([float(r) for r in roots])
    w = np.array([float(Fraction(2) / (N * (N + 1) * _legendre_exact(N, r)[0] ** 2)) for r in roots])
    return x, w


def gauss(q):
    """Gauss-Legendre nodes and weights (q points, exact to degree 2q - 1):
    the roots of P_q and 2 / ((1 - x^2) P_q'(x)^2), polished from numpy's
    values by exact Newton steps and rounded once to binary64."""
    guess, _ = L.leggauss(q)
    roots = [_polish(g, lambda x: _legendre_exact(q, x)[0], lambda x: _dlegendre_exact(q, x)) for g in guess]
    x = np.array([float(r) for r in roots])
    w = np.array([float(Fraction(2) / ((1 - r * r) * _dlegendre_exact(q, r) ** 2)) for r in roots])
    return x, w


def lagrange_basis(nodes, pts):
    """B[a, j] = l_j(pts[a]) and D[a, j] = l_j'(pts[a]) for the Lagrange
    polynomials through `nodes` (product form and its derivative)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    pts = np.asarray(pts, dtype=np.float64)
    n = nodes.size
    B = np.ones((pts.size, n))
    D = np.zeros((pts.size, n))
    for j in range(n):
        others = [m for m in range(n) if m != j]
        den = np.prod([nodes[j] - nodes[m] for m in others])
        for a, x in enumerate(pts):
            terms = [x - nodes[m] for m in others]
            B[a, j] = np.prod(terms) / den
            # d/dx prod_m (x - x_m) = sum_k prod_{m != k} (x - x_m)
            D[a, j] = sum(np.prod([terms[i] for i in range(len(terms)) if i != k]) for k in range(len(terms))) / den
    return B, D


def element_1d(N):
    """(B, D, w): the basis through the GLL points of degree N, evaluated at
    the q = N + 1 Gauss points, and the Gauss weights."""
    x, _ = gll(N)
    xi, wq = gauss(N + 1)
    B, D = lagrange_basis(x, xi)
    return B, D, wq


def element_blocks(N, geo, lam):
    """Dense Helmholtz block S^e + lam M^e of one element with factors
    geo = (G11, G12, G13, G22, G23, G33, |J|)."""
    B, D, wq = element_1d(N)
    W = np.kron(np.kron(np.diag(wq), np.diag(wq)), np.diag(wq))
    A = [np.kron(np.kron(B, B), D), np.kron(np.kron(B, D), B), np.kron(np.kron(D, B), B)]
    G = np.array([[geo[0], geo[1], geo[2]], [geo[1], geo[3], geo[4]], [geo[2], geo[4], geo[5]]])
    S = sum(G[d, e] * (A[d].T @ W @ A[e]) for d in range(3) for e in range(3))
    Bq = np.kron(np.kron(B, B), B)
    M = geo[6] * (Bq.T @ W @ Bq)
    return S + lam * M


def geometry_cube(K, E=None):
    """Per-element factors of the K^3 mesh of the unit cube (any orientation)."""
    h = 1.0 / K
    E = K ** 3 if E is None else E
    g = np.zeros((E, 7))
    g[:, 0] = g[:, 3] = g[:, 5] = h / 2.0
    g[:, 6] = (h / 2.0) ** 3
    return g


def apply_local(N, geo, lam, xL):
    """y_L = A_L x_L, element by element with the dense blocks."""
    P = (N + 1) ** 3
    xL = np.asarray(xL, dtype=np.float64)
    E = xL.size // P
    yL = np.empty_like(xL)
    cache = {}
    for e in range(E):
        key = tuple(geo[e])
        if key not in cache:
            cache[key] = element_blocks(N, geo[e], lam)
        yL[e * P:(e + 1) * P] = cache[key] @ xL[e * P:(e + 1) * P]
    return yL


def apply_assembled(N, geo, lam, scatter_ids, xG):
    """y_G = Z^T A_L Z x_G (eqs. assembled_stiff, assembled_mass): scatter,
    apply the blocks, and add the local results of each global node; masked
    copies (negative ids) read 0 and add nothing."""
    ids = np.asarray(scatter_ids, dtype=np.int64)
    xG = np.asarray(xG, dtype=np.float64)
    live = ids >= 0
    xL = np.zeros(ids.size)
    xL[live] = xG[ids[live]]
    yL = apply_local(N, geo, lam, xL)
    yG = np.zeros_like(xG)
    np.add.at(yG, ids[live], yL[live])
    return yG


def helmholtz_cg(N, geo, lam, scatter_ids, b, x0=None, tol=1e-10, max_iter=10000):
    """Algorithm 1 on the assembled operator.  Returns (x, iterations, true
    relative residual)."""
    from oracle.cg import cg_operator
    return cg_operator(lambda v: apply_assembled(N, geo, lam, scatter_ids, v), b, x0, tol, max_iter)


def lumped_weights(N, geo):
    """d_l of the lumped mass, element by element (see the readings)."""
    _, w = gll(N)
    P1 = N + 1
    w3 = np.empty(P1 ** 3)
    for k in range(P1):
        for j in range(P1):
            for i in range(P1):
                w3[i + P1 * (j + P1 * k)] = (w[i] * w[j]) * w[k]
    return (np.asarray(geo, dtype=np.float64)[:, 6][:, None] * w3[None, :]).ravel()


def apply_lumped(N, geo, row_starts, col_ids, xG):
    """y_G[g] = ((+0.0 + d_l0 x_g) + d_l1 x_g) + ... over the copies l0 < l1 < ...
    of g (the CSR rows of Z^T), never forming x_L."""
    d = lumped_weights(N, geo)
    rs = np.asarray(row_starts, dtype=np.int64)
    ci = np.asarray(col_ids, dtype=np.int64)
    xG = np.asarray(xG, dtype=np.float64)
    deg = np.diff(rs)
    acc = np.zeros_like(xG)
    for j in range(int(deg.max()) if deg.size else 0):
        rows = np.nonzero(deg > j)[0]
        acc[rows] = acc[rows] + d[ci[rs[rows] + j]] * xG[rows]
    return acc


def node_coordinates(K, N):
    """Physical (x, y, z) of every global node of the K^3 mesh of the unit
    cube: lattice index X = N qx + o lies at (qx + (1 + r_o) / 2) / K with
    r_o the o-th GLL point."""
    r, _ = gll(N)
    M = K * N + 1
    idx = np.arange(M)
    q, o = idx // N, idx % N
    c = (q + (1.0 + r[o]) / 2.0) / K
    c[-1] = 1.0
    X = np.tile(c, M * M)
    Y = np.tile(np.repeat(c, M), M)
    Z = np.repeat(c, M * M)
    return X, Y, Z
