"""Pins of the oracle's mesh, scatter map, CSR inverse, degrees and weights.

The map is checked against geometry: node coordinates built from the
Gauss-Lobatto-Legendre points and the rotation matrices of the reference
cube, de-duplicated and numbered without any use of the oracle's index
arithmetic.  Degrees are checked against a closed-form count.
"""

import itertools

import numpy as np
import pytest

import bsgen
from oracle import mesh, ops


def gll(N):
    from numpy.polynomial import legendre
    inner = legendre.Legendre.basis(N).deriv().roots().real if N > 1 else np.zeros(0)
    return np.concatenate([[-1.0], np.sort(inner), [1.0]])


def rotation_matrix(pi, flips):
    R = np.zeros((3, 3))
    for d in range(3):
        R[d, pi[d]] = -1.0 if flips[d] else 1.0
    return R


def geometric_map(K, N, perm, orient):
    """Global ids from coordinates: rotate reference nodes, place, de-duplicate."""
    E = K ** 3
    r = gll(N)
    kk, jj, ii = np.meshgrid(r, r, r, indexing="ij")
    ref = np.stack([ii.ravel(), jj.ravel(), kk.ravel()])  # local order, i fastest
    table = mesh.orientation_table()
    h = 1.0 / K
    pts = []
    for s in range(E):
        e = int(perm[s])
        origin = np.array([e % K, (e // K) % K, e // (K * K)], dtype=np.float64) * h
        R = rotation_matrix(*table[int(orient[s])])
        pts.append(origin[:, None] + h * (1.0 + R @ ref) / 2.0)
    P = np.concatenate(pts, axis=1).T  # (N_L, 3) coordinates
    key = np.round(P * 1e9).astype(np.int64)
    uniq, inv = np.unique(key, axis=0, return_inverse=True)
    # number the unique points lexicographically by (z, y, x)
    order = np.lexsort((uniq[:, 0], uniq[:, 1], uniq[:, 2]))
    rank = np.empty_like(order)
    rank[order] = np.arange(order.size)
    return rank[inv.ravel()], P


def test_orientation_table_is_the_rotation_group():
    table = mesh.orientation_table()
    assert len(table) == 24
    mats = [rotation_matrix(*o) for o in table]
    assert np.array_equal(mats[0], np.eye(3))
    for R in mats:
        assert round(np.linalg.det(R)) == 1
    keys = {tuple(R.ravel()) for R in mats}
    assert len(keys) == 24
    for A, B in itertools.product(mats, mats):
        assert tuple((A @ B).ravel()) in keys


@pytest.mark.parametrize("K,N,seed", [(1, 1, 0), (2, 1, 1), (2, 2, 2), (3, 3, 3), (2, 4, 4), (3, 2, 5)])
def test_map_matches_geometry(K, N, seed):
    E, NL, NG = mesh.sizes(K, N)
    perm = bsgen.permutation(seed, E)
    orient = bsgen.orientations(seed, E)
    ids = mesh.hex_map(K, N, perm, orient)
    geo, _ = geometric_map(K, N, perm, orient)
    assert ids.shape == (NL,)
    assert np.array_equal(ids, geo)
    assert np.unique(ids).size == NG


def test_lexicographic_identity_map_small_case():
    # K = 1, N = 1: the 8 corners, local order equals lattice order
    assert list(mesh.hex_map(1, 1)) == list(range(8))
    # K = 2, N = 1, element 1 (x = 1): corners shifted by one along x
    ids = mesh.hex_map(2, 1)
    assert list(ids[8:16]) == [1, 2, 4, 5, 10, 11, 13, 14]


def test_linear_field_closed_form_through_scatter():
    K, N = 3, 4
    E, NL, NG = mesh.sizes(K, N)
    perm = bsgen.permutation(8, E)
    orient = bsgen.orientations(8, E)
    ids = mesh.hex_map(K, N, perm, orient)
    _, P = geometric_map(K, N, perm, orient)
    a, b, c, d = 0.25, -1.5, 2.0, 0.75
    # global coordinates from the lattice: X -> element X // N, node X % N
    M = K * N + 1
    r = gll(N)
    one_d = np.array([((X // N) + (1.0 + r[X % N]) / 2.0) / K if X < K * N else 1.0 for X in range(M)])
    g = np.arange(NG)
    gx, gy, gz = one_d[g % M], one_d[(g // M) % M], one_d[g // (M * M)]
    fG = a + b * gx + c * gy + d * gz
    fL = ops.scatter(ids, fG, np.zeros(NL))
    exact = a + b * P[:, 0] + c * P[:, 1] + d * P[:, 2]
    assert np.max(np.abs(fL - exact)) <= 1e-14


@pytest.mark.parametrize("K,N", [(8, 3), (2, 1), (3, 7), (5, 2), (4, 6)])
def test_degree_histogram_closed_form(K, N):
    E, NL, NG = mesh.sizes(K, N)
    ids = mesh.hex_map(K, N, bsgen.permutation(K, E), bsgen.orientations(K, E))
    deg = mesh.degree(ids, NG)
    a, b = K - 1, K * (N - 1) + 2
    hist = np.bincount(deg, minlength=9)
    assert hist[1] == b ** 3 and hist[2] == 3 * a * b * b
    assert hist[4] == 3 * a * a * b and hist[8] == a ** 3
    assert hist.sum() == NG and int(deg.sum()) == NL
    if (K, N) == (8, 3):
        assert (hist[1], hist[2], hist[4], hist[8]) == (5832, 6804, 2646, 343)


def test_each_element_has_distinct_nodes_and_permutation_keeps_rows():
    K, N = 4, 3
    E, NL, NG = mesh.sizes(K, N)
    base = mesh.hex_map(K, N)
    perm = bsgen.permutation(9, E)
    orient = bsgen.orientations(9, E)
    ids = mesh.hex_map(K, N, perm, orient)
    per_el = ids.reshape(E, -1)
    for row in per_el:
        assert np.unique(row).size == (N + 1) ** 3
    # slot s of the permuted mesh carries the node set of lattice element perm[s]
    base_el = base.reshape(E, -1)
    for s in range(E):
        assert set(per_el[s]) == set(base_el[perm[s]])


def test_csr_inverse_rows_ascending_and_consistent():
    K, N = 3, 2
    E, NL, NG = mesh.sizes(K, N)
    ids = mesh.hex_map(K, N, bsgen.permutation(1, E), bsgen.orientations(1, E))
    ids = ids.copy()
    ids[::7] = -1  # mask some entries
    rs, ci = mesh.csr_inverse(ids, NG)
    assert rs[0] == 0 and rs[-1] == np.count_nonzero(ids >= 0)
    for g in range(NG):
        row = ci[rs[g]:rs[g + 1]]
        assert np.all(np.diff(row) > 0)
        assert np.all(ids[row] == g)
        assert row.size == np.count_nonzero(ids == g)


def test_weights_are_reciprocal_degrees():
    K, N = 3, 3
    E, NL, NG = mesh.sizes(K, N)
    ids = mesh.hex_map(K, N)
    w = mesh.weights(ids, NG)
    deg = mesh.degree(ids, NG)
    assert set(np.unique(w)) <= {1.0, 0.5, 0.25, 0.125}
    assert np.all(w * deg[ids] == 1.0)
    masked = ids.copy()
    masked[:5] = -1
    assert np.all(mesh.weights(masked, NG)[:5] == 0.0)
