"""Structured hex mesh, scatter map Z and the CSR form of Z^T (Section 2, 5).

The paper's meshes are K x K x K hexahedra of the unit cube, each carrying
the (N+1)^3 tensor-product Gauss-Lobatto-Legendre nodes of degree N
(Section 2).  Node values are stored twice: once per unique node (global
vector, length N_G) and once per element node (local vector, element-major,
length N_L = E (N+1)^3); Z maps global to local (eq. scatter_def) with one
nonzero per row, stored as an id array (the BS7 listing's scatterIds).

The paper leaves the numbering conventions open.  The readings used here:

* local node (i, j, k) of the element in slot s has index
  l = s (N+1)^3 + i + (N+1)(j + (N+1)k), i fastest, in the element's frame;
* slot s holds lattice element e = perm[s], with lattice position
  (e mod K, (e div K) mod K, e div K^2);
* the element frame is turned by orientation o = (pi, f): a permutation pi of
  the three axes and a flip bit per axis.  The 24 proper rotations are those
  with parity(pi) xor f0 xor f1 xor f2 == 0, listed for pi in lexicographic
  order and f = f0 + 2 f1 + 4 f2 ascending; index 0 is the identity;
* local (i, j, k) lands on lattice offset o_d = t[pi[d]] (or N - t[pi[d]]
  when f_d is set), t = (i, j, k), i.e. lattice point
  (N qx + o_0, N qy + o_1, N qz + o_2);
* the global id of lattice point (X, Y, Z) is X + M (Y + M Z), M = K N + 1,
  whatever the element order.

TEST INFRASTRUCTURE ONLY: not part of the library path.
"""

import itertools

import numpy as np


def _parity(p):
    inv = sum(1 for a in range(3) for b in range(a + 1, 3) if p[a] > p[b])
    return inv & 1


def orientation_table():
    """The 24 proper hex orientations as (pi, flips) pairs, identity first."""
    table = []
    for pi in itertools.permutations(range(3)):
        for f in range(8):
            flips = (f & 1, (f >> 1) & 1, (f >> 2) & 1)
            if _parity(pi) ^ flips[0] ^ flips[1] ^ flips[2] == 0:
                table.append((tuple(pi), flips))
    return table


def sizes(K, N):
    """(E, N_L, N_G) of the K^3 mesh at degree N."""
    E = K ** 3
    return E, E * (N + 1) ** 3, (K * N + 1) ** 3


def hex_map(K, N, perm=None, orient=None):
    """Scatter ids (map[l] = global id of local node l) of the K^3 mesh.

    perm[s] is the lattice element in slot s and orient[s] its orientation.
    Passing the entries of a subset of slots gives the map rows of just those
    slots, in that order ((N+1)^3 ids per slot).
    """
    Np = N + 1
    M = K * N + 1
    perm = np.arange(K ** 3, dtype=np.int64) if perm is None else np.asarray(perm, dtype=np.int64)
    orient = np.zeros(perm.size, dtype=np.int64) if orient is None else np.asarray(orient, dtype=np.int64)
    E = perm.size
    table = orientation_table()
    # local (i, j, k) of one element, in local order (i fastest)
    kk, jj, ii = np.meshgrid(np.arange(Np), np.arange(Np), np.arange(Np), indexing="ij")
    t = np.stack([ii.ravel(), jj.ravel(), kk.ravel()])  # shape (3, Np^3)
    qx = perm % K
    qy = (perm // K) % K
    qz = perm // (K * K)
    q = np.stack([qx, qy, qz])  # shape (3, E)
    out = np.empty((E, Np ** 3), dtype=np.int64)
    for o, (pi, flips) in enumerate(table):
        slots = np.nonzero(orient == o)[0]
        if slots.size == 0:
            continue
        offs = []
        for d in range(3):
            od = t[pi[d]]
            offs.append(N - od if flips[d] else od)
        lat = [N * q[d][slots][:, None] + offs[d][None, :] for d in range(3)]
        out[slots] = lat[0] + M * (lat[1] + M * lat[2])
    return out.ravel()


def box_side(E):
    """Smallest m with m^3 >= E."""
    m = 1
    while m ** 3 < E:
        m += 1
    return m


def box_map(E, N):
    """Scatter ids of the first E elements of an m^3 box, m = box_side(E).

    Elements are taken in lexicographic order (x fastest), all with the
    identity orientation; local node (i, j, k) of element (qx, qy, qz) sits on
    lattice point (N qx + i, N qy + j, N qz + k).  The global nodes are the
    lattice points some element touches, numbered by rank in lexicographic
    order (X fastest).  Returns (scatter_ids, n_global).
    """
    m = box_side(E)
    ids = hex_map(m, N, np.arange(E, dtype=np.int64))  # lattice keys X + M(Y + M Z)
    keys, inv = np.unique(ids, return_inverse=True)
    return inv.astype(np.int64).ravel(), int(keys.size)


def csr_inverse(scatter_ids, n_global):
    """CSR of Z^T without values: (row_starts, col_ids) (Section 5).

    Row g lists the local indices l with scatter_ids[l] == g in ascending
    order (stable sort of the ids); negative (masked) ids are left out.
    """
    ids = np.asarray(scatter_ids, dtype=np.int64)
    keep = np.nonzero(ids >= 0)[0]
    order = np.argsort(ids[keep], kind="stable")
    col_ids = keep[order]
    deg = np.bincount(ids[keep], minlength=n_global)
    row_starts = np.zeros(n_global + 1, dtype=np.int64)
    np.cumsum(deg, out=row_starts[1:])
    return row_starts, col_ids


def degree(scatter_ids, n_global):
    """Number of unmasked local copies of each global node."""
    ids = np.asarray(scatter_ids, dtype=np.int64)
    return np.bincount(ids[ids >= 0], minlength=n_global)


def weights(scatter_ids, n_global):
    """Local weights w_l = 1/deg(map[l]) (IEEE division); masked l get 0.

    With these weights a local weighted inner product equals the global one
    on continuous fields (the scattered form, Section 2).
    """
    ids = np.asarray(scatter_ids, dtype=np.int64)
    deg = degree(ids, n_global).astype(np.float64)
    w = np.zeros(ids.size, dtype=np.float64)
    keep = ids >= 0
    w[keep] = 1.0 / deg[ids[keep]]
    return w
