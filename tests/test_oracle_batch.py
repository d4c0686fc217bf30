"""Pins of the box-mesh instances and of the batched step's oracle.

The box mesh (first E elements of an m^3 box, lexicographic, identity
orientation) is pinned by closed forms: a full cube is the structured mesh,
full z-slabs plus a partial layer have a counted node total, and the missing
corner element of a 2^3 box leaves one node shared by seven elements.  The
batch step is made of the single-operation oracles (pinned elsewhere); its
CG part is pinned by a property of CG itself: on the diagonal operator
Z^T Z it stops within as many iterations as there are distinct degrees.
"""

import numpy as np
import pytest

import bsgen
from oracle import batch, mesh, ops


@pytest.mark.parametrize("m,N", [(1, 2), (2, 3), (3, 2)])
def test_full_box_is_the_structured_mesh(m, N):
    ids, ng = mesh.box_map(m ** 3, N)
    assert ng == (m * N + 1) ** 3
    assert np.array_equal(ids, mesh.hex_map(m, N))


@pytest.mark.parametrize("N", [2, 5, 8])
def test_single_element(N):
    ids, ng = mesh.box_map(1, N)
    assert ng == (N + 1) ** 3 and np.array_equal(ids, np.arange(ng))


@pytest.mark.parametrize("m,z,y,N", [(3, 1, 0, 2), (3, 1, 2, 3), (4, 2, 1, 2), (4, 3, 3, 4)])
def test_slabs_plus_partial_layer(m, z, y, N):
    # z full slabs of m^2 elements, then y full rows of the next slab
    E = m * m * z + m * y
    assert mesh.box_side(E) == m
    ids, ng = mesh.box_map(E, N)
    M = m * N + 1
    expect = M * M * (z * N + 1) + (M * (y * N + 1) * N if y else 0)
    assert ng == expect
    assert np.array_equal(np.sort(np.unique(ids)), np.arange(ng))


@pytest.mark.parametrize("N", [2, 3, 6])
def test_reentrant_corner(N):
    ids, ng = mesh.box_map(7, N)  # 2^3 box without element (1,1,1)
    assert ng == (2 * N + 1) ** 3 - N ** 3
    deg = mesh.degree(ids, ng)
    assert deg.max() == 7 and np.count_nonzero(deg == 7) == 1
    assert set(np.unique(deg)) <= {1, 2, 3, 4, 5, 6, 7}


def test_instance_descriptors():
    E, N = bsgen.batch_instances(10917, 1024)
    assert E.min() >= 1 and E.max() <= 4096 and N.min() == 2 and N.max() == 8
    # log-uniform: about a twelfth of the instances per octave
    counts = np.bincount(np.floor(np.log2(E)).astype(int), minlength=13)
    assert counts[:12].min() > 40
    total_local = int(np.sum(E * (N + 1) ** 3))
    assert 1.2e8 < total_local < 1.7e8


def test_step_matches_the_operations_one_by_one():
    ids, ng = mesh.box_map(11, 3)
    nl = ids.size
    rng = np.random.default_rng(1)
    v = {k: rng.uniform(-1, 1, ng) for k in ("x", "y", "p", "r", "Ap")}
    v.update({k: rng.uniform(-1, 1, nl) for k in ("xL", "pL")})
    v["wL"] = mesh.weights(ids, ng)
    out, s = batch.step(ids, ng, v, 0.37, 0.61)
    deg = mesh.degree(ids, ng).astype(float)
    # steps 6-7 act on x after step 5; Z^T Z is diag(degree) up to the
    # rounding of repeated addition
    x5 = v["x"] + 0.37 * v["p"]
    assert np.array_equal(out["xL"], x5[ids])
    assert np.all(np.abs(out["y"] - deg * x5) <= deg * deg * 2.0 ** -52 * np.abs(x5))
    assert np.all(np.abs(out["Ap"] - deg * v["p"]) <= deg * deg * 2.0 ** -52 * np.abs(v["p"]))
    assert s["alpha"] == s["rr"] / s["pAp"] and s["beta"] == s["rr2"] / s["rr"]
    assert s["norm"] == ops.norm(v["xL"], v["wL"])
    # the weighted local norm of a scattered field is its global norm
    g = rng.uniform(-1, 1, ng)
    assert abs(ops.norm(g[ids], v["wL"]) - ops.norm(g)) <= 1e-13 * ops.norm(g)


@pytest.mark.parametrize("E,N", [(7, 2), (20, 3), (64, 2)])
def test_cg_on_diag_degree_stops_within_distinct_degrees(E, N):
    ids, ng = mesh.box_map(E, N)
    deg = mesh.degree(ids, ng)
    b = bsgen.uniform(3, 10, ng)
    x, it = batch.cg_iterations(ids, ng, b, tol=1e-13)
    assert it <= len(np.unique(deg)) + 1
    assert np.allclose(x * deg, b, rtol=0, atol=1e-12)
