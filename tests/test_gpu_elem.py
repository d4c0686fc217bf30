"""GPU parity of the element operators (Section 2: the Helmholtz blocks
S^e + lambda M^e in the scattered form, and the lumped mass) against the
oracle's dense blocks.

The library's local operator is sum-factorised on the matrix cores, so it
is compared with the dense products within a bound that follows from the
arithmetic: every entry within 1e-13 of (|A^e| |u|)_l, about 450 units in
the last place of the largest term that can enter it (four contraction
levels of eight terms forward and back, plus the rules' last-bit
differences).  The lumped mass adds rounded products in the gather's
order, so only the rounding of the GLL weights separates it from the
oracle: rows within 8 ulps.
"""

import numpy as np
import pytest
import torch

import bsgen
from oracle import elem, mesh, ops

pytestmark = pytest.mark.gpu

import paper_2009_10917_amd as bs  # noqa: E402
from gpu_util import to_host  # noqa: E402

F64 = torch.float64
EPS = 2.0 ** -52


def _mesh(K, N, seed, mask_every=0):
    E = K ** 3
    perm = None if seed is None else bsgen.permutation(seed, E)
    orient = None if seed is None else bsgen.orientations(seed, E)
    ids = mesh.hex_map(K, N, perm, orient).copy()
    if mask_every:
        ids[::mask_every] = -1
    return ids


def _dense_abs(N, geo, lam, xL):
    """|A^e| |u| element by element (the scale of each entry's rounding)."""
    P = (N + 1) ** 3
    A = np.abs(elem.element_blocks(N, geo[0], lam))
    return (np.abs(xL).reshape(-1, P) @ A.T).ravel()


@pytest.mark.parametrize("N", [1, 2, 3, 5, 7, 10, 15])
def test_rules_match_the_oracle(ctx, N):
    el = bs.bs_elem_create(ctx, N)
    gx, gw, qx, qw = bs.bs_elem_rules(el)
    ox, ow = elem.gll(N)
    qox, qow = elem.gauss(N + 1)
    for a, b in ((gx, ox), (gw, ow), (qx, qox), (qw, qow)):
        assert np.all(np.abs(a - b) <= 4 * EPS * np.maximum(np.abs(b), 1.0)), (N, a - b)
    assert abs(gw.sum() - 2.0) <= 4 * EPS and abs(qw.sum() - 2.0) <= 4 * EPS
    el.close()


@pytest.mark.parametrize("K,N,seed,mask", [(2, 1, 1, 0), (3, 2, 2, 0), (2, 3, 3, 5), (2, 5, 4, 0), (3, 7, 5, 0),
                                           (2, 7, None, 0), (2, 7, 6, 9), (1, 4, None, 0)])
def test_helmholtz_local_matches_dense_blocks(ctx, K, N, seed, mask):
    ids = _mesh(K, N, seed, mask)
    E, NL, NG = mesh.sizes(K, N)
    geo = elem.geometry_cube(K)
    lam = 0.7
    xG = bsgen.uniform(11, 12, NG)
    xL = np.where(ids >= 0, xG[np.maximum(ids, 0)], 0.0)
    ref = elem.apply_local(N, geo, lam, xL)
    scale = _dense_abs(N, geo, lam, xL)
    el = bs.bs_elem_create(ctx, N)
    yL = torch.full((NL,), float("nan"), dtype=F64, device="cuda")
    bs.bs_helmholtz_local(ctx, el, torch.from_numpy(ids.astype(np.int32)).cuda(),
                          torch.from_numpy(geo.ravel()).cuda(), lam, torch.from_numpy(xG).cuda(), yL)
    got = to_host(yL)
    assert np.all(np.isfinite(got))
    assert np.all(np.abs(got - ref) <= 1e-13 * scale + 1e-300), float(np.max(np.abs(got - ref) / scale))
    el.close()


def test_helmholtz_local_general_geometry(ctx):
    # sheared elements: every factor G_dd' nonzero, |J| varying per element
    K, N = 2, 4
    ids = _mesh(K, N, 8)
    E, NL, NG = mesh.sizes(K, N)
    rng = np.random.default_rng(3)
    geo = np.empty((E, 7))
    for e in range(E):
        J = np.eye(3) * 0.3 + 0.05 * rng.standard_normal((3, 3))
        dj = np.linalg.det(J)
        Ji = np.linalg.inv(J)
        G = dj * Ji @ Ji.T
        geo[e] = (G[0, 0], G[0, 1], G[0, 2], G[1, 1], G[1, 2], G[2, 2], dj)
    lam = 1.3
    xG = bsgen.uniform(12, 12, NG)
    xL = xG[ids]
    P = (N + 1) ** 3
    ref = np.concatenate([elem.element_blocks(N, geo[e], lam) @ xL[e * P:(e + 1) * P] for e in range(E)])
    scale = np.concatenate([np.abs(elem.element_blocks(N, geo[e], lam)) @ np.abs(xL[e * P:(e + 1) * P])
                            for e in range(E)])
    el = bs.bs_elem_create(ctx, N)
    yL = torch.empty(NL, dtype=F64, device="cuda")
    bs.bs_helmholtz_local(ctx, el, torch.from_numpy(ids.astype(np.int32)).cuda(),
                          torch.from_numpy(geo.ravel()).cuda(), lam, torch.from_numpy(xG).cuda(), yL)
    got = to_host(yL)
    assert np.all(np.abs(got - ref) <= 1e-13 * scale)
    el.close()


@pytest.mark.parametrize("K,N,seed", [(3, 3, 1), (2, 7, 2)])
def test_helmholtz_apply_assembled(ctx, K, N, seed):
    ids = _mesh(K, N, seed)
    E, NL, NG = mesh.sizes(K, N)
    geo = elem.geometry_cube(K)
    lam = 0.25
    xG = bsgen.uniform(13, 12, NG)
    ref = elem.apply_assembled(N, geo, lam, ids, xG)
    rs, ci = mesh.csr_inverse(ids, NG)
    scale = ops.gather(rs, ci, _dense_abs(N, geo, lam, xG[ids]))
    d_map = torch.from_numpy(ids.astype(np.int32)).cuda()
    plan = bs.bs_gs_create(ctx, d_map, NG)
    el = bs.bs_elem_create(ctx, N)
    work = torch.empty(NL, dtype=F64, device="cuda")
    yG = torch.empty(NG, dtype=F64, device="cuda")
    bs.bs_helmholtz_apply(ctx, el, plan, torch.from_numpy(geo.ravel()).cuda(), lam, torch.from_numpy(xG).cuda(), work,
                          yG)
    got = to_host(yG)
    assert np.all(np.abs(got - ref) <= 1e-13 * scale)
    # constants: S 1 = 0, so with lambda = 0 the result vanishes to rounding
    one = torch.ones(NG, dtype=F64, device="cuda")
    bs.bs_helmholtz_apply(ctx, el, plan, torch.from_numpy(geo.ravel()).cuda(), 0.0, one, work, yG)
    assert float(to_host(yG).__abs__().max()) <= 1e-12
    el.close()
    plan.close()


@pytest.mark.parametrize("K,N,seed,mask", [(4, 3, 1, 0), (2, 7, 2, 0), (3, 1, 3, 7), (2, 10, 4, 0), (1, 15, None, 0)])
def test_lumped_mass_matches_oracle(ctx, K, N, seed, mask):
    ids = _mesh(K, N, seed, mask)
    E, NL, NG = mesh.sizes(K, N)
    rs, ci = mesh.csr_inverse(ids, NG)
    geo = elem.geometry_cube(K)
    xG = bsgen.uniform(14, 12, NG)
    ref = elem.apply_lumped(N, geo, rs, ci, xG)
    plan = bs.bs_gs_create(ctx, torch.from_numpy(ids.astype(np.int32)).cuda(), NG)
    el = bs.bs_elem_create(ctx, N)
    yG = torch.full((NG,), float("nan"), dtype=F64, device="cuda")
    bs.bs_mass_lumped(ctx, el, plan, torch.from_numpy(geo.ravel()).cuda(), torch.from_numpy(xG).cuda(), yG)
    got = to_host(yG)
    deg = np.diff(rs)
    # positive weights times one x per row: a well-conditioned sum of deg terms
    assert np.all(np.abs(got - ref) <= (8 + deg) * EPS * np.abs(ref)), float(np.max(np.abs(got - ref) / np.abs(ref)))
    assert np.all(got[deg == 0] == 0.0)
    # the volume of the unit cube
    one = torch.ones(NG, dtype=F64, device="cuda")
    bs.bs_mass_lumped(ctx, el, plan, torch.from_numpy(geo.ravel()).cuda(), one, yG)
    if not mask:
        assert abs(float(to_host(yG).sum()) - 1.0) <= 1e-13
    el.close()
    plan.close()


def test_element_argument_checks(ctx):
    el = bs.bs_elem_create(ctx, 9)
    m = torch.zeros((10 ** 3), dtype=torch.int32, device="cuda")
    x = torch.zeros(8, dtype=F64, device="cuda")
    with pytest.raises(bs.BSError) as e:  # the local operator stops at N = 7
        bs.bs_helmholtz_local(ctx, el, m, torch.zeros(7, dtype=F64, device="cuda"), 1.0, x,
                              torch.zeros(10 ** 3, dtype=F64, device="cuda"))
    assert e.value.status == 2
    el.close()
    with pytest.raises(bs.BSError):
        bs.bs_elem_create(ctx, 16)


def _interior_problem(K, N, seed):
    """-Lap u = f on the unit cube, u = x(1-x) y(1-y) z(1-z) vanishing on the
    boundary: every copy of a boundary node masked, b the consistent mass of
    f against the interior test functions (all computed by the oracle)."""
    ids = _mesh(K, N, seed)
    X, Y, Z = elem.node_coordinates(K, N)
    on_bnd = np.zeros(X.size, dtype=bool)
    for c in (X, Y, Z):
        on_bnd |= (np.abs(c) < 1e-14) | (np.abs(c - 1.0) < 1e-14)
    masked = np.where(on_bnd[ids], -1, ids)
    geo = elem.geometry_cube(K)
    geo_mass = geo.copy()
    geo_mass[:, :6] = 0.0
    q = lambda t: t * (1.0 - t)  # noqa: E731
    u = q(X) * q(Y) * q(Z)
    f = 2.0 * (q(Y) * q(Z) + q(X) * q(Z) + q(X) * q(Y))
    b = np.where(on_bnd, 0.0, elem.apply_assembled(N, geo_mass, 1.0, ids, f))
    return masked, geo, u, b, on_bnd


def _solve(ctx, N, ids, geo, lam, b, tol, max_iter=100000, x0=None, check=True):
    NG = b.size
    plan = bs.bs_gs_create(ctx, torch.from_numpy(ids.astype(np.int32)).cuda(), NG)
    el = bs.bs_elem_create(ctx, N)
    x = torch.zeros(NG, dtype=F64, device="cuda") if x0 is None else torch.from_numpy(x0.copy()).cuda()
    try:
        res = bs.bs_helmholtz_cg_solve(ctx, el, plan, torch.from_numpy(geo.ravel()).cuda(), lam,
                                       torch.from_numpy(b).cuda(), x, tol, max_iter, check=check)
        return to_host(x), res
    finally:
        el.close()
        plan.close()


@pytest.mark.parametrize("K,N,seed", [(2, 3, 3), (3, 5, 4), (2, 7, None)])
def test_helmholtz_cg_recovers_a_polynomial_solution(ctx, K, N, seed):
    # u lies in the discrete space (degree 2 per axis, N >= 2): the Galerkin
    # solution is its interpolant, so the solve must return u at the nodes
    masked, geo, u, b, on_bnd = _interior_problem(K, N, seed)
    tol = 1e-12
    x, res = _solve(ctx, N, masked, geo, 0.0, b, tol)
    assert res["status"] == "BS_OK"
    r = b - elem.apply_assembled(N, geo, 0.0, masked, x)
    assert np.linalg.norm(r) <= tol * np.linalg.norm(b) * (1 + 1e-6)
    assert np.all(x[on_bnd] == 0.0)
    assert np.max(np.abs(x - u)) <= 1e-10
    # the oracle's Algorithm 1 on the same system takes about as many steps
    _, it_ref, _ = elem.helmholtz_cg(N, geo, 0.0, masked, b, tol=tol)
    assert abs(res["iterations"] - it_ref) <= max(3, it_ref // 10), (res["iterations"], it_ref)


@pytest.mark.parametrize("K,N,seed,lam", [(3, 4, 7, 0.5), (2, 7, 8, 10.0), (4, 2, 9, 0.01)])
def test_helmholtz_cg_matches_the_oracle(ctx, K, N, seed, lam):
    ids = _mesh(K, N, seed)
    E, NL, NG = mesh.sizes(K, N)
    geo = elem.geometry_cube(K)
    b = bsgen.uniform(21, 12, NG)
    tol = 1e-11
    x, res = _solve(ctx, N, ids, geo, lam, b, tol)
    assert res["status"] == "BS_OK" and res["iterations"] > 0
    r = b - elem.apply_assembled(N, geo, lam, ids, x)
    assert np.linalg.norm(r) <= tol * np.linalg.norm(b) * (1 + 1e-6)
    assert abs(res["rel_residual"] - np.linalg.norm(r) / np.linalg.norm(b)) <= 1e-3 * tol
    x_ref, it_ref, _ = elem.helmholtz_cg(N, geo, lam, ids, b, tol=tol)
    assert abs(res["iterations"] - it_ref) <= max(3, it_ref // 10), (res["iterations"], it_ref)
    assert np.linalg.norm(x - x_ref) <= 1e-6 * np.linalg.norm(x_ref)


def test_helmholtz_cg_limits_and_start(ctx):
    K, N, lam = 2, 4, 0.3
    ids = _mesh(K, N, 10)
    E, NL, NG = mesh.sizes(K, N)
    geo = elem.geometry_cube(K)
    b = bsgen.uniform(22, 12, NG)
    # three iterations, then the limit: the record says so and x moved
    x, res = _solve(ctx, N, ids, geo, lam, b, 1e-12, max_iter=3, check=False)
    assert res["status"] == "BS_ERR_NO_CONVERGENCE" and res["iterations"] == 3
    x3, _, _ = elem.helmholtz_cg(N, geo, lam, ids, b, tol=1e-30, max_iter=3)
    assert np.linalg.norm(x - x3) <= 1e-10 * np.linalg.norm(x3)
    # starting from a converged x takes no iteration
    x_ref, _, _ = elem.helmholtz_cg(N, geo, lam, ids, b, tol=1e-12)
    x2, res2 = _solve(ctx, N, ids, geo, lam, b, 1e-9, x0=x_ref)
    assert res2["status"] == "BS_OK" and res2["iterations"] == 0
    assert np.array_equal(x2, x_ref)
    # b = 0 from x = 0: done at once, x stays 0
    x0, res0 = _solve(ctx, N, ids, geo, lam, np.zeros(NG), 1e-9)
    assert res0["iterations"] == 0 and not np.any(x0)


def test_helmholtz_cg_argument_checks(ctx):
    K, N = 2, 3
    ids = _mesh(K, N, 1)
    E, NL, NG = mesh.sizes(K, N)
    plan = bs.bs_gs_create(ctx, torch.from_numpy(ids.astype(np.int32)).cuda(), NG)
    el = bs.bs_elem_create(ctx, N)
    geo = torch.from_numpy(elem.geometry_cube(K).ravel()).cuda()
    b = torch.ones(NG, dtype=F64, device="cuda")
    x = torch.zeros(NG, dtype=F64, device="cuda")
    try:
        for bad in ({"tol": 0.0}, {"max_iter": -1}):
            args = {"tol": 1e-10, "max_iter": 10, **bad}
            with pytest.raises(bs.BSError) as e:
                bs.bs_helmholtz_cg_solve(ctx, el, plan, geo, 1.0, b, x, args["tol"], args["max_iter"])
            assert e.value.status == 1
        with pytest.raises(bs.BSError):  # x overlapping b
            bs.bs_helmholtz_cg_solve(ctx, el, plan, geo, 1.0, b, b, 1e-10, 10)
        with pytest.raises(ValueError):  # wrong length
            bs.bs_helmholtz_cg_solve(ctx, el, plan, geo, 1.0, b[:-1], x[:-1], 1e-10, 10)
        big = bs.bs_elem_create(ctx, 9)  # the local operator stops at N = 7
        st = bs.lib.bs_helmholtz_cg_solve(ctx.handle, big.handle, plan.handle, geo.data_ptr(), 1.0, b.data_ptr(),
                                          x.data_ptr(), 1e-10, 10, None, None)
        assert st == 2
        big.close()
    finally:
        el.close()
        plan.close()
