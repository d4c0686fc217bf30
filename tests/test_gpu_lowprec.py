"""GPU parity of the binary32 and bfloat16 paths against the binary64 oracle.

Vectors are stored narrow (binary64 draws rounded to nearest even, exactly
as the device generator rounds them), arithmetic is binary32, reductions are
compensated binary32 finished in binary64.  The oracle works in binary64 on
the stored values; the bounds below follow from the arithmetic (u32 = 2^-24,
u_s the storage unit roundoff: 0 for binary32 results, 2^-8 for bfloat16):

  copy, scatter, weights   bit-exact on the stored bits
  axpy, cg_update vectors  |err| <= (u_s + 3 u32)(|a x| + |b y|)   (alpha and
                           beta are rounded to binary32 too)
  norm                     |err| <= 3 u32 S         (positive terms; binary32
                           squares of binary32 inputs are rounded)
  dot                      |err| <= 2 u32 |S| + 1e-12 sum|x y|  (exact products,
                           compensated sums)
  gather                   |err| <= u_s |S| + deg u32 sum|terms|
"""

import numpy as np
import pytest
import torch

import bsgen
from oracle import mesh, ops

pytestmark = pytest.mark.gpu

import paper_2009_10917_amd as bs  # noqa: E402
from gpu_util import scalar_out, to_host  # noqa: E402

U32 = 2.0 ** -24
DTYPES = {"f32": (torch.float32, 0.0), "bf16": (torch.bfloat16, 2.0 ** -8)}
SEED = 77
SIZES = [1, 7, 1000, 65_537, 1_000_003]


def stored(dt, n, stream, lo=-1.0):
    """Device vector in dtype dt and the binary64 values it holds."""
    t = torch.empty(n, dtype=dt, device="cuda")
    if n:
        bsgen.device_uniform(t, SEED, stream, lo=lo)
    return t, as_f64(t)


def as_f64(t):
    torch.cuda.synchronize()
    if t.dtype == torch.bfloat16:
        return bsgen.bf16_bits_to_f64(t.view(torch.int16).cpu().numpy().view(np.uint16))
    return t.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("name", list(DTYPES))
@pytest.mark.parametrize("n", SIZES)
def test_copy_bit_exact(ctx, name, n):
    dt, _ = DTYPES[name]
    x, _ = stored(dt, n, 1)
    y = torch.zeros_like(x)
    bs.bs_copy(ctx, x, y)
    torch.cuda.synchronize()
    assert torch.equal(x.view(torch.int16 if dt == torch.bfloat16 else torch.int32),
                       y.view(torch.int16 if dt == torch.bfloat16 else torch.int32))
    # the device generator rounds exactly like the host one
    ref = bsgen.uniform(SEED, 1, n)
    if dt == torch.float32:
        assert np.array_equal(to_host(x), bsgen.round_f32(ref))
    else:
        assert np.array_equal(to_host(x), bsgen.round_bf16_bits(ref))


@pytest.mark.parametrize("name", list(DTYPES))
@pytest.mark.parametrize("n", SIZES)
def test_axpy_within_bound(ctx, name, n):
    dt, us = DTYPES[name]
    a, b = 0.37, 0.91
    x, hx = stored(dt, n, 1)
    y, hy = stored(dt, n, 2)
    bs.bs_axpy(ctx, a, x, b, y)
    got = as_f64(y)
    exact = a * hx + b * hy  # binary64 products of short operands: far inside the bound
    bound = (us + 3 * U32) * (np.abs(a * hx) + np.abs(b * hy)) * 1.01 + 1e-40
    assert np.all(np.abs(got - exact) <= bound)


@pytest.mark.parametrize("name", list(DTYPES))
@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("weighted", [False, True])
def test_norm_within_bound(ctx, name, n, weighted):
    dt, _ = DTYPES[name]
    x, hx = stored(dt, n, 1)
    w, hw = stored(dt, n, 6, lo=0.0) if weighted else (None, None)
    o = scalar_out()
    bs.bs_norm(ctx, x, w, o)
    S = ops.norm(hx, hw)
    got = float(to_host(o)[0])
    assert abs(got - S) <= 3 * U32 * S + 1e-300
    if dt == torch.bfloat16:
        # bfloat16 squares (and weighted squares) are exact in binary32
        assert abs(got - S) <= 2 * U32 * S + 1e-300


@pytest.mark.parametrize("name", list(DTYPES))
@pytest.mark.parametrize("n", SIZES)
def test_dot_within_bound(ctx, name, n):
    dt, _ = DTYPES[name]
    x, hx = stored(dt, n, 1)
    y, hy = stored(dt, n, 2)
    o = scalar_out()
    bs.bs_dot(ctx, x, y, o)
    S = ops.dot(hx, hy)
    got = float(to_host(o)[0])
    assert abs(got - S) <= 2 * U32 * abs(S) + 1e-12 * float(np.sum(np.abs(hx * hy)))


@pytest.mark.parametrize("name", list(DTYPES))
def test_dot_compensation_binary32(ctx, name):
    # a cancelling pair far apart: an uncompensated binary32 sum loses the rest
    dt, _ = DTYPES[name]
    n = 400_001
    hx = bsgen.uniform(SEED, 1, n) * 1e-3
    hy = bsgen.uniform(SEED, 2, n)
    hx[3], hy[3] = 2.0 ** 20, 1.0
    hx[n - 2], hy[n - 2] = -(2.0 ** 20), 1.0
    x = torch.from_numpy(hx).to(dt).cuda()
    y = torch.from_numpy(hy).to(dt).cuda()
    hx, hy = as_f64(x), as_f64(y)
    o = scalar_out()
    bs.bs_dot(ctx, x, y, o)
    S = ops.dot(hx, hy)
    assert abs(float(to_host(o)[0]) - S) <= 2 * U32 * abs(S) + 1e-12 * float(np.sum(np.abs(hx * hy)))


@pytest.mark.parametrize("name", list(DTYPES))
@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("weighted", [False, True])
def test_cg_update_within_bound(ctx, name, n, weighted):
    dt, us = DTYPES[name]
    a = 0.37
    x, hx = stored(dt, n, 1)
    p, hp = stored(dt, n, 3)
    r, hr = stored(dt, n, 4)
    Ap, hA = stored(dt, n, 5)
    w, hw = stored(dt, n, 6, lo=0.0) if weighted else (None, None)
    o = scalar_out()
    bs.bs_cg_update(ctx, a, x, p, r, Ap, w, o)
    gx, gr = as_f64(x), as_f64(r)
    assert np.all(np.abs(gx - (hx + a * hp)) <= (us + 3 * U32) * (np.abs(hx) + np.abs(a * hp)) * 1.01 + 1e-40)
    assert np.all(np.abs(gr - (hr - a * hA)) <= (us + 3 * U32) * (np.abs(hr) + np.abs(a * hA)) * 1.01 + 1e-40)
    # the reduction is over the stored new residual
    S = ops.norm(gr, hw)
    assert abs(float(to_host(o)[0]) - S) <= 3 * U32 * S + 1e-300


@pytest.mark.parametrize("name", list(DTYPES))
def test_gather_scatter_weights(ctx, name):
    dt, us = DTYPES[name]
    K, N = 6, 5
    E, NL, NG = mesh.sizes(K, N)
    perm, orient = bsgen.permutation(SEED, E), bsgen.orientations(SEED, E)
    ids = mesh.hex_map(K, N, perm, orient)
    plan = bs.bs_gs_create(ctx, torch.from_numpy(ids.astype(np.int32)).cuda(), NG)
    rs, ci = mesh.csr_inverse(ids, NG)
    xL, hxL = stored(dt, NL, 11)
    xG = torch.empty(NG, dtype=dt, device="cuda")
    bs.bs_gather(ctx, plan, xL, xG)
    got = as_f64(xG)
    S = ops.gather(rs, ci, hxL)
    A = ops.gather(rs, ci, np.abs(hxL))
    deg = np.diff(rs)
    assert np.all(np.abs(got - S) <= us * np.abs(S) + deg * U32 * A + 1e-40)
    # scatter copies stored values exactly
    g2, hg2 = stored(dt, NG, 12)
    bs.bs_gs_scatter(ctx, plan, g2, xL)
    assert np.array_equal(as_f64(xL), hg2[ids])
    # weights round 1/deg to the storage type
    wL = torch.empty(NL, dtype=dt, device="cuda")
    bs.bs_gs_weights(plan, wL)
    w64 = mesh.weights(ids, NG)
    if dt == torch.float32:
        assert np.array_equal(to_host(wL), bsgen.round_f32(w64))
    else:
        assert np.array_equal(to_host(wL), bsgen.round_bf16_bits(w64))
    # and the weighted norm of ones is still the global node count
    o = scalar_out()
    bs.bs_norm(ctx, torch.ones(NL, dtype=dt, device="cuda"), wL, o)
    assert float(to_host(o)[0]) == float(NG)


@pytest.mark.parametrize("name", list(DTYPES))
def test_gather_scatter_every_variant(name):
    # every gather variant adds each row's copies in the same order in the
    # same type, so all give the same bits (also after the lattice row
    # order); every scatter variant copies stored values exactly
    dt, us = DTYPES[name]
    K, N = 7, 7
    E, NL, NG = mesh.sizes(K, N)
    M = K * N + 1
    perm, orient = bsgen.permutation(SEED, E), bsgen.orientations(SEED, E)
    ids = mesh.hex_map(K, N, perm, orient)
    ids[5::37] = -1
    c = bs.bs_ctx_create(0)  # its own context: one launch shape for every length
    plan = bs.bs_gs_create(c, torch.from_numpy(ids.astype(np.int32)).cuda(), NG)
    rs, ci = mesh.csr_inverse(ids, NG)
    xL, hxL = stored(dt, NL, 11)
    S = ops.gather(rs, ci, hxL)
    A = ops.gather(rs, ci, np.abs(hxL))
    deg = np.diff(rs)
    outs = []
    for order in ("plan", "lattice"):
        if order == "lattice":
            bs.bs_gs_order_rows(plan, M, M, M, 21, (21, 7, 7))
        for v in (0, 1, 2, 4, 5, 6):
            bs.bs_ctx_set_tune(c, "gather", 1, 1 << 30, v)
            xG = torch.full((NG,), float("nan"), dtype=dt, device="cuda")
            bs.bs_gather(c, plan, xL, xG)
            got = as_f64(xG)
            assert np.all(np.abs(got - S) <= us * np.abs(S) + deg * U32 * A + 1e-40), (order, v)
            outs.append(got.view(np.int64).copy())
    assert all(np.array_equal(outs[0], o) for o in outs[1:])
    g2, hg2 = stored(dt, NG, 12)
    ref = hxL.copy()
    ref[ids >= 0] = hg2[ids[ids >= 0]]
    for v in (0, 1, 2, 4, 5, 6):
        for u in ((1, 2, 4) if v % 4 < 2 else (1, 8)):
            bs.bs_ctx_set_tune(c, "scatter", u, 1 << 30, v)
            x2 = xL.clone()
            bs.bs_gs_scatter(c, plan, g2, x2)
            assert np.array_equal(as_f64(x2), ref), (v, u)
    torch.cuda.synchronize()
    plan.close()
    c.close()
