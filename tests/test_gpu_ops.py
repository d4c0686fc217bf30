"""GPU parity of BS1-BS5 (binary64) against the oracle.

Copy, AXPY and the vector part of the fused CG update are compared bit for
bit; the reductions must lie within 1e-14 relative of the oracle's
correctly rounded exact sum.  Sizes span several 256-thread tiles and grid
trips, with ragged tails and 8-byte (not 16-byte) aligned pointers.
"""

import numpy as np
import pytest
import torch

import bsgen
from oracle import ops

pytestmark = pytest.mark.gpu

import paper_2009_10917_amd as bs  # noqa: E402
from gpu_util import bits, dev_uniform, host_uniform, rel_err, scalar_out, to_host  # noqa: E402

SIZES = [0, 1, 2, 3, 7, 255, 256, 257, 2047, 2048, 2049, 100003, (1 << 20) + 3, 5_000_011]
OFFSETS = [(0, 0), (1, 1), (1, 0), (0, 1)]  # element offsets of the two main operands
TOL = 1e-14


def test_device_generator_matches_host_generator():
    for n, start in ((1, 0), (1000, 0), (4097, 123456)):
        for stream in (1, 6):
            for lo in (-1.0, 0.0):
                t = torch.empty(n, dtype=torch.float64, device="cuda")
                bsgen.device_uniform(t, 77, stream, lo=lo, start=start)
                ref = bsgen.uniform(77, stream, n, lo=lo, start=start)
                assert np.array_equal(bits(to_host(t)), bits(ref))
    x = bsgen.uniform(5, 2, 10000)
    t32 = torch.empty(10000, dtype=torch.float32, device="cuda")
    bsgen.device_uniform(t32, 5, 2)
    assert np.array_equal(to_host(t32), bsgen.round_f32(x))
    t16 = torch.empty(10000, dtype=torch.bfloat16, device="cuda")
    bsgen.device_uniform(t16, 5, 2)
    assert np.array_equal(to_host(t16), bsgen.round_bf16_bits(x))


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("offs", OFFSETS)
def test_copy_bit_exact(ctx, n, offs):
    x = dev_uniform(n, 1, offset=offs[0])
    y = dev_uniform(n, 2, offset=offs[1])
    bs.bs_copy(ctx, x, y)
    assert np.array_equal(bits(to_host(y)), bits(host_uniform(n, 1)))


def test_copy_special_values(ctx):
    special = np.array([0.0, -0.0, np.inf, -np.inf, 5e-324, -1.5], dtype=np.float64)
    nans = np.array([0x7FF8000000000ABC, 0xFFF0000000000001, 0x7FF0000000C0FFEE], dtype=np.uint64).view(np.float64)
    src = np.tile(np.concatenate([special, nans]), 1000)
    x = torch.from_numpy(src).cuda()
    y = torch.zeros_like(x)
    bs.bs_copy(ctx, x, y)
    assert np.array_equal(bits(to_host(y)), bits(src))


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("offs", OFFSETS)
@pytest.mark.parametrize("ab", [(0.37, 1.0), (1.0, 0.37), (-2.5, 0.0)])
def test_axpy_bit_exact(ctx, n, offs, ab):
    a, b = ab
    x = dev_uniform(n, 1, offset=offs[0])
    y = dev_uniform(n, 2, offset=offs[1])
    bs.bs_axpy(ctx, a, x, b, y)
    ref = ops.axpy(a, host_uniform(n, 1), b, host_uniform(n, 2))
    assert np.array_equal(bits(to_host(y)), bits(ref))


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("offs", [(0, 0), (1, 1), (1, 0)])
def test_norm_within_tolerance(ctx, n, weighted, offs):
    x = dev_uniform(n, 1, offset=offs[0])
    w = dev_uniform(n, 6, lo=0.0, offset=offs[1]) if weighted else None
    out = scalar_out()
    bs.bs_norm(ctx, x, w, out)
    ref = ops.norm(host_uniform(n, 1), host_uniform(n, 6, lo=0.0) if weighted else None)
    got = float(to_host(out)[0])
    if n == 0:
        assert got == 0.0
    assert rel_err(got, ref) <= TOL, (got, ref)


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("offs", [(0, 0), (1, 1), (0, 1)])
def test_dot_within_tolerance(ctx, n, offs):
    x = dev_uniform(n, 1, offset=offs[0])
    y = dev_uniform(n, 2, offset=offs[1])
    out = scalar_out()
    bs.bs_dot(ctx, x, y, out)
    ref = ops.dot(host_uniform(n, 1), host_uniform(n, 2))
    got = float(to_host(out)[0])
    assert rel_err(got, ref) <= TOL, (got, ref)


def test_dot_compensation_under_cancellation(ctx):
    # two terms of +-1e16 far apart in the vector cancel exactly; an
    # uncompensated binary64 sum loses the O(1) remainder's low digits
    n = 3_000_017
    xh = host_uniform(n, 1)
    yh = host_uniform(n, 2)
    xh[7], yh[7] = 1e16, 1.0
    xh[n - 5], yh[n - 5] = -1e16, 1.0
    xh[n // 2], yh[n // 2] = 3e15, 3.0
    xh[n // 3], yh[n // 3] = -9e15, 1.0
    x, y = torch.from_numpy(xh).cuda(), torch.from_numpy(yh).cuda()
    out = scalar_out()
    bs.bs_dot(ctx, x, y, out)
    ref = ops.dot(xh, yh)
    assert rel_err(float(to_host(out)[0]), ref) <= TOL


def test_dot_of_x_with_itself_equals_norm(ctx):
    n = 2_000_003
    x = dev_uniform(n, 1)
    a, b = scalar_out(), scalar_out()
    bs.bs_dot(ctx, x, x, a)
    bs.bs_norm(ctx, x, None, b)
    assert rel_err(float(to_host(a)[0]), float(to_host(b)[0])) <= TOL


def test_norm_constant_vector_exact(ctx):
    for n in (1, 1000, 4_194_304 + 77):
        for c in (1.0, 0.5, -3.0):
            x = torch.full((n,), c, dtype=torch.float64, device="cuda")
            out = scalar_out()
            bs.bs_norm(ctx, x, None, out)
            assert float(to_host(out)[0]) == n * c * c


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("alpha", [0.37, 0.0])
def test_cg_update(ctx, n, weighted, alpha):
    x, p, r, Ap = (dev_uniform(n, s) for s in (1, 3, 4, 5))
    w = dev_uniform(n, 6, lo=0.0) if weighted else None
    out = scalar_out()
    bs.bs_cg_update(ctx, alpha, x, p, r, Ap, w, out)
    hx, hp, hr, hA = (host_uniform(n, s) for s in (1, 3, 4, 5))
    hw = host_uniform(n, 6, lo=0.0) if weighted else None
    xr, rr, rho = ops.cg_update(alpha, hx, hp, hr, hA, hw)
    assert np.array_equal(bits(to_host(x)), bits(xr))
    assert np.array_equal(bits(to_host(r)), bits(rr))
    assert rel_err(float(to_host(out)[0]), rho) <= TOL
    if alpha == 0.0:
        assert np.array_equal(bits(to_host(r)), bits(hr))


def test_cg_update_unaligned(ctx):
    n = 100_003
    x, p, r, Ap = (dev_uniform(n, s, offset=1) for s in (1, 3, 4, 5))
    out = scalar_out()
    bs.bs_cg_update(ctx, 0.37, x, p, r, Ap, None, out)
    xr, rr, rho = ops.cg_update(0.37, *(host_uniform(n, s) for s in (1, 3, 4, 5)))
    assert np.array_equal(bits(to_host(x)), bits(xr)) and np.array_equal(bits(to_host(r)), bits(rr))
    assert rel_err(float(to_host(out)[0]), rho) <= TOL


def test_reductions_deterministic(ctx):
    n = 3_000_001
    x, y = dev_uniform(n, 1), dev_uniform(n, 2)
    outs = []
    for _ in range(4):
        o = scalar_out()
        bs.bs_dot(ctx, x, y, o)
        outs.append(to_host(o)[0])
    assert len({np.float64(v).tobytes() for v in outs}) == 1


@pytest.mark.parametrize("unroll", [1, 2, 4, 8])
@pytest.mark.parametrize("cap", [1, 7, 300, 8192, 65536])
def test_launch_shapes_do_not_change_results(unroll, cap):
    n = 1_000_003
    # its own context: one launch shape for every length replaces the whole tune table
    ctx = bs.bs_ctx_create(0)
    try:
        for op in ("copy", "axpy", "norm", "dot", "cg_update"):
            bs.bs_ctx_set_tune(ctx, op, unroll, cap)
        x, y = dev_uniform(n, 1), dev_uniform(n, 2)
        bs.bs_axpy(ctx, 0.37, x, 1.0, y)
        assert np.array_equal(bits(to_host(y)), bits(ops.axpy(0.37, host_uniform(n, 1), 1.0, host_uniform(n, 2))))
        z = torch.empty_like(x)
        bs.bs_copy(ctx, x, z)
        assert np.array_equal(bits(to_host(z)), bits(host_uniform(n, 1)))
        o = scalar_out()
        bs.bs_dot(ctx, x, z, o)
        assert rel_err(float(to_host(o)[0]), ops.norm(host_uniform(n, 1))) <= TOL
    finally:
        torch.cuda.synchronize()
        ctx.close()


@pytest.fixture(scope="module")
def order_case():
    # long enough that unroll 1 launches several groups of 2048 workgroups and a ragged last one
    n = 9_000_017
    h = {k: host_uniform(n, s, lo=0.0 if k == "w" else -1.0) for k, s in (("x", 1), ("y", 2), ("p", 3), ("Ap", 4), ("w", 5))}
    xr, rr, rho = ops.cg_update(0.37, h["x"], h["p"], h["y"], h["Ap"], h["w"])
    return n, {"axpy": bits(ops.axpy(0.37, h["x"], 0.61, h["y"])), "norm": ops.norm(h["x"], h["w"]),
               "dot": ops.dot(h["x"], h["y"]), "cg_x": bits(xr), "cg_r": bits(rr), "cg_rho": rho,
               "x": bits(h["x"])}


@pytest.mark.parametrize("order", [1, 2, 4, 5, 6, 8, 9, 10])
@pytest.mark.parametrize("unroll,cap", [(1, 1 << 30), (4, 65536), (2, 3000), (8, 7)])
def test_workgroup_orders_do_not_change_results(order_case, order, unroll, cap):
    # variant 1 and 2 of the streaming operations renumber workgroups per XCD, + 4 and + 8
    # run 128- and 512-thread workgroups; every element is still handled once, so vectors
    # stay bit-exact and sums within tolerance
    n, want = order_case
    ctx = bs.bs_ctx_create(0)
    try:
        for op in ("copy", "axpy", "norm", "dot", "cg_update"):
            bs.bs_ctx_set_tune(ctx, op, unroll, cap, order)
            assert bs.bs_ctx_tune_for(ctx, op, n) == (unroll, cap, order)
        x, y, p, Ap, w = (dev_uniform(n, s, lo=0.0 if s == 5 else -1.0) for s in (1, 2, 3, 4, 5))
        z = torch.full_like(x, float("nan"))
        bs.bs_copy(ctx, x, z)
        assert np.array_equal(bits(to_host(z)), want["x"])
        o = scalar_out()
        bs.bs_norm(ctx, x, w, o)
        assert rel_err(float(to_host(o)[0]), want["norm"]) <= TOL
        bs.bs_dot(ctx, x, y, o)
        assert rel_err(float(to_host(o)[0]), want["dot"]) <= TOL
        r = y.clone()
        bs.bs_cg_update(ctx, 0.37, z, p, r, Ap, w, o)
        assert np.array_equal(bits(to_host(z)), want["cg_x"]) and np.array_equal(bits(to_host(r)), want["cg_r"])
        assert rel_err(float(to_host(o)[0]), want["cg_rho"]) <= TOL
        bs.bs_axpy(ctx, 0.37, x, 0.61, y)
        assert np.array_equal(bits(to_host(y)), want["axpy"])
    finally:
        torch.cuda.synchronize()
        ctx.close()


@pytest.mark.parametrize("unroll,cap", [(1, 16384), (1, 16385), (1, 1 << 30), (8, 1 << 30)])
def test_reductions_past_the_direct_finish(order_case, unroll, cap):
    # above 16384 workgroups the pairs are first added in chunks of 4096 (cap 16385 leaves a
    # last chunk of one pair), then the chunk sums in order: sums stay within the tolerance
    # and repeat bit for bit
    n, want = order_case
    ctx = bs.bs_ctx_create(0)
    try:
        for op in ("norm", "dot", "cg_update"):
            bs.bs_ctx_set_tune(ctx, op, unroll, cap)
        x, y, p, Ap, w = (dev_uniform(n, s, lo=0.0 if s == 5 else -1.0) for s in (1, 2, 3, 4, 5))
        o1, o2 = scalar_out(), scalar_out()
        bs.bs_norm(ctx, x, w, o1)
        bs.bs_norm(ctx, x, w, o2)
        assert rel_err(float(to_host(o1)[0]), want["norm"]) <= TOL
        assert bits(to_host(o1)) == bits(to_host(o2))
        bs.bs_dot(ctx, x, y, o1)
        bs.bs_dot(ctx, x, y, o2)
        assert rel_err(float(to_host(o1)[0]), want["dot"]) <= TOL
        assert bits(to_host(o1)) == bits(to_host(o2))
        bs.bs_cg_update(ctx, 0.37, x, p, y, Ap, w, o1)
        assert np.array_equal(bits(to_host(x)), want["cg_x"]) and np.array_equal(bits(to_host(y)), want["cg_r"])
        assert rel_err(float(to_host(o1)[0]), want["cg_rho"]) <= TOL
    finally:
        torch.cuda.synchronize()
        ctx.close()


def test_error_paths(ctx):
    L = bs.lib
    x = torch.zeros(64, dtype=torch.float64, device="cuda")
    y = torch.zeros(64, dtype=torch.float64, device="cuda")
    o = scalar_out()
    s = torch.cuda.current_stream().cuda_stream
    INVALID = 1
    h = ctx.handle
    assert L.bs_copy(h, 0, -1, x.data_ptr(), y.data_ptr(), s) == INVALID
    assert L.bs_copy(h, 0, 10, None, y.data_ptr(), s) == INVALID
    assert L.bs_copy(h, 0, 10, x.data_ptr() + 1, y.data_ptr(), s) == INVALID  # misaligned
    assert L.bs_copy(h, 9, 10, x.data_ptr(), y.data_ptr(), s) == INVALID  # unknown dtype
    assert L.bs_copy(h, 0, 10, x.data_ptr(), x.data_ptr() + 8, s) == INVALID  # overlap
    assert L.bs_axpy(h, 0, 10, 1.0, x.data_ptr(), 1.0, x.data_ptr(), s) == INVALID  # y aliases x
    assert L.bs_norm(h, 0, 10, x.data_ptr(), None, None, s) == INVALID
    assert L.bs_dot(h, 0, 10, x.data_ptr(), y.data_ptr(), o.data_ptr() + 4, s) == INVALID
    assert L.bs_cg_update(h, 0, 10, 1.0, x.data_ptr(), y.data_ptr(), x.data_ptr(), y.data_ptr(), None,
                          o.data_ptr(), s) == INVALID  # r aliases x
    assert L.bs_ctx_set_tune(h, 0, 0, 3, 16, 0) == INVALID
    assert L.bs_ctx_set_tune(h, 99, 0, 4, 16, 0) == INVALID
    assert L.bs_ctx_set_tune(h, 0, 0, 4, 16, 3) == INVALID
    assert L.bs_ctx_set_tune(h, 0, 0, 4, 16, 12) == INVALID  # dispatch order and XCD runs at once
    assert L.bs_ctx_set_tune(h, 0, 0, 4, 16, 11) == INVALID
    assert L.bs_ctx_set_tune(h, 0, 0, 4, 16, 16 + 3) == INVALID
    assert L.bs_ctx_set_tune(h, 0, 0, 4, 16, 16 + 12) == INVALID
    assert L.bs_ctx_set_tune(h, 0, 0, 4, 16, 32) == INVALID
    # n == 0 with NULL pointers is a valid no-op; reductions write 0
    assert L.bs_copy(h, 0, 0, None, None, s) == 0
    assert L.bs_dot(h, 0, 0, None, None, o.data_ptr(), s) == 0
    assert float(to_host(o)[0]) == 0.0
    with pytest.raises(bs.BSError):
        bs.bs_copy(ctx, x, x)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16])
@pytest.mark.parametrize("n", [1, 77, 4097, 1_000_003])
@pytest.mark.parametrize("unroll,cap", [(1, 1), (4, 1 << 30), (2, 300)])
def test_workgroup_sizes_agree(dtype, n, unroll, cap):
    # 128- and 512-thread workgroups (variant + 4, + 8) against 256: vectors bit-identical,
    # reductions within the compensated sums' tolerance
    res = {}
    for v in (0, 4, 8):
        ctx = bs.bs_ctx_create(0)
        try:
            for op in ("copy", "axpy", "norm", "dot", "cg_update"):
                bs.bs_ctx_set_tune(ctx, op, unroll, cap, v)
            x, y, p, Ap, w = (dev_uniform(n, s, lo=0.0 if s == 5 else -1.0, dtype=dtype) for s in (1, 2, 3, 4, 5))
            z = torch.empty_like(x)
            bs.bs_copy(ctx, x, z)
            o = torch.zeros(3, dtype=torch.float64, device="cuda")
            bs.bs_norm(ctx, x, w, o[0:1])
            bs.bs_dot(ctx, x, y, o[1:2])
            bs.bs_cg_update(ctx, 0.37, z, p, y, Ap, w, o[2:3])
            bs.bs_axpy(ctx, 0.37, x, 0.61, p)
            res[v] = [bits(to_host(t)) for t in (z, y, p)] + list(to_host(o))
        finally:
            torch.cuda.synchronize()
            ctx.close()
    for v in (4, 8):
        for a, b in zip(res[0][:3], res[v][:3]):
            assert np.array_equal(a, b), v
        for a, b in zip(res[0][3:], res[v][3:]):
            if dtype == torch.float64:
                assert rel_err(b, a) <= 1e-14, (v, a, b)
            else:  # compensated binary32 sums of n terms of magnitude <= 1: within 2u * n each
                assert abs(b - a) <= 4 * 2.0 ** -24 * n, (v, a, b)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16])
@pytest.mark.parametrize("n,unroll,cap,order", [(1000003, 4, 1 << 30, 0), (4194305, 8, 4096, 1), (777, 1, 1, 2)])
def test_cache_policies_agree(dtype, n, unroll, cap, order):
    # cached accesses (variant + 16) against nontemporal ones: every vector and
    # every reduction bit-identical (same packets, same order of additions)
    res = {}
    for v in (order, order + 16, order + 4 + 16):
        ctx = bs.bs_ctx_create(0)
        try:
            for op in ("copy", "axpy", "norm", "dot", "cg_update"):
                bs.bs_ctx_set_tune(ctx, op, unroll, cap, v)
            x, y, p, Ap, w = (dev_uniform(n, s, lo=0.0 if s == 5 else -1.0, dtype=dtype) for s in (1, 2, 3, 4, 5))
            z = torch.empty_like(x)
            bs.bs_copy(ctx, x, z)
            o = torch.zeros(3, dtype=torch.float64, device="cuda")
            bs.bs_norm(ctx, x, w, o[0:1])
            bs.bs_dot(ctx, x, y, o[1:2])
            bs.bs_cg_update(ctx, 0.37, z, p, y, Ap, w, o[2:3])
            bs.bs_axpy(ctx, 0.37, x, 0.61, p)
            res[v] = [bits(to_host(t)) for t in (z, y, p)] + [bits(to_host(o))]
        finally:
            torch.cuda.synchronize()
            ctx.close()
    for a, b in zip(res[order], res[order + 16]):
        assert np.array_equal(a, b)
    # with a different workgroup size only the vectors stay bit-identical
    for a, b in zip(res[order][:3], res[order + 4 + 16][:3]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_single_launch_finish_across_its_limit(dtype):
    # grids of up to 128 workgroups add the pairs in the launch that reads the vectors (the
    # last workgroup to take a ticket does it and resets the counter); 129 and more use a
    # second launch. Calls alternate between the two so that a counter left nonzero would
    # show; each cap repeats bit for bit, and every sum stays within the tolerance.
    n = 300_007
    tol = TOL if dtype == torch.float64 else 1e-6
    h = {k: host_uniform(n, s, lo=0.0 if k == "w" else -1.0) for k, s in (("x", 1), ("y", 2), ("w", 5))}
    if dtype == torch.float32:
        h = {k: v.astype(np.float32).astype(np.float64) for k, v in h.items()}
    want_norm, want_dot = ops.norm(h["x"], h["w"]), ops.dot(h["x"], h["y"])
    x, y, w = (torch.from_numpy(h[k]).to(dtype).cuda() for k in ("x", "y", "w"))
    ctx = bs.bs_ctx_create(0)
    try:
        seen = {}
        for cap in (2, 128, 129, 64, 300, 127, 128, 2, 129):
            for op in ("norm", "dot"):
                bs.bs_ctx_set_tune(ctx, op, 1, cap)
            o = scalar_out()
            bs.bs_norm(ctx, x, w, o)
            nv = to_host(o).copy()
            bs.bs_dot(ctx, x, y, o)
            dv = to_host(o).copy()
            assert rel_err(float(nv[0]), want_norm) <= tol and rel_err(float(dv[0]), want_dot) <= tol, cap
            if cap in seen:
                assert np.array_equal(bits(seen[cap][0]), bits(nv)), cap
                assert np.array_equal(bits(seen[cap][1]), bits(dv)), cap
            seen[cap] = (nv, dv)
    finally:
        torch.cuda.synchronize()
        ctx.close()


def test_single_launch_finish_in_graph_replays():
    # the ticket counter is reset by the kernel itself (no memset), so a captured sequence of
    # finishing launches gives the eager bits on every replay, with eager work in between
    n = 200_003
    x, y, w = dev_uniform(n, 1), dev_uniform(n, 2), dev_uniform(n, 5, lo=0.0)
    ctx = bs.bs_ctx_create(0)
    try:
        for op in ("norm", "dot"):
            bs.bs_ctx_set_tune(ctx, op, 2, 100)
        eager_n, eager_d = scalar_out(), scalar_out()
        bs.bs_norm(ctx, x, w, eager_n)
        bs.bs_dot(ctx, x, y, eager_d)
        want = (bits(to_host(eager_n)), bits(to_host(eager_d)))
        gn, gd = scalar_out(), scalar_out()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            bs.bs_norm(ctx, x, w, gn)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(3):
                bs.bs_norm(ctx, x, w, gn)
                bs.bs_dot(ctx, x, y, gd)
        for _ in range(3):
            gn.fill_(0.0)
            gd.fill_(0.0)
            g.replay()
            torch.cuda.synchronize()
            assert np.array_equal(bits(to_host(gn)), want[0]) and np.array_equal(bits(to_host(gd)), want[1])
            o = scalar_out()
            bs.bs_dot(ctx, x, w, o)  # eager work between replays
            torch.cuda.synchronize()
        del g
    finally:
        torch.cuda.synchronize()
        ctx.close()
