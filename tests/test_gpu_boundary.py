"""The remaining entry points of the C ABI: the map-based scatter and the
device-scalar forms of AXPY and the fused CG update.

bs_scatter reads the scatter ids directly (Listing 5): it must equal the
oracle's scatter bit for bit, masked ids leaving x_L untouched.  The
device-scalar forms read alpha and beta as num / den from device memory
(Algorithm 1, steps 7-11): with the same scalar they give the host forms'
bits, and a whole CG iteration built from public calls (operator, dot, the
fused update with alpha = r.r / p.Ap, the direction update with
beta = r'.r' / r.r) captures into one graph whose replays follow the
oracle's Algorithm 1.
"""

import math

import numpy as np
import pytest
import torch

import bsgen
from oracle import cg, mesh, ops

pytestmark = pytest.mark.gpu

import paper_2009_10917_amd as bs  # noqa: E402
from gpu_util import bits, dev_uniform, host_uniform, rel_err, scalar_out, to_host  # noqa: E402

TORCH = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}


def _host_values(n, stream, dt):
    """The seeded values as stored in dtype dt, held exactly in binary64."""
    v = host_uniform(n, stream)
    if dt == "f32":
        return bsgen.round_f32(v).astype(np.float64)
    if dt == "bf16":
        return bsgen.bf16_bits_to_f64(bsgen.round_bf16_bits(v))
    return v


def _stored_bits(v, dt):
    if dt == "f64":
        return bits(v)
    if dt == "f32":
        return bits(v.astype(np.float32))
    return bsgen.round_bf16_bits(v)  # exact: v holds bfloat16 values


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("trim", [0, 37])
def test_map_scatter_bit_exact_with_masks(ctx, dt, trim):
    K, N = 4, 3
    E, NL, NG = mesh.sizes(K, N)
    ids = mesh.hex_map(K, N, bsgen.permutation(4, E), bsgen.orientations(4, E)).copy()
    ids[::7] = -1             # masked
    ids[5::11] = NG + 5       # out of range: treated as masked
    ids[6::13] = -(2 ** 31)
    nl = NL - trim            # a ragged local length
    ids = ids[:nl]
    d_map = torch.from_numpy(ids.astype(np.int32)).cuda()
    xG = dev_uniform(NG, 12, dtype=TORCH[dt])
    xL = dev_uniform(nl, 11, dtype=TORCH[dt])
    bs.bs_scatter(ctx, d_map, xG, xL)
    gb, lb = _host_values(NG, 12, dt), _host_values(nl, 11, dt)
    ref = ops.scatter(np.where(ids >= NG, -1, ids), gb, lb)
    assert np.array_equal(bits(to_host(xL)), _stored_bits(ref, dt))


def test_map_scatter_equals_plan_scatter_and_empty(ctx):
    K, N = 5, 4
    E, NL, NG = mesh.sizes(K, N)
    d_map = torch.from_numpy(mesh.hex_map(K, N, bsgen.permutation(8, E), bsgen.orientations(8, E))
                             .astype(np.int32)).cuda()
    plan = bs.bs_gs_create(ctx, d_map, NG)
    xG = dev_uniform(NG, 12)
    a, b = torch.zeros(NL, dtype=torch.float64, device="cuda"), torch.ones(NL, dtype=torch.float64, device="cuda")
    bs.bs_scatter(ctx, d_map, xG, a)
    bs.bs_gs_scatter(ctx, plan, xG, b)
    assert torch.equal(a.view(torch.int64), b.view(torch.int64))
    empty = torch.empty(0, dtype=torch.int32, device="cuda")
    bs.bs_scatter(ctx, empty, xG, torch.empty(0, dtype=torch.float64, device="cuda"))
    with pytest.raises(bs.BSError):  # x_L overlapping x_G
        bs.bs_scatter(ctx, d_map[:NG], xG, xG)
    plan.close()


def _scalars(*vals):
    return [torch.tensor([v], dtype=torch.float64, device="cuda") for v in vals]


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("n", [0, 1, 257, 100003])
def test_axpy_dev_equals_host_form(ctx, dt, n):
    an, ad, bn, bd = 0.9, 2.3, -1.7, 3.1
    alpha = 0.5 * (an / ad)
    beta = 2.0 * (bn / bd)
    a_num, a_den, b_num, b_den = _scalars(an, ad, bn, bd)
    x = dev_uniform(n, 1, dtype=TORCH[dt])
    y1 = dev_uniform(n, 2, dtype=TORCH[dt])
    y2 = y1.clone()
    bs.bs_axpy_dev(ctx, x, y1, alpha=0.5, alpha_num=a_num, alpha_den=a_den, beta=2.0, beta_num=b_num,
                   beta_den=b_den)
    bs.bs_axpy(ctx, alpha, x, beta, y2)
    assert np.array_equal(bits(to_host(y1)), bits(to_host(y2)))
    if dt == "f64":
        ref = ops.axpy(alpha, host_uniform(n, 1), beta, host_uniform(n, 2))
        assert np.array_equal(bits(to_host(y1)), bits(ref))
    # only a numerator, and no device scalar at all
    y3 = dev_uniform(n, 2, dtype=TORCH[dt])
    bs.bs_axpy_dev(ctx, x, y3, alpha_num=a_num, beta=0.25)
    y4 = dev_uniform(n, 2, dtype=TORCH[dt])
    bs.bs_axpy(ctx, an, x, 0.25, y4)
    assert np.array_equal(bits(to_host(y3)), bits(to_host(y4)))


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("n", [0, 3, 2049, 1_000_003])
@pytest.mark.parametrize("weighted", [False, True])
def test_cg_update_dev_equals_host_form(ctx, dt, n, weighted):
    num, den = 0.8125, 1.3
    alpha = num / den
    d_num, d_den = _scalars(num, den)
    v = {k: dev_uniform(n, s, dtype=TORCH[dt]) for k, s in (("x", 1), ("p", 3), ("r", 4), ("Ap", 5))}
    w = dev_uniform(n, 6, dtype=TORCH[dt], lo=0.0) if weighted else None
    u = {k: t.clone() for k, t in v.items()}
    o1, o2 = scalar_out(), scalar_out()
    bs.bs_cg_update_dev(ctx, v["x"], v["p"], v["r"], v["Ap"], w, o1, alpha_num=d_num, alpha_den=d_den)
    bs.bs_cg_update(ctx, alpha, u["x"], u["p"], u["r"], u["Ap"], w, o2)
    for k in ("x", "r"):
        assert np.array_equal(bits(to_host(v[k])), bits(to_host(u[k]))), k
    assert to_host(o1)[0] == to_host(o2)[0]
    if dt == "f64":
        hw = host_uniform(n, 6, lo=0.0) if weighted else None
        xr, rr, rho = ops.cg_update(alpha, host_uniform(n, 1), host_uniform(n, 3), host_uniform(n, 4),
                                    host_uniform(n, 5), hw)
        assert np.array_equal(bits(to_host(v["x"])), bits(xr)) and np.array_equal(bits(to_host(v["r"])), bits(rr))
        assert rel_err(to_host(o1)[0], rho) <= 1e-14


def test_dev_scalar_argument_checks(ctx):
    x = dev_uniform(16, 1)
    y = dev_uniform(16, 2)
    o = scalar_out()
    with pytest.raises(bs.BSError):  # the reduction result may not be a scalar input
        bs.bs_cg_update_dev(ctx, x, y, y.clone(), y.clone(), None, o, alpha_num=o)
    with pytest.raises(ValueError):
        bs.bs_axpy_dev(ctx, x, y, alpha_num=torch.zeros(2, dtype=torch.float64, device="cuda"))
    L = bs.lib
    s = torch.cuda.current_stream().cuda_stream
    # a misaligned scalar pointer is rejected on the host
    assert L.bs_axpy_dev(ctx.handle, 0, 16, 1.0, o.data_ptr() + 4, None, x.data_ptr(), 1.0, None, None,
                         y.data_ptr(), s) == 1


SHIFT = 0.01


def _iteration(ctx, m, v):
    """One CG iteration (Algorithm 1) from public calls only."""
    bs.bs_stencil7(ctx, m, SHIFT, v["p"], v["Ap"])
    bs.bs_dot(ctx, v["p"], v["Ap"], v["pAp"])
    bs.bs_cg_update_dev(ctx, v["x"], v["p"], v["r"], v["Ap"], None, v["rr_new"], alpha_num=v["rr"],
                        alpha_den=v["pAp"])
    bs.bs_axpy_dev(ctx, v["r"], v["p"], alpha=1.0, beta_num=v["rr_new"], beta_den=v["rr"])
    bs.bs_copy(ctx, v["rr_new"], v["rr"])


def _start(ctx, m, b):
    n = m ** 3
    v = {"x": torch.zeros(n, dtype=torch.float64, device="cuda"),
         "r": torch.from_numpy(b).cuda(), "p": torch.from_numpy(b).cuda(),
         "Ap": torch.empty(n, dtype=torch.float64, device="cuda")}
    for k in ("rr", "rr_new", "pAp"):
        v[k] = scalar_out()
    bs.bs_norm(ctx, v["r"], None, v["rr"])
    return v


def test_cg_iteration_from_public_calls_captured_in_a_graph(ctx):
    m = 21
    b = bsgen.uniform(5, bsgen.STREAM["b"], m ** 3)
    eager = _start(ctx, m, b)
    cap = _start(ctx, m, b)
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        _iteration(ctx, m, _start(ctx, m, b))  # warm-up outside capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        _iteration(ctx, m, cap)
    for k in range(1, 34):
        _iteration(ctx, m, eager)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for key in ("x", "r", "p", "rr"):
            assert torch.equal(cap[key].view(torch.int64), eager[key].view(torch.int64)), (k, key)
        if k in (1, 2, 5, 16, 17, 33):
            xo, it, _ = cg.cg(b, m, SHIFT, tol=1e-30, max_iter=k)
            assert it == k
            xg = to_host(cap["x"])
            assert np.linalg.norm(xg - xo) <= 1e-13 * np.linalg.norm(xo), k
    # the recursive residual norm after 33 iterations is the true one, up to rounding
    r_true = b - cg.stencil7(to_host(cap["x"]), m, SHIFT)
    assert rel_err(to_host(cap["rr"])[0], float(np.dot(r_true, r_true))) <= 1e-6
    assert math.isfinite(to_host(cap["rr"])[0])
