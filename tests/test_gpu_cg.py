"""GPU parity of the 7-point operator and of the CG solvers.

The operator is compared bit for bit with the oracle in every storage type:
the order of the additions is fixed, binary32 storage computes in binary32,
bfloat16 storage computes in binary32 and rounds the result once.  Solvers are
compared by what is unique about their result: the true relative residual,
recomputed by the oracle from the GPU's x, and the solution itself within
kappa times the tolerance.  Iteration counts of the binary64 CG must match
the oracle's Algorithm 1 to within a few iterations (the reductions add in a
different order).
"""

import math

import numpy as np
import pytest
import torch

import bsgen
from oracle import cg

pytestmark = pytest.mark.gpu

import paper_2009_10917_amd as bs  # noqa: E402
from gpu_util import bits, to_host  # noqa: E402

SHIFT = 0.01


def rhs(m, seed=10917):
    return bsgen.uniform(seed, bsgen.STREAM["b"], m ** 3)


def true_relres(x, b, m):
    r = b - cg.stencil7(x, m, SHIFT)
    return math.sqrt(float(np.dot(r, r)) / float(np.dot(b, b)))


@pytest.mark.parametrize("m", [1, 2, 3, 7, 64, 65, 130])
def test_stencil_binary64_bit_exact(ctx, m):
    x = bsgen.uniform(3, 1, m ** 3)
    y = torch.empty(m ** 3, dtype=torch.float64, device="cuda")
    bs.bs_stencil7(ctx, m, SHIFT, torch.from_numpy(x).cuda(), y)
    assert np.array_equal(bits(to_host(y)), bits(cg.stencil7(x, m, SHIFT)))


@pytest.mark.parametrize("m", [1, 5, 64, 67])
def test_stencil_binary32_bit_exact(ctx, m):
    # binary32 storage and arithmetic: the same rounded operations in the same order
    x = torch.empty(m ** 3, dtype=torch.float32, device="cuda")
    bsgen.device_uniform(x, 3, 1)
    y = torch.empty_like(x)
    bs.bs_stencil7(ctx, m, SHIFT, x, y)
    torch.cuda.synchronize()
    ref = cg.stencil7(x.cpu().numpy(), m, SHIFT, dtype=np.float32)
    assert np.array_equal(y.cpu().numpy().view(np.uint32), ref.view(np.uint32))


@pytest.mark.parametrize("m", [1, 5, 64, 67])
def test_stencil_bfloat16_bit_exact(ctx, m):
    # bfloat16 storage, binary32 arithmetic, one rounding of the result to bfloat16
    x = torch.empty(m ** 3, dtype=torch.bfloat16, device="cuda")
    bsgen.device_uniform(x, 3, 1)
    y = torch.empty_like(x)
    bs.bs_stencil7(ctx, m, SHIFT, x, y)
    torch.cuda.synchronize()
    xs = bsgen.bf16_bits_to_f64(x.view(torch.int16).cpu().numpy().view(np.uint16)).astype(np.float32)
    ref = bsgen.round_bf16_bits(cg.stencil7(xs, m, SHIFT, dtype=np.float32).astype(np.float64))
    assert np.array_equal(y.view(torch.int16).cpu().numpy().view(np.uint16), ref)


@pytest.mark.parametrize("m", [16, 33, 64])
def test_cg_binary64_matches_algorithm_1(ctx, m):
    b = rhs(m)
    x = torch.zeros(m ** 3, dtype=torch.float64, device="cuda")
    res = bs.bs_cg_solve(ctx, m, SHIFT, torch.from_numpy(b).cuda(), x, tol=1e-10)
    xo, it, _ = cg.cg(b, m, SHIFT, tol=1e-10)
    xg = to_host(x)
    assert res["rel_residual"] <= 1e-10 and true_relres(xg, b, m) <= 1e-10
    assert abs(res["iterations"] - it) <= 3
    assert np.linalg.norm(xg - xo) <= 1e-8 * np.linalg.norm(xo)


@pytest.mark.parametrize("k", [1, 2, 5, 16, 17, 33])
def test_cg_iterate_after_k_steps(ctx, k):
    # stops inside and across the batches of captured iterations, on both
    # parities of the alternating direction buffers
    m = 21
    b = rhs(m, seed=5)
    x = torch.zeros(m ** 3, dtype=torch.float64, device="cuda")
    res = bs.bs_cg_solve(ctx, m, SHIFT, torch.from_numpy(b).cuda(), x, tol=1e-30, max_iter=k, check=False)
    assert res["status"] == "BS_ERR_NO_CONVERGENCE" and res["iterations"] == k and res["restarts"] == 0
    xo, it, rel = cg.cg(b, m, SHIFT, tol=1e-30, max_iter=k)
    assert it == k
    assert np.linalg.norm(to_host(x) - xo) <= 1e-13 * np.linalg.norm(xo)
    assert abs(res["rel_residual"] - rel) <= 1e-9 * rel


def test_cg_eigenvector_one_iteration(ctx):
    m = 17
    v = cg.sine_mode(m, 2, 3, 5)
    lam = cg.eigenvalue(m, SHIFT, 2, 3, 5)
    x = torch.zeros(m ** 3, dtype=torch.float64, device="cuda")
    res = bs.bs_cg_solve(ctx, m, SHIFT, torch.from_numpy(v).cuda(), x, tol=1e-12)
    assert res["iterations"] == 1
    assert np.allclose(to_host(x), v / lam, rtol=0, atol=1e-13)


def test_cg_warm_start_and_zero_rhs(ctx):
    m = 20
    b = rhs(m)
    xo, _, _ = cg.cg(b, m, SHIFT, tol=1e-13)
    x = torch.from_numpy(xo.copy()).cuda()
    res = bs.bs_cg_solve(ctx, m, SHIFT, torch.from_numpy(b).cuda(), x, tol=1e-10)
    assert res["iterations"] == 0 and res["rel_residual"] <= 1e-10
    with pytest.raises(bs.BSError) as e:
        bs.bs_cg_solve(ctx, m, SHIFT, torch.from_numpy(b).cuda(), torch.zeros_like(x), tol=1e-10, max_iter=5)
    assert e.value.status == 5  # no convergence in 5 iterations


@pytest.mark.parametrize("m", [24, 64])
def test_ir_cg_binary32_reaches_binary64_accuracy(ctx, m):
    b = rhs(m)
    x = torch.zeros(m ** 3, dtype=torch.float64, device="cuda")
    res = bs.bs_cg_ir_solve(ctx, bs.BS_F32, m, SHIFT, torch.from_numpy(b).cuda(), x, tol=1e-10, inner_tol=1e-4)
    xg = to_host(x)
    assert res["rel_residual"] <= 1e-10 and true_relres(xg, b, m) <= 1e-10
    assert 2 <= res["outer_iterations"] <= 6
    xo, _, _ = cg.cg(b, m, SHIFT, tol=1e-12)
    kappa = cg.eigenvalue(m, SHIFT, m, m, m) / cg.eigenvalue(m, SHIFT, 1, 1, 1)
    assert np.linalg.norm(xg - xo) <= kappa * 1e-10 * np.linalg.norm(xo)


@pytest.mark.parametrize("inner_tol", [0.1, 3e-3])
def test_ir_cg_bfloat16_reports_its_outcome(ctx, inner_tol):
    # bfloat16 storage: kappa * 2^-8 is above 1 on this grid, so inner solves may
    # fail to contract; the solver must then say so instead of looping
    m = 64
    b = rhs(m)
    x = torch.zeros(m ** 3, dtype=torch.float64, device="cuda")
    res = bs.bs_cg_ir_solve(ctx, bs.BS_BF16, m, SHIFT, torch.from_numpy(b).cuda(), x, tol=1e-10,
                            inner_tol=inner_tol, max_outer=60, check=False)
    rr = true_relres(to_host(x), b, m)
    assert abs(rr - res["rel_residual"]) <= 1e-6 * max(rr, 1e-12) + 1e-14
    if res["status"] == "BS_OK":
        assert rr <= 1e-10
    else:
        assert res["status"] == "BS_ERR_NO_CONVERGENCE" and np.isfinite(rr)


@pytest.mark.slow
def test_full_size_fp64_and_mixed(ctx):
    m = 225
    b = rhs(m)
    db = torch.from_numpy(b).cuda()
    x64 = torch.zeros(m ** 3, dtype=torch.float64, device="cuda")
    r64 = bs.bs_cg_solve(ctx, m, SHIFT, db, x64, tol=1e-10)
    x32 = torch.zeros_like(x64)
    r32 = bs.bs_cg_ir_solve(ctx, bs.BS_F32, m, SHIFT, db, x32, tol=1e-10, inner_tol=1e-4)
    x16 = torch.zeros_like(x64)
    r16 = bs.bs_cg_ir_solve(ctx, bs.BS_BF16, m, SHIFT, db, x16, tol=1e-10, inner_tol=0.1, max_outer=60)
    assert r16["status"] == "BS_OK"
    a, c, d = to_host(x64), to_host(x32), to_host(x16)
    # true residuals recomputed by the oracle's operator from the library's x
    assert true_relres(a, b, m) <= 1e-10 and true_relres(c, b, m) <= 1e-10 and true_relres(d, b, m) <= 1e-10
    kappa = cg.eigenvalue(m, SHIFT, m, m, m) / cg.eigenvalue(m, SHIFT, 1, 1, 1)
    assert np.linalg.norm(a - c) <= kappa * 2e-10 * np.linalg.norm(a)
    assert np.linalg.norm(a - d) <= kappa * 2e-10 * np.linalg.norm(a)
    assert r16["outer_iterations"] >= 2 and r32["outer_iterations"] >= 2
    # the benchmark's bfloat16 inner tolerance
    x16b = torch.zeros_like(x64)
    r16b = bs.bs_cg_ir_solve(ctx, bs.BS_BF16, m, SHIFT, db, x16b, tol=1e-10, inner_tol=3e-3, max_outer=60)
    assert r16b["status"] == "BS_OK"
    e = to_host(x16b)
    assert true_relres(e, b, m) <= 1e-10
    assert np.linalg.norm(a - e) <= kappa * 2e-10 * np.linalg.norm(a)
    # Chebyshev bound on the A-norm error, turned into one on the residual
    # (a factor sqrt(kappa) between the two): a ceiling, not an estimate
    ceiling = math.sqrt(kappa) / 2 * math.log(2 * math.sqrt(kappa) / 1e-10)
    assert 1 <= r64["iterations"] <= ceiling


def test_solver_argument_errors(ctx):
    L = bs.lib
    x = torch.zeros(27, dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    assert L.bs_cg_solve(ctx.handle, 0, SHIFT, x.data_ptr(), x.data_ptr(), 1e-10, 10, None, s) == 1
    assert L.bs_cg_solve(ctx.handle, 3, SHIFT, None, x.data_ptr(), 1e-10, 10, None, s) == 1
    assert L.bs_cg_solve(ctx.handle, 3, SHIFT, x.data_ptr(), x.data_ptr(), 0.0, 10, None, s) == 1
    assert L.bs_cg_ir_solve(ctx.handle, 1, 3, SHIFT, x.data_ptr(), x.data_ptr(), 1e-10, 1.5, 10, 10, None, s) == 1
    assert L.bs_cg_ir_solve(ctx.handle, 7, 3, SHIFT, x.data_ptr(), x.data_ptr(), 1e-10, 0.1, 10, 10, None, s) == 1
    assert L.bs_stencil7(ctx.handle, 0, 3, SHIFT, x.data_ptr(), x.data_ptr(), s) == 1  # y aliases x
