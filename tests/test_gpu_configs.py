"""GPU parity on the benchmark configurations.

* K=8, N=3 lexicographic mesh (32,768 local, 15,625 global nodes): all seven
  operations on global and on local vectors, in full.
* K=48, N=7 permuted and oriented mesh (56.6M local, 38.3M global nodes):
  map, CSR, gather and scatter in full.
* N = 1..15 at about 5e7 local nodes: map, degrees, gather and scatter on
  samples the oracle computes one row at a time, plus gather(scatter(f)) =
  deg * f over the whole mesh.
* The benchmark's size (n = 721,734,273; N=7, K=128 mesh), in the launch
  configuration bench.py times: vectors on sampled indices, reductions on
  full-length vectors whose support is a sample, gather and scatter on
  sampled slots.
"""

import numpy as np
import pytest
import torch

import bsgen
from mesh_sample import MeshSample, seeded_mesh
from oracle import mesh, ops

pytestmark = pytest.mark.gpu

import paper_2009_10917_amd as bs  # noqa: E402
from gpu_util import bits, dev_uniform, rel_err, scalar_out, to_host  # noqa: E402

TOL = 1e-14
SEED = bsgen.DEFAULT_SEED


def device_mesh(ctx, K, N, perm, orient):
    E, NL, NG = mesh.sizes(K, N)
    d_map = torch.empty(NL, dtype=torch.int32, device="cuda")
    dp = None if perm is None else torch.from_numpy(np.asarray(perm, dtype=np.int32)).cuda()
    do = None if orient is None else torch.from_numpy(np.asarray(orient, dtype=np.uint8)).cuda()
    bs.bs_mesh_hex_map(K, N, dp, do, d_map)
    return d_map, bs.bs_gs_create(ctx, d_map, NG)


def at(t, idx):
    """Entries of a device tensor at host indices."""
    return t[torch.from_numpy(np.asarray(idx, dtype=np.int64)).cuda()].cpu().numpy()


# ---------------------------------------------------------------- K=8, N=3: everything

def test_small_mesh_all_seven_ops(ctx):
    K, N = 8, 3
    E, NL, NG = mesh.sizes(K, N)
    d_map, plan = device_mesh(ctx, K, N, None, None)
    ids = mesh.hex_map(K, N)
    assert np.array_equal(to_host(d_map), ids)
    rs, ci = mesh.csr_inverse(ids, NG)
    w = mesh.weights(ids, NG)
    d_w = torch.empty(NL, dtype=torch.float64, device="cuda")
    bs.bs_gs_weights(plan, d_w)
    assert np.array_equal(bits(to_host(d_w)), bits(w))
    alpha, beta = 0.37, 1.0
    for n, weights in ((NG, None), (NL, w)):
        h = {k: bsgen.uniform(SEED, s, n) for k, s in (("x", 1), ("y", 2), ("p", 3), ("r", 4), ("Ap", 5))}
        d = {k: torch.from_numpy(v).cuda() for k, v in h.items()}
        dw = None if weights is None else d_w
        y2 = torch.empty_like(d["x"])
        bs.bs_copy(ctx, d["x"], y2)
        assert np.array_equal(bits(to_host(y2)), bits(h["x"]))
        o = scalar_out()
        bs.bs_norm(ctx, d["x"], dw, o)
        assert rel_err(float(to_host(o)[0]), ops.norm(h["x"], weights)) <= TOL
        bs.bs_dot(ctx, d["x"], d["y"], o)
        assert rel_err(float(to_host(o)[0]), ops.dot(h["x"], h["y"])) <= TOL
        bs.bs_axpy(ctx, alpha, d["x"], beta, d["y"])
        assert np.array_equal(bits(to_host(d["y"])), bits(ops.axpy(alpha, h["x"], beta, h["y"])))
        bs.bs_cg_update(ctx, alpha, d["x"], d["p"], d["r"], d["Ap"], dw, o)
        xr, rr, rho = ops.cg_update(alpha, h["x"], h["p"], h["r"], h["Ap"], weights)
        assert np.array_equal(bits(to_host(d["x"])), bits(xr)) and np.array_equal(bits(to_host(d["r"])), bits(rr))
        assert rel_err(float(to_host(o)[0]), rho) <= TOL
    # the weighted norm of ones is the global node count, exactly
    o = scalar_out()
    bs.bs_norm(ctx, torch.ones(NL, dtype=torch.float64, device="cuda"), d_w, o)
    assert float(to_host(o)[0]) == float(NG)
    xG = bsgen.uniform(SEED, 12, NG)
    xL = torch.empty(NL, dtype=torch.float64, device="cuda")
    bs.bs_gs_scatter(ctx, plan, torch.from_numpy(xG).cuda(), xL)
    assert np.array_equal(bits(to_host(xL)), bits(ops.scatter(ids, xG, np.zeros(NL))))
    # local weighted norm of a scattered field equals its global norm
    bs.bs_norm(ctx, xL, d_w, o)
    assert rel_err(float(to_host(o)[0]), ops.norm(xG)) <= TOL
    g = torch.empty(NG, dtype=torch.float64, device="cuda")
    xLh = bsgen.uniform(SEED, 11, NL)
    bs.bs_gather(ctx, plan, torch.from_numpy(xLh).cuda(), g)
    assert np.array_equal(bits(to_host(g)), bits(ops.gather(rs, ci, xLh)))


# ---------------------------------------------------------------- K=48, N=7 in full

def test_k48_n7_permuted_oriented_in_full(ctx):
    K, N = 48, 7
    E, NL, NG = mesh.sizes(K, N)
    assert (NL, NG) == (56_623_104, 38_272_753)
    perm, orient = seeded_mesh(K, N, SEED)
    d_map, plan = device_mesh(ctx, K, N, perm, orient)
    ids = mesh.hex_map(K, N, perm, orient)
    assert np.array_equal(to_host(d_map).astype(np.int64), ids)
    del d_map
    rs, ci = mesh.csr_inverse(ids, NG)
    d_rs = torch.empty(NG + 1, dtype=torch.int32, device="cuda")
    d_ci = torch.empty(NL, dtype=torch.int32, device="cuda")
    bs.bs_gs_csr(plan, d_rs, d_ci)
    assert np.array_equal(to_host(d_rs), rs) and np.array_equal(to_host(d_ci), ci)
    del d_rs, d_ci
    xLh = bsgen.uniform(SEED, 11, NL)
    xG = torch.empty(NG, dtype=torch.float64, device="cuda")
    bs.bs_gather(ctx, plan, dev_uniform(NL, 11), xG)
    assert np.array_equal(bits(to_host(xG)), bits(ops.gather(rs, ci, xLh)))
    xGh = bsgen.uniform(SEED, 12, NG)
    xL = dev_uniform(NL, 11)
    bs.bs_gs_scatter(ctx, plan, dev_uniform(NG, 12), xL)
    assert np.array_equal(bits(to_host(xL)), bits(ops.scatter(ids, xGh, xLh)))


# ---------------------------------------------------------------- N = 1..15 at ~5e7 local nodes

N_SWEEP = [(1, 184), (2, 123), (3, 92), (4, 74), (5, 61), (6, 53), (7, 46), (8, 41), (9, 37), (10, 33),
           (11, 31), (12, 28), (13, 26), (14, 25), (15, 23)]


@pytest.mark.parametrize("N,K", N_SWEEP)
def test_degree_sweep_sampled(ctx, N, K):
    E, NL, NG = mesh.sizes(K, N)
    perm, orient = seeded_mesh(K, N, SEED + N)
    d_map, plan = device_mesh(ctx, K, N, perm, orient)
    ms = MeshSample(K, N, perm, orient, n_slots=48, seed=N)
    l, g = ms.sampled_locals()
    assert np.array_equal(at(d_map, l).astype(np.int64), g)
    del d_map
    # degrees: closed-form histogram over the whole mesh, exact per sampled row
    deg = torch.empty(NG, dtype=torch.int32, device="cuda")
    bs.bs_gs_degree(plan, deg)
    a, b = K - 1, K * (N - 1) + 2
    hist = torch.bincount(deg.long(), minlength=9).cpu().numpy()
    assert (hist[1], hist[2], hist[4], hist[8]) == (b ** 3, 3 * a * b * b, 3 * a * a * b, a ** 3)
    assert np.array_equal(at(deg, ms.g), ms.degrees())
    # gather on sampled rows, bit for bit
    xL = dev_uniform(NL, 11)
    xG = torch.empty(NG, dtype=torch.float64, device="cuda")
    bs.bs_gather(ctx, plan, xL, xG)
    ref = ms.gather_rows(lambda idx: bsgen.uniform_at(SEED, 11, idx))
    assert np.array_equal(bits(at(xG, ms.g)), bits(ref))
    # scatter on sampled slots, bit for bit
    bs.bs_gs_scatter(ctx, plan, dev_uniform(NG, 12), xL)
    assert np.array_equal(bits(at(xL, l)), bits(bsgen.uniform_at(SEED, 12, g)))
    # gather(scatter(f)) = deg * f over the whole mesh, for dyadic f
    f = (torch.arange(NG, device="cuda", dtype=torch.float64) % 97) * 0.125 - 6.0
    bs.bs_gs_scatter(ctx, plan, f, xL)
    bs.bs_gather(ctx, plan, xL, xG)
    assert torch.equal(xG, f * deg.double())


# ---------------------------------------------------------------- the benchmark's size

N_BIG = (7 * 128 + 1) ** 3


def sample_indices(n, rng, k=1 << 20):
    edge = np.concatenate([np.arange(4096), np.arange(n - 4096, n)])
    mid = np.concatenate([np.arange(m - 8, m + 8) for m in range(1 << 22, n - 8, 1 << 26)])
    return np.unique(np.concatenate([edge, mid, rng.integers(0, n, k)]))


def sparse(n, idx, vals):
    t = torch.zeros(n, dtype=torch.float64, device="cuda")
    t[torch.from_numpy(idx).cuda()] = torch.from_numpy(vals).cuda()
    return t


@pytest.mark.slow
def test_benchmark_size_vectors_and_reductions(ctx):
    n = N_BIG
    rng = np.random.default_rng(5)
    idx = sample_indices(n, rng)
    S = bsgen.STREAM
    h = {k: bsgen.uniform_at(SEED, S[k], idx) for k in ("x", "y", "p", "r", "Ap")}
    hw = bsgen.uniform_at(SEED, S["w"], idx, lo=0.0)
    alpha, beta = (float(v) for v in bsgen.scalars(SEED, 128))
    x = dev_uniform(n, S["x"])
    y = dev_uniform(n, S["y"])
    w = dev_uniform(n, S["w"], lo=0.0)
    # BS1, BS2 on sampled indices
    z = torch.empty_like(x)
    bs.bs_copy(ctx, x, z)
    assert np.array_equal(bits(at(z, idx)), bits(h["x"]))
    bs.bs_axpy(ctx, alpha, x, beta, y)
    assert np.array_equal(bits(at(y, idx)), bits(ops.axpy(alpha, h["x"], beta, h["y"])))
    # BS3, BS4 over full-length vectors whose support is the sample
    xs = sparse(n, idx, h["x"])
    o = scalar_out()
    bs.bs_norm(ctx, xs, None, o)
    assert rel_err(float(to_host(o)[0]), ops.norm(h["x"])) <= TOL
    bs.bs_norm(ctx, xs, w, o)
    assert rel_err(float(to_host(o)[0]), ops.norm(h["x"], hw)) <= TOL
    yh = ops.axpy(alpha, h["x"], beta, h["y"])
    bs.bs_dot(ctx, xs, y, o)
    assert rel_err(float(to_host(o)[0]), ops.dot(h["x"], yh)) <= TOL
    # full random data: dot(x, x) equals norm(x); constant vector closed form
    a, b2 = scalar_out(), scalar_out()
    bs.bs_dot(ctx, x, x, a)
    bs.bs_norm(ctx, x, None, b2)
    assert rel_err(float(to_host(a)[0]), float(to_host(b2)[0])) <= TOL
    z.fill_(0.5)
    bs.bs_norm(ctx, z, None, o)
    assert float(to_host(o)[0]) == n * 0.25
    # one-pass reduction grids at this length (1,409,638 workgroups; 345 chunk sums in the second stage)
    own = bs.bs_ctx_create(0)
    try:
        for op in ("norm", "dot"):
            bs.bs_ctx_set_tune(own, op, 1, 1 << 30)
        a2 = scalar_out()
        bs.bs_dot(own, x, x, a2)
        assert rel_err(float(to_host(a2)[0]), float(to_host(b2)[0])) <= TOL
        bs.bs_norm(own, z, None, a2)
        assert float(to_host(a2)[0]) == n * 0.25
    finally:
        torch.cuda.synchronize()
        own.close()
    del z, y, xs
    # BS5: x, p dense; r, Ap supported on the sample so that r'.r' is exact
    p = dev_uniform(n, S["p"])
    r = sparse(n, idx, h["r"])
    Ap = sparse(n, idx, h["Ap"])
    bs.bs_cg_update(ctx, alpha, x, p, r, Ap, w, o)
    xr, rr, rho = ops.cg_update(alpha, h["x"], h["p"], h["r"], h["Ap"], hw)
    assert np.array_equal(bits(at(x, idx)), bits(xr))
    assert np.array_equal(bits(at(r, idx)), bits(rr))
    assert rel_err(float(to_host(o)[0]), rho) <= TOL
    off = np.setdiff1d(rng.integers(0, n, 4096), idx)
    assert np.all(at(r, off) == 0.0)


@pytest.mark.slow
def test_benchmark_size_gather_scatter(ctx):
    K, N = 128, 7
    E, NL, NG = mesh.sizes(K, N)
    assert NG == N_BIG and NL == 1 << 30
    perm, orient = seeded_mesh(K, N, SEED)
    d_map, plan = device_mesh(ctx, K, N, perm, orient)
    ms = MeshSample(K, N, perm, orient, n_slots=32, seed=11)
    l, g = ms.sampled_locals()
    assert np.array_equal(at(d_map, l).astype(np.int64), g)
    del d_map
    xL = dev_uniform(NL, 11)
    xG = torch.empty(NG, dtype=torch.float64, device="cuda")
    bs.bs_gather(ctx, plan, xL, xG)
    ref = ms.gather_rows(lambda i: bsgen.uniform_at(SEED, 11, i))
    assert np.array_equal(bits(at(xG, ms.g)), bits(ref))
    # the benchmark's gather: lattice-tiled rows in its tiles and boxes, its variant
    from bench import GATHER_BOX, GATHER_TILE, GATHER_VARIANT
    M = K * N + 1
    bs.bs_gs_order_rows(plan, M, M, M, GATHER_TILE, GATHER_BOX)
    own = bs.bs_ctx_create(0)  # its own context: one launch shape for every length
    bs.bs_ctx_set_tune(own, "gather", 1, 1 << 30, GATHER_VARIANT)
    xG.fill_(float("nan"))
    bs.bs_gather(own, plan, xL, xG)
    torch.cuda.synchronize()
    own.close()
    assert np.array_equal(bits(at(xG, ms.g)), bits(ref))
    assert not torch.isnan(xG).any()
    bs.bs_gs_scatter(ctx, plan, dev_uniform(NG, 12), xL)
    assert np.array_equal(bits(at(xL, l)), bits(bsgen.uniform_at(SEED, 12, g)))
