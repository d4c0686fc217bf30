"""GPU parity of the batched step (many box-mesh instances in one batch).

The three forms (per-instance launches, per-phase launches, one persistent
launch that claims work items in dependency order) run the same code on the
same chunks and must agree bit for bit; the persistent form's waits must
never have run into their time limit.  Against the oracle's step, instance by instance: vectors that do
not depend on a reduction (y, xL, pL, Ap, and x after step 5) are bit-exact
in binary64; reductions are within 1e-14 relative of the exact sums; x, r
and p after the CG iteration carry the rounding of a = rr/pAp and
b = rr2/rr and are compared within 1e-13 relative of their terms.
"""

import numpy as np
import pytest
import torch

import bsgen
from oracle import batch as obatch
from oracle import mesh

pytestmark = pytest.mark.gpu

import paper_2009_10917_amd as bs  # noqa: E402
from gpu_util import to_host  # noqa: E402

SEED = 10917
ALPHA, BETA = 0.37, 0.61
STREAMS = {"x": 1, "y": 2, "p": 3, "r": 4, "Ap": 5, "xL": 11, "pL": 12, "wL": 6}


def small_instances(n, cap):
    E, N = bsgen.batch_instances(SEED, n)
    return np.minimum(E, cap), N


def build(ctx, E, N):
    maps, nl, ng = [], [], []
    for e, d in zip(E, N):
        m, g = bs.bs_mesh_box_map_host(int(e), int(d))
        maps.append(m)
        nl.append(m.size)
        ng.append(g)
    d_map = torch.from_numpy(np.concatenate(maps)).cuda()
    return bs.bs_batch_create(ctx, nl, ng, d_map), maps, ng


def inputs(b, dtype=torch.float64):
    v = {}
    for k, sid in STREAMS.items():
        n = b.n_global if k in bs.BATCH_GLOBAL else b.n_local
        t = torch.empty(n, dtype=dtype, device="cuda")
        bsgen.device_uniform(t, SEED, sid, lo=0.0 if k == "wL" else -1.0)
        v[k] = t
    return v


def run(ctx, b, v0, mode):
    v = {k: t.clone() for k, t in v0.items()}
    out = torch.zeros(8 * b.n_inst, dtype=torch.float64, device="cuda")
    bs.bs_batch_step(ctx, b, v, ALPHA, BETA, out, mode)
    torch.cuda.synchronize()
    return v, out


@pytest.fixture(scope="module")
def small(ctx):
    E, N = small_instances(24, 150)
    b, maps, ng = build(ctx, E, N)
    return b, maps, ng


def bits(t):
    return t.view(torch.int64 if t.dtype == torch.float64 else torch.int32).cpu()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_forms_agree_bit_for_bit(ctx, small, dtype):
    b = small[0]
    v0 = inputs(b, dtype)
    res = [run(ctx, b, v0, m) for m in (0, 1, 2)]
    for v, out in res[1:]:
        assert torch.equal(out.view(torch.int64), res[0][1].view(torch.int64))
        for k in v:
            assert torch.equal(bits(v[k]), bits(res[0][0][k])), k
    assert bs.bs_batch_barrier_timeouts(b) == 0


def test_persistent_form_repeats(ctx, small):
    # the schedule resets itself at the end of each launch
    b = small[0]
    v0 = inputs(b)
    ref, out_ref = run(ctx, b, v0, bs.BS_BATCH_PER_PHASE)
    for _ in range(3):
        v, out = run(ctx, b, v0, bs.BS_BATCH_PERSISTENT)
        assert torch.equal(out.view(torch.int64), out_ref.view(torch.int64))
        assert torch.equal(bits(v["p"]), bits(ref["p"]))
    assert bs.bs_batch_barrier_timeouts(b) == 0


@pytest.mark.parametrize("claim,cap", [(1, 1 << 30), (2, 7), (4, 64), (8, 1)])
def test_persistent_claim_sizes(ctx, small, claim, cap):
    # the tune entry of op "batch" sets the items per claim and caps the workgroups;
    # the schedule finishes with any of them and gives the per-phase bits
    b = small[0]
    v0 = inputs(b)
    ref, out_ref = run(ctx, b, v0, bs.BS_BATCH_PER_PHASE)
    own = bs.bs_ctx_create(torch.cuda.current_device())
    try:
        bs.bs_ctx_set_tune(own, "batch", claim, cap, 0)
        for _ in range(2):
            v, out = run(own, b, v0, bs.BS_BATCH_PERSISTENT)
            assert torch.equal(out.view(torch.int64), out_ref.view(torch.int64))
            for k in v:
                assert torch.equal(bits(v[k]), bits(ref[k])), k
    finally:
        torch.cuda.synchronize()
        own.close()
    assert bs.bs_batch_barrier_timeouts(b) == 0


def test_binary64_matches_oracle(ctx, small):
    b, maps, ng = small
    v0 = inputs(b)
    v, out = run(ctx, b, v0, bs.BS_BATCH_PERSISTENT)
    h0 = {k: to_host(t) for k, t in v0.items()}
    hv = {k: to_host(t) for k, t in v.items()}
    ho = to_host(out).reshape(-1, 8)
    for i in range(b.n_inst):
        gs = slice(b.off_global[i], b.off_global[i + 1])
        ls = slice(b.off_local[i], b.off_local[i + 1])
        vi = {k: h0[k][gs if k in bs.BATCH_GLOBAL else ls] for k in h0}
        ref, sc = obatch.step(maps[i].astype(np.int64), ng[i], vi, ALPHA, BETA)
        got = {k: hv[k][gs if k in bs.BATCH_GLOBAL else ls] for k in hv}
        for k in ("y", "xL", "pL", "Ap", "wL"):
            assert np.array_equal(got[k].view(np.int64), ref[k].view(np.int64)), (i, k)
        for j, name in enumerate(bs.BATCH_SLOTS):
            tol = 1e-14 if name in ("norm", "dot", "rr", "pAp") else 1e-12
            assert abs(ho[i, j] - sc[name]) <= tol * abs(sc[name]), (i, name)
        a = sc["alpha"]
        x5 = vi["x"] + ALPHA * vi["p"]
        r5 = vi["r"] - ALPHA * vi["Ap"]
        assert np.all(np.abs(got["x"] - ref["x"]) <= 1e-13 * (np.abs(x5) + np.abs(a * vi["p"])) + 1e-300), i
        assert np.all(np.abs(got["r"] - ref["r"]) <= 1e-13 * (np.abs(r5) + np.abs(a * ref["Ap"])) + 1e-300), i
        assert np.all(np.abs(got["p"] - ref["p"]) <= 1e-13 * (np.abs(ref["r"]) + np.abs(sc["beta"] * vi["p"])) + 1e-300), i


def test_binary32_within_bounds(ctx, small):
    b, maps, ng = small
    v0 = inputs(b, torch.float32)
    v, out = run(ctx, b, v0, bs.BS_BATCH_PER_PHASE)
    h0 = {k: t.double().cpu().numpy() for k, t in v0.items()}
    ho = to_host(out).reshape(-1, 8)
    hv = {k: t.double().cpu().numpy() for k, t in v.items()}
    for i in range(0, b.n_inst, 3):
        gs = slice(b.off_global[i], b.off_global[i + 1])
        ls = slice(b.off_local[i], b.off_local[i + 1])
        vi = {k: h0[k][gs if k in bs.BATCH_GLOBAL else ls] for k in h0}
        ref, sc = obatch.step(maps[i].astype(np.int64), ng[i], vi, ALPHA, BETA)
        # scatter copies exactly; the norm's terms take two binary32 roundings
        # (3 u32 with the compensated sum); p.Ap's terms deg p^2 also carry
        # the up to 7 roundings of a gathered row of degree <= 8 (10 u32)
        assert np.array_equal(hv["pL"][ls], ref["pL"]), i
        for name, bound in (("norm", 3), ("pAp", 10)):
            j = bs.BATCH_SLOTS.index(name)
            assert abs(ho[i, j] - sc[name]) <= bound * 2.0 ** -24 * abs(sc[name]), (i, name)


@pytest.mark.parametrize("mode", [bs.BS_BATCH_PER_PHASE, bs.BS_BATCH_PERSISTENT])
def test_graph_replays_match_eager(ctx, small, mode):
    b = small[0]
    v0 = inputs(b)
    eager, out_e = run(ctx, b, v0, mode)
    v = {k: t.clone() for k, t in v0.items()}
    out = torch.zeros(8 * b.n_inst, dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        bs.bs_batch_step(ctx, b, v, ALPHA, BETA, out, mode, stream=s.cuda_stream)  # warm-up outside capture
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        bs.bs_batch_step(ctx, b, v, ALPHA, BETA, out, mode)
    for rep in range(3):
        for k in v:
            v[k].copy_(v0[k])
        out.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out.view(torch.int64), out_e.view(torch.int64)), rep
        for k in v:
            assert torch.equal(bits(v[k]), bits(eager[k])), (rep, k)
        _ = torch.ones(1000, device="cuda").sum()  # eager work between replays
    assert bs.bs_batch_barrier_timeouts(b) == 0


def test_full_descriptor_set_builds_and_runs(ctx):
    # the real 1024 instances, checked on sampled instances against the oracle
    E, N = bsgen.batch_instances(SEED, 1024)
    b, maps, ng = build(ctx, E, N)
    assert 1.2e8 < b.n_local < 1.7e8
    v0 = inputs(b)
    v, out = run(ctx, b, v0, bs.BS_BATCH_PERSISTENT)
    v1, out1 = run(ctx, b, v0, bs.BS_BATCH_PER_PHASE)
    assert torch.equal(out.view(torch.int64), out1.view(torch.int64))
    assert bs.bs_batch_barrier_timeouts(b) == 0
    ho = to_host(out).reshape(-1, 8)
    for i in (0, 511, 1023, int(np.argmax(E * (N + 1) ** 3))):
        gs = slice(b.off_global[i], b.off_global[i + 1])
        ls = slice(b.off_local[i], b.off_local[i + 1])
        vi = {k: to_host(v0[k][gs if k in bs.BATCH_GLOBAL else ls]) for k in v0}
        ref, sc = obatch.step(maps[i].astype(np.int64), ng[i], vi, ALPHA, BETA)
        assert np.array_equal(to_host(v["Ap"][gs]).view(np.int64), ref["Ap"].view(np.int64)), i
        for j, name in enumerate(bs.BATCH_SLOTS[:4]):
            assert abs(ho[i, j] - sc[name]) <= 1e-14 * abs(sc[name]), (i, name)
    b.close()


def test_batch_argument_errors(ctx, small):
    b = small[0]
    v = inputs(b)
    out = torch.zeros(8 * b.n_inst, dtype=torch.float64, device="cuda")
    with pytest.raises(bs.BSError):
        bs.bs_batch_step(ctx, b, v, ALPHA, BETA, out, mode=7)
    bad = torch.tensor([0, 1, 99], dtype=torch.int32, device="cuda")
    with pytest.raises(bs.BSError):
        bs.bs_batch_create(ctx, [3], [3], bad)
