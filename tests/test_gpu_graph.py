"""The operations capture into a HIP graph and replay to the eager bits.

Every operation launches only kernels on the caller's stream (no allocation,
synchronisation, memset or read-back), so a whole CG-style step can be
captured.  The graph is replayed several times with eager work and
synchronisations in between, and every replay is compared bit for bit with
the same step run eagerly.
"""

import numpy as np
import pytest
import torch

import bsgen
from oracle import mesh

pytestmark = pytest.mark.gpu

import paper_2009_10917_amd as bs  # noqa: E402


def test_captured_step_replays_match_eager(ctx):
    K, N = 10, 5
    E, NL, NG = mesh.sizes(K, N)
    perm, orient = bsgen.permutation(3, E), bsgen.orientations(3, E)
    d_map = torch.from_numpy(mesh.hex_map(K, N, perm, orient).astype(np.int32)).cuda()
    plan = bs.bs_gs_create(ctx, d_map, NG)
    w = torch.empty(NL, dtype=torch.float64, device="cuda")
    bs.bs_gs_weights(plan, w)

    def fresh():
        v = {}
        for k, s in (("xG", 12), ("p", 3), ("r", 4), ("x", 1)):
            t = torch.empty(NG if k == "xG" else NL, dtype=torch.float64, device="cuda")
            bsgen.device_uniform(t, 9, s)
            v[k] = t
        v["pL"] = torch.empty(NL, dtype=torch.float64, device="cuda")
        v["Ap"] = torch.empty(NG, dtype=torch.float64, device="cuda")
        v["ApL"] = torch.empty(NL, dtype=torch.float64, device="cuda")
        v["out"] = torch.zeros(4, dtype=torch.float64, device="cuda")
        return v

    def step(v):
        # one CG-like pass of streaming operations on local vectors
        bs.bs_gs_scatter(ctx, plan, v["xG"], v["pL"])
        bs.bs_gather(ctx, plan, v["pL"], v["Ap"])
        bs.bs_gs_scatter(ctx, plan, v["Ap"], v["ApL"])
        bs.bs_dot(ctx, v["pL"], v["ApL"], v["out"][0:1])
        bs.bs_cg_update(ctx, 0.01, v["x"], v["pL"], v["r"], v["ApL"], w, v["out"][1:2])
        bs.bs_axpy(ctx, 1.0, v["r"], 0.5, v["p"])
        bs.bs_norm(ctx, v["p"], w, v["out"][2:3])
        bs.bs_copy(ctx, v["p"], v["pL"])

    eager = fresh()
    step(eager)
    torch.cuda.synchronize()

    cap = fresh()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step(fresh())  # warm-up outside capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        step(cap)
    for rep in range(3):
        # reset the captured buffers eagerly, then replay
        ref = fresh()
        for k in cap:
            cap[k].copy_(ref[k])
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in ("pL", "Ap", "ApL", "x", "r", "p", "out"):
            assert torch.equal(cap[k].view(torch.int64), eager[k].view(torch.int64)), (rep, k)
