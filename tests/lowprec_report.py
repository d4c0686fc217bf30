"""Measured errors of the binary32 and bfloat16 paths against the binary64
oracle at n = 11,390,625 (the 225^3 grid of the mixed-precision
configuration), written as a markdown table.

    python tests/lowprec_report.py [out.md]     (on a GPU host)

For each operation and storage type the library runs on the stored
(rounded) inputs; the oracle runs in binary64 (exact sums for the
reductions) on (a) the same stored inputs and (b) the original binary64
draws.  Reported: the largest elementwise error divided by the largest
|reference| (vectors), or the relative error (reductions), and the ratio of
that error to the stated bound against (a).  The refinement solves are
compared with the binary64 CG by their true residuals, recomputed here in
binary64 from each x, and by the distance between solutions.

Test infrastructure: it calls the library through its binding and checks it
against the oracle; nothing in the library imports it.
"""

import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

import bsgen  # noqa: E402
import paper_2009_10917_amd as bs  # noqa: E402
from oracle import cg, mesh, ops  # noqa: E402

U32 = 2.0 ** -24
SEED = 10917
M, K, N = 225, 32, 7
ALPHA, BETA = 0.37, 1.0


def narrow(x, name):
    """binary64 draws -> the values the narrow storage holds (as binary64)."""
    if name == "f32":
        return bsgen.round_f32(x).astype(np.float64)
    return bsgen.bf16_bits_to_f64(bsgen.round_bf16_bits(x))


def to_dev(v, dt):
    if dt == torch.bfloat16:
        return torch.from_numpy(bsgen.round_bf16_bits(v).view(np.int16)).cuda().view(torch.bfloat16)
    return torch.from_numpy(v.astype(np.float32)).cuda()


def from_dev(t):
    torch.cuda.synchronize()
    if t.dtype == torch.bfloat16:
        return bsgen.bf16_bits_to_f64(t.view(torch.int16).cpu().numpy().view(np.uint16))
    return t.cpu().numpy().astype(np.float64)


def vec_err(got, ref):
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300))


def rel(got, ref):
    return abs(got - ref) / abs(ref) if ref else abs(got)


def main(out_path):
    ctx = bs.bs_ctx_create(0)
    n = M ** 3
    E = K ** 3
    S = bsgen.STREAM
    d64 = {k: bsgen.uniform(SEED, S[k], n, lo=0.0 if k == "w" else -1.0) for k in ("x", "y", "p", "r", "Ap", "w")}
    ids = mesh.hex_map(K, N, bsgen.permutation(SEED, E), bsgen.orientations(SEED, E))
    NL = ids.size
    rs, ci = mesh.csr_inverse(ids, n)
    deg = np.diff(rs)
    xL64 = bsgen.uniform(SEED, S["xL"], NL)
    plan = bs.bs_gs_create(ctx, torch.from_numpy(ids.astype(np.int32)).cuda(), n)
    rows = []
    for name, dt, us in (("f32", torch.float32, 0.0), ("bf16", torch.bfloat16, 2.0 ** -8)):
        t0 = time.time()
        st = {k: narrow(v, name) for k, v in d64.items()}
        xLs = narrow(xL64, name)
        dev = {k: to_dev(v, dt) for k, v in st.items()}
        out = torch.zeros(4, dtype=torch.float64, device="cuda")
        # BS1 copy
        y = torch.empty_like(dev["x"])
        bs.bs_copy(ctx, dev["x"], y)
        got = from_dev(y)
        rows.append((name, "copy", vec_err(got, st["x"]), vec_err(got, d64["x"]), 0.0, "bit-exact on stored bits"))
        # BS2 axpy
        y = dev["y"].clone()
        bs.bs_axpy(ctx, ALPHA, dev["x"], BETA, y)
        got = from_dev(y)
        ref_s = ops.axpy(ALPHA, st["x"], BETA, st["y"])
        ref_d = ops.axpy(ALPHA, d64["x"], BETA, d64["y"])
        bound = (us + 3 * U32) * (np.abs(ALPHA * st["x"]) + np.abs(BETA * st["y"]))
        ratio = float(np.max(np.abs(got - ref_s) / np.maximum(bound, 1e-300)))
        rows.append((name, "axpy", vec_err(got, ref_s), vec_err(got, ref_d), ratio, "(u_s + 3u32)(|a x| + |b y|)"))
        # BS3 weighted norm
        bs.bs_norm(ctx, dev["x"], dev["w"], out[0:1])
        g = float(from_dev(out)[0])
        ref_s, ref_d = ops.norm(st["x"], st["w"]), ops.norm(d64["x"], d64["w"])
        rows.append((name, "norm (weighted)", rel(g, ref_s), rel(g, ref_d), rel(g, ref_s) / (3 * U32), "3 u32 S"))
        # BS4 dot
        bs.bs_dot(ctx, dev["x"], dev["y"], out[1:2])
        g = float(from_dev(out)[1])
        ref_s, ref_d = ops.dot(st["x"], st["y"]), ops.dot(d64["x"], d64["y"])
        sabs = float(np.sum(np.abs(st["x"] * st["y"])))
        b = 2 * U32 * abs(ref_s) + 1e-12 * sabs
        rows.append((name, "dot", rel(g, ref_s), rel(g, ref_d), abs(g - ref_s) / b, "2 u32 |S| + 1e-12 sum|x y|"))
        # BS5 fused CG update (weighted)
        xv, rv = dev["x"].clone(), dev["r"].clone()
        a = 1e-3
        bs.bs_cg_update(ctx, a, xv, dev["p"], rv, dev["Ap"], dev["w"], out[2:3])
        gx, gr, g = from_dev(xv), from_dev(rv), float(from_dev(out)[2])
        xr, rr, rho = ops.cg_update(a, st["x"], st["p"], st["r"], st["Ap"], st["w"])
        xd, rd, rhod = ops.cg_update(a, d64["x"], d64["p"], d64["r"], d64["Ap"], d64["w"])
        bx = (us + 3 * U32) * (np.abs(st["x"]) + np.abs(a * st["p"]))
        br = (us + 3 * U32) * (np.abs(st["r"]) + np.abs(a * st["Ap"]))
        rows.append((name, "cg_update x", vec_err(gx, xr), vec_err(gx, xd),
                     float(np.max(np.abs(gx - xr) / np.maximum(bx, 1e-300))), "(u_s + 3u32)(|x| + |a p|)"))
        rows.append((name, "cg_update r", vec_err(gr, rr), vec_err(gr, rd),
                     float(np.max(np.abs(gr - rr) / np.maximum(br, 1e-300))), "(u_s + 3u32)(|r| + |a Ap|)"))
        # the reduction runs over the stored new r: compare with the oracle's sum over the library's r
        rho_g = ops.norm(gr, st["w"])
        rows.append((name, "cg_update r.r", rel(g, rho_g), rel(g, rhod), rel(g, rho_g) / (3 * U32),
                     "3 u32 S (over the stored r)"))
        # BS7 scatter (map form and plan form)
        xLd = to_dev(xLs, dt)
        bs.bs_gs_scatter(ctx, plan, dev["x"], xLd)
        got = from_dev(xLd)
        ref_s = ops.scatter(ids, st["x"], xLs)
        rows.append((name, "scatter", vec_err(got, ref_s), vec_err(got, ops.scatter(ids, d64["x"], xL64)), 0.0,
                     "bit-exact on stored bits"))
        # BS6 gather
        xLd = to_dev(xLs, dt)
        xG = torch.empty_like(dev["x"])
        bs.bs_gather(ctx, plan, xLd, xG)
        got = from_dev(xG)
        ref_s = ops.gather(rs, ci, xLs)
        ref_d = ops.gather(rs, ci, xL64)
        absum = ops.gather(rs, ci, np.abs(xLs))
        bound = us * np.abs(ref_s) + deg * U32 * absum
        rows.append((name, "gather", vec_err(got, ref_s), vec_err(got, ref_d),
                     float(np.max(np.abs(got - ref_s) / np.maximum(bound, 1e-300))), "u_s |S| + deg u32 sum|terms|"))
        print(f"# {name} ops done in {time.time() - t0:.1f} s", flush=True)
        del dev, xLd, xG
    plan.close()

    # refinement solves against the binary64 CG
    shift = 0.01
    b = bsgen.uniform(SEED, S["b"], n)
    db = torch.from_numpy(b).cuda()
    lam_min = cg.eigenvalue(M, shift, 1, 1, 1)
    lam_max = cg.eigenvalue(M, shift, M, M, M)
    nb = math.sqrt(float(np.dot(b, b)))
    sol = {}
    for name, inner, tol_in in (("f64", None, None), ("ir_f32", bs.BS_F32, 1e-4), ("ir_bf16", bs.BS_BF16, 0.1)):
        x = torch.zeros(n, dtype=torch.float64, device="cuda")
        if inner is None:
            res = bs.bs_cg_solve(ctx, M, shift, db, x, tol=1e-10)
        else:
            res = bs.bs_cg_ir_solve(ctx, inner, M, shift, db, x, tol=1e-10, inner_tol=tol_in, max_outer=40)
        xh = x.cpu().numpy()
        r = b - cg.stencil7(xh, M, shift)
        sol[name] = (xh, math.sqrt(float(np.dot(r, r))), res)
        print(f"# solve {name} done", flush=True)
    x64, r64, _ = sol["f64"]
    solves = []
    for name in ("f64", "ir_f32", "ir_bf16"):
        xh, rn, res = sol[name]
        d = float(np.linalg.norm(xh - x64) / np.linalg.norm(x64))
        bound = (rn + r64) / lam_min / float(np.linalg.norm(x64))   # ||x - x*|| <= ||b - A x|| / lambda_min
        solves.append((name, res["iterations"], res["outer_iterations"], res["rel_residual"], rn / nb, d, bound))

    lines = ["# Binary32 and bfloat16 paths: measured error against the binary64 oracle", "",
             "Command (from the repository root on the GPU host):", "",
             "    python3 tests/lowprec_report.py profiles/lowprec_errors_n11390625.md", "",
             f"n = {n} (225^3); BS1-BS5 on global vectors (seed {SEED}, uniform[-1,1), weights uniform[0,1),",
             f"alpha = {ALPHA}, beta = {BETA}, CG-update alpha = 1e-3); BS7/BS6 on the N = 7, E = 32^3 mesh",
             f"(N_L = {NL}, elements permuted and oriented). \"err vs stored\": the oracle on the same rounded",
             "inputs (what the library is asked to compute); \"err vs f64\": the oracle on the original binary64",
             "draws (adds the storage rounding of the inputs). Vectors: max |err| / max |ref|; reductions:",
             "relative error. \"/ bound\": the largest error against the stated bound (<= 1 required).", "",
             "| dtype | operation | err vs stored | err vs f64 inputs | / bound | bound |", "|---|---|---|---|---|---|"]
    for name, op, es, ed, ratio, bnd in rows:
        lines.append(f"| {name} | {op} | {es:.3e} | {ed:.3e} | {ratio:.3f} | {bnd} |")
    lines += ["", f"Refinement to a true relative residual of 1e-10 on the 225^3 shifted 7-point operator",
              f"(lambda_min = {lam_min:.6g}, lambda_max = {lam_max:.6g}, kappa = {lam_max / lam_min:.1f});",
              "residuals recomputed here in binary64 from each x. Distance to the binary64 CG solution, and its",
              "bound (||r|| + ||r_64||) / (lambda_min ||x_64||) from ||x - x*|| <= ||b - A x|| / lambda_min:", "",
              "| form | iterations | outer | library residual | recomputed residual | ||x - x_64|| / ||x_64|| | bound |",
              "|---|---|---|---|---|---|---|"]
    for name, it, outer, lib_r, rr, d, bound in solves:
        lines.append(f"| {name} | {it} | {outer} | {lib_r:.3e} | {rr:.3e} | {d:.3e} | {bound:.3e} |")
    text = "\n".join(lines) + "\n"
    if out_path:
        with open(out_path, "w") as fh:
            fh.write(text)
    print(text)
    bad = [r for r in rows if r[4] > 1.0] + [s for s in solves if s[4] > 1e-10 or s[5] > s[6]]
    ctx.close()
    return 1 if bad else 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1] if len(sys.argv) > 1 else ""))
