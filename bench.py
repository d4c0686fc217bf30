#!/usr/bin/env python3
"""Benchmark of the seven Benchmark-Streaming operations on one MI355X.

One step is one pass of the whole hot path over resident synthetic inputs:
BS1 copy, BS2 AXPY, BS3 weighted norm, BS4 inner product and BS5 fused CG
update on global vectors of n = (7*128+1)^3 = 721,734,273 binary64 values
(the N = 7, E = 128^3 global mesh vector, the top of the length sweep), then
BS7 scatter and BS6 gather on that mesh's element map (E = 128^3, N = 7:
1,073,741,824 local nodes; elements randomly permuted and oriented).

Prints one JSON line: aggregate algorithmic GB/s over the step (`value`),
per-operation GB/s, fraction of the 8 TB/s HBM peak and GDOF/s, the
roofline record of the dominant kernel (the fused CG update) and a timed
CPU baseline (the oracle on a bounded sample of the same workload).

    python bench.py [--steps K] [--warmup W] [--small] [--no-cpu-baseline]
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "HBM GB/s & %peak per op; CG-update GDOF/s, FP64 plain vs mixed/batched"
HBM_PEAK_GBS = 8000.0
OPS = ("copy", "axpy", "norm", "dot", "cg_update", "scatter", "gather")


def alg_bytes(n, nl, ng, s=8, idx=4):
    """Algorithmic bytes per call (weighted norm and CG update)."""
    return {
        "copy": 2 * s * n,
        "axpy": 3 * s * n,
        "norm": 2 * s * n,
        "dot": 2 * s * n,
        "cg_update": 7 * s * n,
        "scatter": idx * nl + s * ng + s * nl,
        "gather": s * nl + idx * nl + s * ng,
    }


def source_digest():
    """Digest of what decides the CG-update launch: the streaming kernels'
    sources, the library's constants and the installed tune table."""
    h = hashlib.sha256()
    pkg = os.path.join(ROOT, "paper_2009_10917_amd")
    for f in ("csrc/bs_device.h", "csrc/bs_stream_ops.h", "csrc/bs_stream.hip", "csrc/bs_internal.h", "tune_gfx950.txt"):
        with open(os.path.join(pkg, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def committed_kernel_average(kernel):
    """Average duration (us) and command of `kernel` in the committed
    rocprofv3 kernel statistics of the benchmark step (its first table,
    whose header names the columns), or (None, None)."""
    path = os.path.join(ROOT, "profiles", "bench_step_kernel_stats_K128.md")
    if not os.path.exists(path):
        return None, None
    cmd, cols = None, None
    for line in open(path):
        if line.strip().startswith("cd /tmp") and cmd is None:
            cmd = line.strip()
        if not line.strip().startswith("|"):
            continue
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if cols is None and "kernel" in cells and "average (us)" in cells:
            cols = (cells.index("kernel"), cells.index("average (us)"))
            continue
        if cols and len(cells) > max(cols) and cells[cols[0]] == kernel:
            try:
                return float(cells[cols[1]]), cmd
            except ValueError:
                return None, cmd
    return None, cmd


def read_traffic(per_launch_alg):
    """HBM bytes per launch of the CG-update kernel from the committed counter
    summary, if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "cg_update_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_digest") != source_digest():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cpu_inputs(n_sample, K_mesh, N_mesh, seed):
    import bsgen
    from oracle import mesh

    xs = {k: bsgen.uniform(seed, bsgen.STREAM[k], n_sample) for k in ("x", "y", "p", "r", "Ap")}
    xs["w"] = bsgen.uniform(seed, bsgen.STREAM["w"], n_sample, lo=0.0)
    E, NL, NG = mesh.sizes(K_mesh, N_mesh)
    ids = mesh.hex_map(K_mesh, N_mesh, bsgen.permutation(seed, E), bsgen.orientations(seed, E))
    xL = bsgen.uniform(seed, bsgen.STREAM["xL"], NL)
    xG = bsgen.uniform(seed, bsgen.STREAM["xG"], NG)
    return xs, ids, xL, xG, NL, NG


def _plain_chunk(args):
    """The seven operations in plain numpy (np.dot and np.add.reduceat
    reductions, no exact sums) on a slice of the shared inputs: one worker's
    share of the vectors, of the local entries (scatter) and of the global
    rows (gather)."""
    import numpy as np
    from multiprocessing import shared_memory

    names, shapes, lo, hi, glo, ghi, rlo, rhi, a, b = args
    shm = {k: shared_memory.SharedMemory(name=v) for k, v in names.items()}
    arr = {k: np.ndarray(shapes[k], dtype=np.int64 if k in ("ids", "rs", "ci") else np.float64, buffer=shm[k].buf)
           for k in names}
    t0 = time.perf_counter()
    x, y, p, r, Ap, w = (arr[k][lo:hi] for k in ("x", "y", "p", "r", "Ap", "w"))
    y2 = x.copy()                                   # BS1
    y2 = a * x + b * y                              # BS2 (into a new array: inputs stay shared)
    nrm = float(np.dot(w * x, x))                   # BS3 weighted
    dt = float(np.dot(x, y2))                       # BS4
    x2 = x + a * p                                  # BS5
    r2 = r - a * Ap
    rr = float(np.dot(w * r2, r2))
    xL = arr["xG"][arr["ids"][glo:ghi]]             # BS7 on this slice of local entries
    rs = arr["rs"][rlo:rhi + 1]                     # BS6 on this range of global rows (no empty rows here)
    g = np.add.reduceat(arr["xL"][arr["ci"][rs[0]:rs[-1]]], rs[:-1] - rs[0]) if rhi > rlo else np.zeros(1)
    out = (time.perf_counter() - t0, nrm + dt + rr + float(y2[:1].sum() + x2[:1].sum() + xL[:1].sum() + g[:1].sum()))
    for v in shm.values():
        v.close()
    return out


def _plain_timing(xs, ids, rs, ci, xL, xG, workers, a, b):
    """Wall time of the plain numpy forms over `workers` processes (one
    process on one pinned core when workers == 1), inputs in shared memory."""
    import numpy as np
    import multiprocessing as mp
    from multiprocessing import shared_memory

    data = dict(xs, ids=ids.astype(np.int64), rs=np.asarray(rs, dtype=np.int64), ci=np.asarray(ci, dtype=np.int64),
                xL=xL, xG=xG)
    shm, names, shapes = {}, {}, {}
    try:
        for k, v in data.items():
            m = shared_memory.SharedMemory(create=True, size=max(v.nbytes, 1))
            np.ndarray(v.shape, dtype=v.dtype, buffer=m.buf)[:] = v
            shm[k], names[k], shapes[k] = m, m.name, v.shape
        n, nl, ng = xs["x"].size, ids.size, xG.size
        cuts = [(n * i // workers, n * (i + 1) // workers, nl * i // workers, nl * (i + 1) // workers,
                 ng * i // workers, ng * (i + 1) // workers) for i in range(workers)]
        ctx = mp.get_context("spawn")
        env_keep = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
        for k in env_keep:
            os.environ[k] = "1"
        try:
            with ctx.Pool(workers, initializer=_pin_worker, initargs=(workers,)) as pool:
                pool.map(_plain_chunk, [(names, shapes, *c, a, b) for c in cuts])  # warm-up (imports, pages)
                t0 = time.perf_counter()
                pool.map(_plain_chunk, [(names, shapes, *c, a, b) for c in cuts])
                return time.perf_counter() - t0
        finally:
            for k, v in env_keep.items():
                if v is None:
                    os.environ.pop(k, None)
                else:
                    os.environ[k] = v
    finally:
        for m in shm.values():
            m.close()
            m.unlink()


def _pin_worker(workers):
    # one core per worker; a single worker runs on the first allowed core
    try:
        cores = sorted(os.sched_getaffinity(0))
        ident = mp_identity()
        os.sched_setaffinity(0, {cores[ident % len(cores)]} if workers <= len(cores) else set(cores))
    except (AttributeError, OSError):
        pass


def mp_identity():
    import multiprocessing as mp
    ident = mp.current_process()._identity
    return (ident[0] - 1) if ident else 0


def cpu_baseline(n_sample, K_mesh, N_mesh, seed, max_workers=16):
    """CPU baselines on a bounded sample of the workload (BS1-BS5 on n_sample
    values, BS6/BS7 on the K_mesh^3, N_mesh permuted and oriented mesh).

    `value` is the oracle as it stands (numpy binary64 with exact fsum
    reductions) on one thread.  Beside it: the plain numpy forms of the
    seven operations (np.dot and reduceat reductions, no exact sums) on one
    pinned core and over all usable cores (a process pool, inputs in shared
    memory, at most max_workers processes).  All three report algorithmic
    bytes / wall time."""
    import numpy as np

    from oracle import mesh, ops

    xs, ids, xL, xG, NL, NG = _cpu_inputs(n_sample, K_mesh, N_mesh, seed)
    rs, ci = mesh.csr_inverse(ids, NG)
    a, b = 0.37, 0.91
    t0 = time.perf_counter()
    ops.copy(xs["x"])
    ops.axpy(a, xs["x"], b, xs["y"])
    ops.norm(xs["x"], xs["w"])
    ops.dot(xs["x"], xs["y"])
    ops.cg_update(a, xs["x"], xs["p"], xs["r"], xs["Ap"], xs["w"])
    ops.scatter(ids, xG, xL)
    ops.gather(rs, ci, xL)
    dt = time.perf_counter() - t0
    total = sum(alg_bytes(n_sample, NL, NG).values())
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    workers = max(1, min(max_workers, usable))
    t1 = _plain_timing(xs, ids, rs, ci, xL, xG, 1, a, b)
    tn = _plain_timing(xs, ids, rs, ci, xL, xG, workers, a, b)
    sample = (f"BS1-BS5 on n={n_sample} global binary64 values (weighted norm and CG update) and BS7/BS6 on the "
              f"K={K_mesh}, N={N_mesh} permuted/oriented mesh (N_L={NL}, N_G={NG}); algorithmic bytes / wall time")
    return {
        "value": round(total / dt / 1e9, 4),
        "unit": "GB/s",
        "cores": 1,
        "kind": "oracle",
        "seconds": round(dt, 3),
        "sample": "oracle as it stands (numpy binary64, exact fsum reductions), one thread: " + sample,
        "cpu_model": _cpu_model(),
        "os_cpu_count": os.cpu_count(),
        "usable_cores": usable,
        "numpy_one_core": {"value": round(total / t1 / 1e9, 4), "unit": "GB/s", "cores": 1, "seconds": round(t1, 3),
                           "kind": "plain numpy forms (np.dot / reduceat reductions), one process pinned to one core"},
        "numpy_all_cores": {"value": round(total / tn / 1e9, 4), "unit": "GB/s", "cores": workers,
                            "seconds": round(tn, 3),
                            "kind": f"plain numpy forms over {workers} processes (one core each), shared-memory inputs"},
    }


def _time_graph(fn, reps, torch):
    """`reps` calls captured in one HIP graph; seconds per call of a replay.
    Removes the host's per-call cost, leaving the device's launch latency."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(reps):
            fn()
    g.replay()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    g.replay()
    b.record()
    torch.cuda.synchronize()
    del g
    return a.elapsed_time(b) * 1e-3 / reps


def _time_calls(fn, reps, torch):
    """The paper's protocol: `reps` back-to-back calls timed as one block
    (HIP events on the launch stream, and the host clock around a sync)."""
    fn()
    fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    h0 = time.perf_counter()
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    host = (time.perf_counter() - h0) / reps
    return a.elapsed_time(b) * 1e-3 / reps, host


def sweep(args, K_max):
    import numpy as np
    import torch

    import bsgen
    import paper_2009_10917_amd as bs
    from paper_2009_10917_amd import perfmodel

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    ctx = bs.bs_ctx_create(0)
    S = bsgen.STREAM
    n_max = (7 * K_max + 1) ** 3
    vec = {}
    for k in ("x", "y", "p", "r", "Ap", "w"):
        t = torch.empty(n_max, dtype=torch.float64, device=dev)
        bsgen.device_uniform(t, args.seed, S[k], lo=0.0 if k == "w" else -1.0)
        vec[k] = t
    out = torch.zeros(4, dtype=torch.float64, device=dev)
    reps = 20
    results = []
    Ks = list(range(2, K_max + 1, 2))
    for op in ("copy", "axpy", "norm", "dot", "cg_update"):
        pts = []
        for K in Ks:
            n = (7 * K + 1) ** 3
            v = {k: t[:n] for k, t in vec.items()}
            calls = {
                "copy": lambda: bs.bs_copy(ctx, v["x"], v["y"]),
                "axpy": lambda: bs.bs_axpy(ctx, 0.5, v["x"], 0.5, v["y"]),
                "norm": lambda: bs.bs_norm(ctx, v["x"], v["w"], out[0:1]),
                "dot": lambda: bs.bs_dot(ctx, v["x"], v["y"], out[1:2]),
                "cg_update": lambda: bs.bs_cg_update(ctx, 1e-9, v["x"], v["p"], v["r"], v["Ap"], v["w"], out[2:3]),
            }
            t_dev, t_host = _time_calls(calls[op], reps, torch)
            t_graph = _time_graph(calls[op], reps, torch)
            B = alg_bytes(n, 0, 0)[op]
            pts.append({"K": K, "n": n, "bytes": B, "t_event_s": t_dev, "t_host_s": t_host, "t_graph_s": t_graph,
                        "GB_s": B / t_dev / 1e9, "GB_s_host": B / t_host / 1e9, "GB_s_graph": B / t_graph / 1e9})
        print(f"# swept {op}", file=sys.stderr, flush=True)
        results.append(_fit_record(op, pts, perfmodel))
    del vec
    torch.cuda.empty_cache()
    # gather / scatter on N = 7 meshes, K = 2, 4, ..., K_gs
    K_gs = min(64, K_max)
    pts = [_mesh_points(K, 7, args.seed, ctx, bs, bsgen, torch, np, reps) for K in range(2, K_gs + 1, 2)]
    print("# swept gather/scatter over K", file=sys.stderr, flush=True)
    for op in ("scatter", "gather", "gather (lattice rows)"):
        results.append(_fit_record(op + " (N=7)", [p[op] for p in pts], perfmodel))
    # gather / scatter at about 5e7 local nodes for N = 1..15
    pts = [_mesh_points(round(368.4 / (N + 1)), N, args.seed, ctx, bs, bsgen, torch, np, reps) for N in range(1, 16)]
    for op in ("scatter", "gather", "gather (lattice rows)"):
        rec = {"op": op + " (N-sweep, ~5e7 local nodes)", "points": [p[op] for p in pts]}
        print(json.dumps(rec))
        results.append(rec)
    if args.sweep_out:
        _write_sweep_md(args.sweep_out, results, K_max)
    return 0


def _mesh_points(K, N, seed, ctx, bs, bsgen, torch, np, reps):
    E = K ** 3
    NL, NG = E * (N + 1) ** 3, (K * N + 1) ** 3
    perm = torch.from_numpy(bsgen.permutation(seed, E).astype(np.int32)).cuda()
    orient = torch.from_numpy(bsgen.orientations(seed, E).astype(np.uint8)).cuda()
    d_map = torch.empty(NL, dtype=torch.int32, device="cuda")
    bs.bs_mesh_hex_map(K, N, perm, orient, d_map)
    plan = bs.bs_gs_create(ctx, d_map, NG)
    del d_map, perm, orient
    xL = torch.empty(NL, dtype=torch.float64, device="cuda")
    xG = torch.empty(NG, dtype=torch.float64, device="cuda")
    bsgen.device_uniform(xL, seed, bsgen.STREAM["xL"])
    bsgen.device_uniform(xG, seed, bsgen.STREAM["xG"])
    out = {}
    M = K * N + 1
    tile = N * max(1, round(GATHER_TILE / N))  # the benchmark's slabs, one element thick, at degree N

    lat_ctx = bs.bs_ctx_create(0)  # the benchmark's gather variant for every length, leaving ctx's table whole
    bs.bs_ctx_set_tune(lat_ctx, "gather", 1, 1 << 30, GATHER_VARIANT)

    def lattice_gather():
        bs.bs_gather(lat_ctx, plan, xL, xG)

    for op, fn in (("scatter", lambda: bs.bs_gs_scatter(ctx, plan, xG, xL)),
                   ("gather", lambda: bs.bs_gather(ctx, plan, xL, xG)),
                   ("gather (lattice rows)", lattice_gather)):
        if op == "gather (lattice rows)":
            bs.bs_gs_order_rows(plan, M, M, M, tile, (tile, N, N))
        t_dev, t_host = _time_calls(fn, reps, torch)
        t_graph = _time_graph(fn, reps, torch)
        B = alg_bytes(0, NL, NG)["gather" if op.startswith("gather") else op]
        out[op] = {"K": K, "N": N, "n_local": NL, "n_global": NG, "bytes": B, "t_event_s": t_dev,
                   "t_host_s": t_host, "t_graph_s": t_graph, "GB_s": B / t_dev / 1e9,
                   "GB_s_host": B / t_host / 1e9, "GB_s_graph": B / t_graph / 1e9}
    torch.cuda.synchronize()
    plan.close()
    lat_ctx.close()
    return out


def _fit_record(op, pts, perfmodel):
    rec = {"op": op, "points": pts}
    fits = (("all", "t_event_s", pts), ("ge_1GB", "t_event_s", [p for p in pts if p["bytes"] >= 1e9]),
            ("graph_all", "t_graph_s", pts), ("graph_le_256MB", "t_graph_s", [p for p in pts if p["bytes"] <= 256e6]))
    for tag, key, sel in fits:
        if len(sel) >= 2:
            t0, w = perfmodel.fit_time_model([p["bytes"] for p in sel], [p[key] for p in sel])
            # the model has a launch cost T0 >= 0 and a finite positive W_max; a fit that
            # lands outside says the points do not follow T0 + B/W_max (for instance a
            # bandwidth that keeps rising with size) and its T0 and B_0.8 mean nothing
            valid = t0 >= 0.0 and 0.0 < w < float("inf")
            rec["fit_" + tag] = {"T0_us": t0 * 1e6, "W_max_GB_s": w / 1e9,
                                 "B08_MB": perfmodel.fischer_brown_bytes(t0, w) / 1e6, "points": len(sel),
                                 "valid": valid}
    print(json.dumps(rec))
    return rec


def _write_sweep_md(path, results, K_max):
    lines = ["# Length and mesh sweeps with the launch-latency + bandwidth fit", "",
             "Command (from the repository root on the GPU host):", "",
             f"    python3 bench.py --sweep --K {K_max} --sweep-out <this file>", "",
             "20 back-to-back calls per size, timed with HIP events (host-clock figures in the JSON).",
             "Fit: least squares T = T0 + B/W_max (paper Section 4) over all sizes and over sizes >= 1 GB",
             "(smaller working sets stay in the 256 MB Infinity Cache between calls).", "",
             "Graph columns: the 20 calls captured in one HIP graph and replayed, which removes the host's",
             "per-call cost (Python binding and launch) and leaves the device's own launch latency.", "",
             "Gather and scatter run on permuted, oriented meshes with the plan's default order and the",
             "tune table's kernel; \"gather (lattice rows)\" is the same plan after bs_gs_order_rows with",
             "lattice tiles of about 126 points split into slabs one element thick (tile x N x N), gather",
             "variant 0's kernel with each XCD taking runs of 256 blocks (variant 8), as the benchmark step",
             "runs it (same bits, row order only).", "",
             "A fit whose T0 comes out negative does not describe its points (the model needs a",
             "non-negative launch cost); its T0 and B_0.8 cells read \"invalid (T0 < 0)\" and only the",
             "slope's W_max is shown.", "",
             "| operation | T0 (us) | W_max (GB/s) | B_0.8 (MB) | W_max >=1GB (GB/s) | graph T0 (us) | graph W_max (GB/s) | graph T0, <=256MB (us) | best GB/s (size) |",
             "|---|---|---|---|---|---|---|---|---|"]
    for r in results:
        best = max(r["points"], key=lambda p: p["GB_s"])
        fa, fg = r.get("fit_all"), r.get("fit_ge_1GB")
        ga, gs = r.get("fit_graph_all"), r.get("fit_graph_le_256MB")
        def cell(f, k, fmt):
            if not f:
                return "-"
            if not f.get("valid", True) and k != "W_max_GB_s":
                return "invalid (T0 < 0)"
            return fmt % f[k]
        lines.append(f"| {r['op']} | {cell(fa, 'T0_us', '%.2f')} | {cell(fa, 'W_max_GB_s', '%.0f')} | "
                     f"{cell(fa, 'B08_MB', '%.1f')} | {cell(fg, 'W_max_GB_s', '%.0f')} | {cell(ga, 'T0_us', '%.2f')} | "
                     f"{cell(ga, 'W_max_GB_s', '%.0f')} | {cell(gs, 'T0_us', '%.2f')} | "
                     f"{best['GB_s']:.0f} ({best['bytes'] / 1e9:.3g} GB) |")
    lines += ["", "Per-size bandwidth (GB/s, events):", ""]
    for r in results:
        lines.append(f"- {r['op']}: " + ", ".join(
            f"{p['bytes'] / 1e6:.3g} MB: {p['GB_s']:.0f}" for p in r["points"]))
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def mixed_cg(ctx, bs, bsgen, torch, seed, reps, m=225, shift=0.01, tol=1e-10):
    """Time-to-solution of CG on the shifted 7-point operator (m^3 unknowns).

    Forms: binary64 CG; iterative refinement (binary64 outer) around CG in
    binary32 storage and in bfloat16 storage.  Each solve starts from x = 0
    and ends on a true relative residual <= tol recomputed in binary64; its
    time is host wall clock around the whole call (workspace, graph capture
    and every refinement step included).  The effective GDOF/s of a form is
    n * (binary64 CG iterations) / t, so the speedup of a mixed form is
    t_f64 / t_mixed.
    """
    n = m ** 3
    b = torch.empty(n, dtype=torch.float64, device="cuda")
    bsgen.device_uniform(b, seed, bsgen.STREAM["b"])
    x = torch.zeros_like(b)
    forms = (("f64", None, None), ("ir_f32", bs.BS_F32, 1e-4), ("ir_bf16", bs.BS_BF16, 3e-3))
    out = {"m": m, "n": n, "shift": shift, "tol": tol}
    for name, inner, inner_tol in forms:
        times, rec = [], None
        for k in range(reps + 1):  # the first solve warms up code and allocator
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if inner is None:
                rec = bs.bs_cg_solve(ctx, m, shift, b, x, tol=tol, check=False)
            else:
                rec = bs.bs_cg_ir_solve(ctx, inner, m, shift, b, x, tol=tol, inner_tol=inner_tol, max_outer=40,
                                        check=False)
            torch.cuda.synchronize()
            if k:
                times.append(time.perf_counter() - t0)
        t = min(times)
        out[name] = {"status": rec["status"], "ms": round(t * 1e3, 3), "iterations": rec["iterations"],
                     "outer": rec["outer_iterations"], "restarts": rec["restarts"],
                     "true_rel_residual": rec["rel_residual"], "inner_tol": inner_tol,
                     "ms_per_inner_iteration": round(t * 1e3 / max(rec["iterations"], 1), 4)}
        print(f"# cg {name}: {out[name]}", file=sys.stderr, flush=True)
    it64 = out["f64"]["iterations"]
    for name, _, _ in forms:
        f = out[name]
        ok = f["status"] == "BS_OK"
        f["GDOF_s_effective"] = round(n * it64 / (f["ms"] * 1e-3) / 1e9, 3) if ok else None
        f["GDOF_s_ceed"] = round(n * f["iterations"] / (f["ms"] * 1e-3) / 1e9, 3)
        f["speedup_vs_f64"] = round(out["f64"]["ms"] / f["ms"], 3) if ok else None
    del b, x
    return out


def lowprec_ops(ctx, bs, bsgen, torch, np, seed, reps=20, m=225, K=32, N=7):
    """The seven operations at n = m^3 = 11,390,625 (the 225^3 grid of the
    mixed-precision configuration) with vectors stored in binary64, binary32
    and bfloat16: BS1-BS5 on global vectors (weighted norm and CG update),
    BS7/BS6 on the N = 7, E = 32^3 mesh (N_L = 16,777,216, N_G = 11,390,625)
    with the plan's default row order.  Events around `reps` back-to-back
    calls; algorithmic bytes with the storage size.  Working sets of
    23-340 MB partly stay in the 256 MB Infinity Cache between calls, so
    these are not HBM-roofline figures."""
    n = m ** 3
    E, NL = K ** 3, K ** 3 * (N + 1) ** 3
    S = bsgen.STREAM
    perm = torch.from_numpy(bsgen.permutation(seed, E).astype(np.int32)).cuda()
    orient = torch.from_numpy(bsgen.orientations(seed, E).astype(np.uint8)).cuda()
    d_map = torch.empty(NL, dtype=torch.int32, device="cuda")
    bs.bs_mesh_hex_map(K, N, perm, orient, d_map)
    plan = bs.bs_gs_create(ctx, d_map, n)
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    res = {"n": n, "n_local": NL, "n_global": n, "mesh": f"N={N}, E={K}^3, permuted and oriented", "reps": reps}
    for dname, dt, sz in (("f64", torch.float64, 8), ("f32", torch.float32, 4), ("bf16", torch.bfloat16, 2)):
        v = {}
        for k in ("x", "y", "p", "r", "Ap", "w"):
            t = torch.empty(n, dtype=dt, device="cuda")
            bsgen.device_uniform(t, seed, S[k], lo=0.0 if k == "w" else -1.0)
            v[k] = t
        xL = torch.empty(NL, dtype=dt, device="cuda")
        bsgen.device_uniform(xL, seed, S["xL"])
        xG = torch.empty(n, dtype=dt, device="cuda")
        calls = {
            "copy": lambda: bs.bs_copy(ctx, v["x"], v["y"]),
            "axpy": lambda: bs.bs_axpy(ctx, 0.37, v["x"], 1.0, v["y"]),
            "norm": lambda: bs.bs_norm(ctx, v["x"], v["w"], out[0:1]),
            "dot": lambda: bs.bs_dot(ctx, v["x"], v["y"], out[1:2]),
            "cg_update": lambda: bs.bs_cg_update(ctx, 1e-3, v["x"], v["p"], v["r"], v["Ap"], v["w"], out[2:3]),
            "scatter": lambda: bs.bs_gs_scatter(ctx, plan, v["y"], xL),
            "gather": lambda: bs.bs_gather(ctx, plan, xL, xG),
        }
        byt = alg_bytes(n, NL, n, s=sz)
        rec = {}
        for op, fn in calls.items():
            t_dev, _ = _time_calls(fn, reps, torch)
            gbs = byt[op] / t_dev / 1e9
            rec[op] = {"us": round(t_dev * 1e6, 2), "GB_s": round(gbs, 1), "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)}
        res[dname] = rec
        print(f"# lowprec {dname}: " + ", ".join(f"{k} {r['GB_s']}" for k, r in rec.items()), file=sys.stderr,
              flush=True)
        del v, xL, xG
    plan.close()
    res["errors"] = ("measured errors against the binary64 oracle: profiles/lowprec_errors_n11390625.md "
                     "(written by tests/lowprec_report.py)")
    return res


# sum-factorised local Helmholtz operator at degree 7 (padded tensor 8^3): the ten contractions
# of 8 x 8 matrices with the element tensor (forward B_k, B_j, [B; D]_i, Dh_j, Dh_k; backward
# Dh_k^T, Dh_j^T, [B^T D^T]_i, B^T_j, B^T_k) are 49,152 multiply-adds, plus about 22 flops per
# quadrature point for the geometric factors and weights; the matrix cores issue 88
# V_MFMA_F64_16X16X4F64 (2048 flops each, half of some of them on zero rows)
ELEM_FLOPS_N7 = 2 * 49152 + 22 * 512
ELEM_MFMA_FLOPS_N7 = 88 * 2048
FP64_PEAK_TFLOPS = 78.6


def elem_ops(ctx, bs, bsgen, torch, np, seed, reps=10, K=64, N=7):
    """Element operators on the N = 7, E = K^3 mesh (permuted, oriented):
    the sum-factorised local Helmholtz operator with the scatter fused in
    (x_L never written), the full y_G = Z^T A_L Z x_G (local operator + BS6
    gather), and the lumped mass in one pass over the CSR of Z^T, against
    the unfused scatter + gather it replaces; and CG on the assembled
    operator (time per iteration, GDOF/s)."""
    E, P = K ** 3, (N + 1) ** 3
    NL, NG = E * P, (K * N + 1) ** 3
    perm = torch.from_numpy(bsgen.permutation(seed, E).astype(np.int32)).cuda()
    orient = torch.from_numpy(bsgen.orientations(seed, E).astype(np.uint8)).cuda()
    d_map = torch.empty(NL, dtype=torch.int32, device="cuda")
    bs.bs_mesh_hex_map(K, N, perm, orient, d_map)
    plan = bs.bs_gs_create(ctx, d_map, NG)
    el = bs.bs_elem_create(ctx, N)
    h = 1.0 / K
    geo = torch.tensor([h / 2, 0, 0, h / 2, 0, h / 2, (h / 2) ** 3], dtype=torch.float64).repeat(E).cuda()
    xG = torch.empty(NG, dtype=torch.float64, device="cuda")
    bsgen.device_uniform(xG, seed, bsgen.STREAM["xG"])
    yG = torch.empty_like(xG)
    yL = torch.empty(NL, dtype=torch.float64, device="cuda")
    lam = 0.01
    calls = {
        "helmholtz_local": lambda: bs.bs_helmholtz_local(ctx, el, d_map, geo, lam, xG, yL),
        "helmholtz_apply": lambda: bs.bs_helmholtz_apply(ctx, el, plan, geo, lam, xG, yL, yG),
        "mass_lumped": lambda: bs.bs_mass_lumped(ctx, el, plan, geo, xG, yG),
        "scatter_then_gather": lambda: (bs.bs_gs_scatter(ctx, plan, xG, yL), bs.bs_gather(ctx, plan, yL, yG)),
    }
    local_bytes = 4 * NL + 8 * NG + 56 * E + 8 * NL       # map, x_G once, geometry, y_L
    byts = {"helmholtz_local": local_bytes,
            "helmholtz_apply": local_bytes + alg_bytes(0, NL, NG)["gather"],
            "mass_lumped": 4 * NL + 4 * (NG + 1) + 8 * NG + 8 * NG + 56 * E,  # CSR, x_G, y_G, geometry
            "scatter_then_gather": alg_bytes(0, NL, NG)["scatter"] + alg_bytes(0, NL, NG)["gather"]}
    res = {"K": K, "N": N, "elements": E, "n_local": NL, "n_global": NG, "lambda": lam, "reps": reps}
    for name, fn in calls.items():
        t, _ = _time_calls(fn, reps, torch)
        rec = {"us": round(t * 1e6, 2), "alg_bytes": byts[name], "GB_s": round(byts[name] / t / 1e9, 1),
               "frac_hbm_peak": round(byts[name] / t / 1e9 / HBM_PEAK_GBS, 4)}
        if name.startswith("helmholtz"):
            tf = ELEM_FLOPS_N7 * E / t / 1e12
            rec.update({"alg_flops": ELEM_FLOPS_N7 * E, "TFLOP_s": round(tf, 2),
                        "frac_fp64_peak": round(tf / FP64_PEAK_TFLOPS, 4),
                        "mfma_issued_TFLOP_s": round(ELEM_MFMA_FLOPS_N7 * E / t / 1e12, 2)})
        res[name] = rec
        print(f"# elem {name}: {rec}", file=sys.stderr, flush=True)
    # CG on the assembled operator: the time of an iteration from the
    # difference of two solves run to a fixed iteration count (set-up,
    # graph capture and the true residuals cancel)
    b = xG
    x = torch.zeros_like(xG)
    secs = {}
    for it in (16, 112):
        x.zero_()
        torch.cuda.synchronize()
        r = bs.bs_helmholtz_cg_solve(ctx, el, plan, geo, lam, b, x, tol=1e-30, max_iter=it, check=False)
        if r["iterations"] != it:
            raise RuntimeError(f"helmholtz cg stopped after {r['iterations']} of {it} iterations ({r['status']})")
        secs[it] = r["seconds"]
    per_it = (secs[112] - secs[16]) / 96
    it_bytes = byts["helmholtz_apply"] + 48 * NG + 24 * NG  # operator + gather, BS5 update, BS2 direction
    rec = {"ms_per_iteration": round(per_it * 1e3, 4), "GDOF_s": round(NG / per_it / 1e9, 3),
           "alg_bytes_per_iteration": it_bytes, "GB_s": round(it_bytes / per_it / 1e9, 1),
           "TFLOP_s_local": round(ELEM_FLOPS_N7 * E / per_it / 1e12, 2),
           "solve_seconds_16_112": [round(secs[16], 4), round(secs[112], 4)],
           "note": "binary64, lambda 0.01, b uniform; GDOF/s = global unknowns x iterations / time"}
    res["helmholtz_cg"] = rec
    print(f"# elem helmholtz_cg: {rec}", file=sys.stderr, flush=True)
    el.close()
    plan.close()
    return res


# gather row order: lattice tiles of GATHER_TILE^3 points, boxes of GATHER_BOX points inside (0: none);
# 126 = 18 elements of degree 7, boxes one element thick in y and z (slabs along x)
GATHER_TILE, GATHER_BOX = 126, (126, 7, 7)
# gather kernel: the plan's permuted row order (variant 0) with each XCD taking runs of 256 blocks
# in every group of 2048 (+8)
GATHER_VARIANT = 8


def gather_sweep(args, np, torch, bs, bsgen):
    """Gather and scatter on the K^3, N = 7 mesh in each plan order.  The
    gather: global row order (variant 1), the plan's default permuted order
    (variant 0, and 8 with each XCD taking runs of 256 workgroups); the
    scatter (the tune table's kernel, then the sorted-tile kernel with 2 or
    4 tiles per workgroup in each of the three workgroup orders) in the
    default tile order.  Then, for
    each spec in turn, the plan is re-ordered and both are timed again:
    "tile", "tile:side" or "tile:bxXbyXbz" sort the gather rows into lattice
    tiles (bs_gs_order_rows; gather variants 0 and 4); "elem:G" orders rows
    and tiles by elements in groups of G (bs_gs_order_elements with the
    order derived from the map; gather variants 0 and 8).  --mesh chooses
    the element layout: random (permuted and oriented, the benchmark's),
    orient (lexicographic, oriented) or ident (lexicographic, unrotated).
    One JSON line per (operation, order, variant); every output is checked
    bit for bit against the first one.  Each timing is two warm-up calls and
    --reps timed calls, in this order (for per-dispatch counters)."""
    K, N, seed = args.K, 7, args.seed
    E, M = K ** 3, K * N + 1
    P = (N + 1) ** 3
    NL, NG = E * P, M ** 3
    ctx = bs.bs_ctx_create(0)
    perm = orient = None
    if args.mesh == "random":
        perm = torch.from_numpy(bsgen.permutation(seed, E).astype(np.int32)).cuda()
    if args.mesh in ("random", "orient"):
        orient = torch.from_numpy(bsgen.orientations(seed, E).astype(np.uint8)).cuda()
    d_map = torch.empty(NL, dtype=torch.int32, device="cuda")
    bs.bs_mesh_hex_map(K, N, perm, orient, d_map)
    plan = bs.bs_gs_create(ctx, d_map, NG)
    del d_map, perm, orient
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    xL = torch.empty(NL, dtype=torch.float64, device="cuda")
    bsgen.device_uniform(xL, seed, 11)
    xG = torch.empty(NG, dtype=torch.float64, device="cuda")
    bsgen.device_uniform(xG, seed, 12)
    sL = torch.empty_like(xL)
    alg = alg_bytes(0, NL, NG)
    yG = torch.empty_like(xG)
    # explicit launch shapes go to a context of their own; ctx keeps the tune table
    fixed = bs.bs_ctx_create(0)

    def run_gather(variant):
        bs.bs_ctx_set_tune(fixed, "gather", 1, 1 << 30, variant)
        return _time_calls(lambda: bs.bs_gather(fixed, plan, xL, yG), args.reps, torch)[0] * 1e3

    def run_scatter(c=ctx):
        return _time_calls(lambda: bs.bs_gs_scatter(c, plan, xG, sL), args.reps, torch)[0] * 1e3

    def emit(op, order, variant, ms, same):
        print(json.dumps({"op": op, "order": order, "variant": variant, "mesh": args.mesh, "K": K, "ms": round(ms, 4),
                          "GB_s": round(alg[op] / (ms * 1e-3) / 1e9, 1), "bit_equal": same}), flush=True)

    def same(a, b):
        return torch.equal(a.view(torch.int64), b.view(torch.int64))

    ms = run_gather(1)
    ref = yG.clone()
    emit("gather", "global", 1, ms, True)
    for v in (0, 8):
        ms = run_gather(v)
        emit("gather", "plan default (groups of 9 visiting-order tiles)", v, ms, same(yG, ref))
    ms = run_scatter()
    sref = sL.clone()
    emit("scatter", "plan default (tiles by smallest global id)", -1, ms, True)
    for tpw in (2, 4):
        for v in (0, 4, 8):  # workgroup orders: one range per XCD, dispatch order, runs of 256 per XCD
            bs.bs_ctx_set_tune(fixed, "scatter", tpw, 1 << 30, v)
            ms = run_scatter(fixed)
            emit("scatter", f"plan default, {tpw} tiles per workgroup", v, ms, same(sL, sref))
    for spec in [t for t in args.gather_sweep.split(",") if t]:
        if spec.startswith("elem:"):
            bs.bs_gs_order_elements(plan, P, None, int(spec[5:]))
            variants = (0, 8)
        else:
            tile, _, box = spec.partition(":")
            box = tuple(int(v) for v in box.split("x")) if "x" in box else int(box or 0)
            bs.bs_gs_order_rows(plan, M, M, M, int(tile), box)
            variants = (0, 4)
        torch.cuda.synchronize()
        for v in variants:
            ms = run_gather(v)
            emit("gather", spec, v, ms, same(yG, ref))
        ms = run_scatter()
        emit("scatter", spec, -1, ms, same(sL, sref))
        bs.bs_ctx_set_tune(fixed, "scatter", 4, 1 << 30, 8)
        ms = run_scatter(fixed)
        emit("scatter", f"{spec}, 4 tiles per workgroup", 8, ms, same(sL, sref))
    fixed.close()
    return 0


BATCH_STREAMS = {"x": 1, "y": 2, "p": 3, "r": 4, "Ap": 5, "xL": 11, "pL": 12, "wL": 6}


def batch_bytes(n_global, n_local, s, idx=4):
    """Algorithmic bytes of one batch step: the seven operations and one CG
    iteration with A = Z^T Z on every instance (index arrays counted, CSR row
    starts not)."""
    per_g = (2 + 3 + 2 + 6 + 2 + 6 + 3) * s + 2 * s + 2 * s  # vector ops, scatter reads, gather writes
    per_l = 2 * s + 2 * (idx + s) + 2 * (s + idx)             # norm, two scatters, two gathers
    return per_g * n_global + per_l * n_local


def batched(ctx, bs, bsgen, torch, np, seed, reps, n_inst=1024):
    """Batched step over the box-mesh instances, in the three forms.

    Each form runs the same chunked kernels; per-phase and persistent steps
    are also captured in a HIP graph and replayed.  The step is timed with
    HIP events around `reps` back-to-back steps on resident vectors (which
    the steps keep updating).  GDOF/s counts the global unknowns of all
    instances advanced per second.
    """
    E, N = bsgen.batch_instances(seed, n_inst)
    maps, nl, ng = [], [], []
    for e, d in zip(E, N):
        m, g = bs.bs_mesh_box_map_host(int(e), int(d))
        maps.append(m)
        nl.append(m.size)
        ng.append(g)
    d_map = torch.from_numpy(np.concatenate(maps)).cuda()
    del maps
    b = bs.bs_batch_create(ctx, nl, ng, d_map)
    del d_map
    res = {"instances": n_inst, "n_local": b.n_local, "n_global": b.n_global,
           "elements": int(E.sum()), "persistent_workgroups": b.persistent_blocks}
    for dname, dt, size in (("f64", torch.float64, 8), ("f32", torch.float32, 4)):
        v = {}
        for k, sid in BATCH_STREAMS.items():
            t = torch.empty(b.n_global if k in bs.BATCH_GLOBAL else b.n_local, dtype=dt, device="cuda")
            bsgen.device_uniform(t, seed, sid, lo=0.0 if k == "wL" else -1.0)
            v[k] = t
        out = torch.zeros(8 * b.n_inst, dtype=torch.float64, device="cuda")
        byt = batch_bytes(b.n_global, b.n_local, size)
        forms = {}
        for name, mode, graph in (("per_instance", 0, False), ("per_phase", 1, False), ("per_phase_graph", 1, True),
                                  ("persistent", 2, False), ("persistent_graph", 2, True)):
            if mode == 2 and b.persistent_blocks <= 0:
                continue
            call = (lambda mode=mode: bs.bs_batch_step(ctx, b, v, 0.37, 0.61, out, mode))
            try:
                if graph:
                    ms = _time_graph(call, reps, torch) * 1e3
                else:
                    ms = max(_time_calls(call, reps, torch)) * 1e3  # host clock when launches bound it
            except Exception as exc:  # a form the runtime cannot capture is reported, not hidden
                forms[name] = {"error": str(exc)[:200]}
                continue
            forms[name] = {"ms": round(ms, 4), "GB_s": round(byt / (ms * 1e-3) / 1e9, 1),
                           "GDOF_s": round(b.n_global / (ms * 1e-3) / 1e9, 3)}
            print(f"# batch {dname} {name}: {forms[name]}", file=sys.stderr, flush=True)
        base = forms.get("per_instance", {}).get("ms")
        for f in forms.values():
            if base and "ms" in f:
                f["speedup_vs_per_instance"] = round(base / f["ms"], 2)
        forms["alg_bytes"] = byt
        forms["barrier_timeouts"] = bs.bs_batch_barrier_timeouts(b)
        res[dname] = forms
        del v, out
    b.close()
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=10917)
    ap.add_argument("--K", type=int, default=128, help="mesh elements per axis (vector n = (7K+1)^3)")
    ap.add_argument("--small", action="store_true", help="K = 32 (a quick check, not the benchmark workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1 << 25)
    ap.add_argument("--profile", default="",
                    help="comma-separated ops (op or op@variant): run each --reps times after set-up and exit "
                         "(for rocprofv3)")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--sweep", action="store_true",
                    help="length sweep of BS1-BS5 (n = (7K+1)^3, K = 2, 4, ..., --K) and mesh sweeps of BS6/BS7; "
                         "prints one JSON line per operation with the launch-latency + bandwidth fit")
    ap.add_argument("--sweep-out", default="", help="also write a markdown summary of the sweep here")
    ap.add_argument("--cg-only", action="store_true",
                    help="only the mixed-precision CG time-to-solution (225^3 shifted 7-point operator)")
    ap.add_argument("--no-cg", action="store_true", help="skip the mixed-precision CG section")
    ap.add_argument("--batch-only", action="store_true", help="only the batched step over 1024 box-mesh instances")
    ap.add_argument("--gather-sweep", default="",
                    help="comma-separated plan orders after the default (tile, tile:side or tile:bxXbyXbz lattice "
                         "tiles; elem:G element groups): time gather and scatter in each")
    ap.add_argument("--mesh", default="random", choices=("random", "orient", "ident"),
                    help="element layout for --gather-sweep")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched section")
    ap.add_argument("--no-elem", action="store_true", help="skip the element-operator section")
    ap.add_argument("--elem-only", action="store_true", help="only the element-operator section")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; multi-GPU runs are not part of it",
                          "n_gpus": args.gpus}))
        return 2
    K = 32 if args.small else args.K
    N = 7
    if args.sweep:
        return sweep(args, K)

    import numpy as np
    import torch

    import bsgen
    import paper_2009_10917_amd as bs

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        return 1
    if args.gather_sweep:
        return gather_sweep(args, np, torch, bs, bsgen)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    hs = stream.cuda_stream
    ctx = bs.bs_ctx_create(0)
    if args.cg_only:
        print(json.dumps({"metric": METRIC, "mixed_cg": mixed_cg(ctx, bs, bsgen, torch, args.seed, args.reps)}))
        return 0
    if args.elem_only:
        print(json.dumps({"metric": METRIC, "elem_ops": elem_ops(ctx, bs, bsgen, torch, np, args.seed)}))
        return 0
    if args.batch_only:
        print(json.dumps({"metric": METRIC, "batched": batched(ctx, bs, bsgen, torch, np, args.seed, args.reps)}))
        return 0

    E = K ** 3
    n = (K * N + 1) ** 3
    NL = E * (N + 1) ** 3
    print(f"# setup: n={n} NL={NL} (K={K}, N={N})", file=sys.stderr, flush=True)

    def vec(stream_id, lo=-1.0, size=n):
        t = torch.empty(size, dtype=torch.float64, device=dev)
        bsgen.device_uniform(t, args.seed, stream_id, lo=lo)
        return t

    S = bsgen.STREAM
    x, y, p, r, Ap = (vec(S[k]) for k in ("x", "y", "p", "r", "Ap"))
    w = vec(S["w"], lo=0.0)
    alpha, beta = (float(v) for v in bsgen.scalars(args.seed, K))
    out = torch.zeros(4, dtype=torch.float64, device=dev)

    perm = torch.from_numpy(bsgen.permutation(args.seed, E).astype(np.int32)).to(dev)
    orient = torch.from_numpy(bsgen.orientations(args.seed, E).astype(np.uint8)).to(dev)
    d_map = torch.empty(NL, dtype=torch.int32, device=dev)
    bs.bs_mesh_hex_map(K, N, perm, orient, d_map)
    plan = bs.bs_gs_create(ctx, d_map, n)
    del d_map, perm, orient
    # the gather runs in the plan's own row order, derived from the map alone
    # (groups of consecutive tiles of the scatter's visiting order); the
    # lattice-tiled order, which needs the ids to be lattice points, is timed
    # after the step as a structured-mesh extra
    M = K * N + 1
    bs.bs_ctx_set_tune(ctx, "gather", 1, 1 << 30, GATHER_VARIANT)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    xL = vec(S["xL"], size=NL)
    xG = vec(S["xG"], size=n)
    xG_out = torch.empty(n, dtype=torch.float64, device=dev)  # gather target, so no step feeds the next
    torch.cuda.synchronize()
    print("# inputs resident", file=sys.stderr, flush=True)

    def step_calls():
        return (
            lambda: bs.bs_copy(ctx, x, y, hs),
            lambda: bs.bs_axpy(ctx, alpha, x, beta, y, hs),
            lambda: bs.bs_norm(ctx, x, w, out[0:1], hs),
            lambda: bs.bs_dot(ctx, x, y, out[1:2], hs),
            lambda: bs.bs_cg_update(ctx, alpha, x, p, r, Ap, w, out[2:3], hs),
            lambda: bs.bs_gs_scatter(ctx, plan, xG, xL, hs),
            lambda: bs.bs_gather(ctx, plan, xL, xG_out, hs),
        )

    def step(ev=None):
        calls = step_calls()
        for i, c in enumerate(calls):
            if ev is not None:
                ev[i][0].record(stream)
            c()
            if ev is not None:
                ev[i][1].record(stream)

    if args.profile:
        names = [o for o in args.profile.split(",") if o]
        copy_probe = torch.empty_like(x)
        calls = dict(zip(OPS, step_calls()))
        calls["copy_probe"] = lambda: bs.bs_copy(ctx, x, copy_probe, hs)
        for name in names:
            op, _, variant = name.partition("@")
            if variant:
                u, g, _ = bs.bs_ctx_get_tune(ctx, op)
                bs.bs_ctx_set_tune(ctx, op, u, g, int(variant))
            for _ in range(args.reps):
                calls[op]()
            torch.cuda.synchronize()
            print(f"# profiled {name} x{args.reps}", file=sys.stderr, flush=True)
        return 0

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print("# warmup done", file=sys.stderr, flush=True)

    events = [[[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in OPS] for _ in range(args.steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_start.record(stream)
    for k in range(args.steps):
        step(events[k])
    t_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = t_start.elapsed_time(t_end)
    ms_step = max(ms_total, wall * 1e3) / args.steps

    per_ms = {op: sum(events[k][i][0].elapsed_time(events[k][i][1]) for k in range(args.steps)) / args.steps
              for i, op in enumerate(OPS)}
    byt = alg_bytes(n, NL, n)
    step_bytes = sum(byt.values())
    per_op = {}
    for op in OPS:
        gbs = byt[op] / (per_ms[op] * 1e-3) / 1e9
        per_op[op] = {"ms": round(per_ms[op], 4), "GB_s": round(gbs, 1), "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
                      "alg_bytes": byt[op]}
    per_op["cg_update"]["GDOF_s"] = round(n / (per_ms["cg_update"] * 1e-3) / 1e9, 3)
    value = step_bytes / (ms_step * 1e-3) / 1e9

    # structured-mesh extra (not part of the step): the gather in lattice-tiled rows
    bs.bs_gs_order_rows(plan, M, M, M, GATHER_TILE, GATHER_BOX)
    torch.cuda.synchronize()
    bs.bs_gather(ctx, plan, xL, xG_out, hs)
    lat_t, _ = _time_calls(lambda: bs.bs_gather(ctx, plan, xL, xG_out, hs), max(args.steps, 5), torch)
    lat_gbs = byt["gather"] / lat_t / 1e9
    per_op["gather"]["row_order"] = "plan default (map only)"
    per_op["gather_lattice_rows"] = {
        "ms": round(lat_t * 1e3, 4), "GB_s": round(lat_gbs, 1), "frac_hbm_peak": round(lat_gbs / HBM_PEAK_GBS, 4),
        "alg_bytes": byt["gather"], "in_step": False,
        "row_order": ("lattice tiles of {}^3 points, boxes of {}x{}x{} (needs global ids that are lattice points; "
                      "bs_gs_order_rows)").format(GATHER_TILE, *GATHER_BOX)}

    cg_gbs = per_op["cg_update"]["GB_s"]
    traffic = read_traffic(byt["cg_update"])
    cu, cg_cap, cvar = bs.bs_ctx_tune_for(ctx, "cg_update", n)
    cu = 8 if cu >= 8 else 4 if cu >= 4 else 2 if cu >= 2 else 1
    cnb = {1: 128, 2: 512}.get((cvar >> 2) & 3, 256)
    corder = cvar & 3 if (cvar & 3) in (1, 2) else 0
    cg_grid = max(1, min(cg_cap, 1 << 21, -(-(n // 2) // (cnb * cu))))
    cnt = "false" if cvar & 16 else "true"  # nontemporal accesses unless the tune entry asks for cached ones
    roofline = {"bound": "hbm", "kernel": f"k_cg_update<double, 2, {cu}, true, {cnb}, {cnt}>", "workgroups": cg_grid,
                "workgroup_order": corder, "workgroup_size": cnb, "achieved": cg_gbs,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(cg_gbs / HBM_PEAK_GBS, 4),
                "traffic": traffic, "alg_bytes_per_launch": byt["cg_update"],
                "avg_launch_ms": round(per_ms["cg_update"], 4),
                "achieved_source": "HIP events around each launch in this run (launch stream)"}
    avg_us, _ = committed_kernel_average(roofline["kernel"])
    if avg_us:
        a2 = byt["cg_update"] / (avg_us * 1e-6) / 1e9
        roofline["committed_stats"] = {
            "file": "profiles/bench_step_kernel_stats_K128.md", "avg_launch_us": avg_us,
            "achieved": round(a2, 1), "frac": round(a2 / HBM_PEAK_GBS, 4),
            "note": "rocprofv3 kernel-trace average from a separate process; buffer placement moves a "
                    "kernel's time by up to ~13% between processes"}

    result = {
        "metric": METRIC, "value": round(value, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": (f"BS1-BS5 on binary64 global vectors of n=(7*{K}+1)^3={n} (uniform[-1,1), "
                                f"weights uniform[0,1)); BS7 scatter and BS6 gather on the N=7, E={K}^3 hex mesh "
                                f"(N_L={NL}, N_G={n}; elements permuted and oriented from the seed)"),
                   "n": n, "n_local": NL, "n_global": n, "mesh_K": K, "degree_N": N, "seed": args.seed,
                   "gather_row_order": ("plan default, from the map alone: rows in groups of 9 consecutive "
                                        "512-entry tiles of the scatter's visiting order (tiles by smallest global "
                                        "id), ascending global id within a group"),
                   "gather_variant": GATHER_VARIANT, "alpha": alpha, "beta": beta},
        "per_op": per_op,
        "roofline": roofline,
    }
    del x, y, p, r, Ap, w, xL, xG, xG_out
    plan.close()
    torch.cuda.synchronize()
    if not args.no_elem:
        result["elem_ops"] = elem_ops(ctx, bs, bsgen, torch, np, args.seed)
    if not args.no_cg:
        result["lowprec_ops"] = lowprec_ops(ctx, bs, bsgen, torch, np, args.seed)
        result["mixed_cg"] = mixed_cg(ctx, bs, bsgen, torch, args.seed, args.reps)
    if not args.no_batch:
        result["batched"] = batched(ctx, bs, bsgen, torch, np, args.seed, args.reps)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(args.cpu_sample, 16, N, args.seed)
    print(json.dumps(result))
    return 0


if __name__ == "__main__":
    sys.exit(main())
