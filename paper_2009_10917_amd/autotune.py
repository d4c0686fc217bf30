"""Autotuner for the launch shapes of the streaming operations.

    python -m paper_2009_10917_amd.autotune --out tune_gfx950.txt [--quick] [--only PART ...]

Measures, on the current GPU, every candidate launch shape of each
operation, dtype and length bucket, and writes the fastest as a tune table
(the text format bs_ctx_load_tune reads).  Install the table as
``paper_2009_10917_amd/tune_gfx950.txt`` (beside libbs.so), where
bs_ctx_create picks it up; BS_TUNE_FILE overrides it.

Candidates:
  copy, axpy        unroll {1, 2, 4, 8} x grid cap {1024, 4096, 16384, 65536, one pass},
                      same orders and workgroup sizes as below
  norm, dot,        unroll {1, 2, 4, 8} x grid cap {256, 1024, 4096, 16384, 65536,
  cg_update           one pass (up to 2^21 workgroups, the reductions' partial
                      buffer)}, and cap 1
                      up to 2^20 elements (one workgroup finishes the sum in the
                      same launch); from 2^20 elements on, each shape also with
                      the two XCD-grouped workgroup orders (variants 1 and 2);
                      every shape with 256-, 128- and 512-thread workgroups
                      (variant + 0, + 4, + 8); up to 2^24 elements each of
                      those also with cached instead of nontemporal accesses
                      (+ 16: vectors the next call finds in the 256 MB
                      last-level cache)
  batch             items per claim {1, 2, 4, 8} x workgroup cap {128, 256, 512,
                      resident} of the persistent batched step, on the 1024
                      box-mesh instances (binary64, binary32)
  gather, scatter   kernel variant {0, 1, 2}, each in the three workgroup orders
                    (one range per XCD, +4 dispatch order, +8 runs of 256 blocks
                    per XCD), and up to 2^24 local entries kernel 0 with cached
                    accesses (+16), on permuted and oriented N = 7 meshes, with
                    plans as bs_gs_create builds them (a caller that applies
                    bs_gs_order_rows chooses gather variant 0 itself); for the
                    scatter's tile variants (0, 1) also 1, 2 or 4 tiles per
                    workgroup (the unroll field), for its map-order variant (2)
                    1 or 4 entries per thread

Each candidate is timed with HIP events around back-to-back calls on
resident inputs (median of three trials after a warm-up).  A candidate
replaces the built-in default only when it is faster by more than 2%, so
that noise does not move the table.  The timings of every candidate are
written beside the table as JSON lines.
"""

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

STREAM_OPS = ("copy", "axpy", "norm", "dot", "cg_update")
REDUCTIONS = ("norm", "dot", "cg_update")
DTYPES = (("f64", 0), ("f32", 1), ("bf16", 2))
# bucket lower bounds and the length timed in each bucket
# (past 2^24 elements most operations' operands outgrow the last-level cache and the library
# drops cached accesses, so the launch shape timed with them at 2^24 stops at 2^24)
BUCKETS = ((0, 1 << 12), (1 << 13, 1 << 14), (1 << 15, 1 << 15), (1 << 16, 1 << 18), (1 << 20, 1 << 22),
           (1 << 23, 1 << 24), ((1 << 24) + 1, 3 << 23), (1 << 25, 1 << 26), (1 << 27, 1 << 28))
# cached accesses (+16) are tried where an operation's vectors can stay in the 256 MB last-level cache
CACHED_MAX_N = 1 << 24
MESH_K = ((0, 4), (1 << 20, 16), (1 << 24, 32), (1 << 26, 64), (1 << 29, 128))  # (n_min of N_L, K) for gather/scatter
DEFAULTS = {"copy": (1, 1 << 30, 0), "axpy": (1, 1 << 30, 0), "norm": (8, 4096, 0), "dot": (8, 4096, 0),
            "cg_update": (4, 65536, 0), "gather": (1, 1 << 30, 1), "scatter": (2, 1 << 30, 1),
            "batch": (8, 1 << 30, 0)}
MARGIN = 0.98


def _time(torch, fn, reps, trials=3):
    fn()
    torch.cuda.synchronize()
    out = []
    for _ in range(trials):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        out.append(a.elapsed_time(b) / reps)
    return statistics.median(out)


def _time_graph(torch, fn, reps, trials=3):
    """`reps` calls captured in one HIP graph, replayed: the device's time per call
    without the host's per-call cost, which hides launch shapes at short lengths."""
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
    out = []
    for _ in range(trials):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        g.replay()
        b.record()
        torch.cuda.synchronize()
        out.append(a.elapsed_time(b) / reps)
    del g
    return statistics.median(out)


def _pick(times, default):
    """Fastest candidate, unless the default is within the margin."""
    best = min(times, key=times.get)
    if default in times and times[best] >= MARGIN * times[default]:
        return default
    return best


def tune_streaming(torch, bs, bsgen, ctx, quick, log):
    entries = []
    tdt = {0: torch.float64, 1: torch.float32, 2: torch.bfloat16}
    for dname, did in DTYPES:
        for n_min, n in BUCKETS:
            if quick and n > (1 << 24):
                continue
            vec = {}
            for k, sid in (("x", 1), ("y", 2), ("p", 3), ("r", 4), ("Ap", 5), ("w", 6)):
                t = torch.empty(n, dtype=tdt[did], device="cuda")
                bsgen.device_uniform(t, 10917, sid, lo=0.0 if k == "w" else -1.0)
                vec[k] = t
            out = torch.zeros(1, dtype=torch.float64, device="cuda")
            calls = {
                "copy": lambda: bs.bs_copy(ctx, vec["x"], vec["y"]),
                "axpy": lambda: bs.bs_axpy(ctx, 0.37, vec["x"], 0.61, vec["y"]),
                "norm": lambda: bs.bs_norm(ctx, vec["x"], vec["w"], out),
                "dot": lambda: bs.bs_dot(ctx, vec["x"], vec["y"], out),
                "cg_update": lambda: bs.bs_cg_update(ctx, 1e-3, vec["x"], vec["p"], vec["r"], vec["Ap"], vec["w"], out),
            }
            reps = 50 if n <= (1 << 20) else 10
            # up to 2^22 elements a call takes less device time than the host spends issuing it
            timer = _time_graph if n <= (1 << 22) else _time
            for op in STREAM_OPS:
                caps = (256, 1024, 4096, 16384, 65536, 1 << 30) if op in REDUCTIONS else (1024, 4096, 16384, 65536, 1 << 30)
                if op in REDUCTIONS and n <= (1 << 20):
                    # grids of up to 128 workgroups finish the reduction in the same launch
                    caps = (1, 16, 64, 128) + caps
                times = {}
                # below 2^20 elements a launch has fewer than 2048 workgroups (or one),
                # where the orders differ little
                orders = (0, 1, 2) if n >= (1 << 20) else (0,)
                # workgroup size: + 0 for 256 threads, + 4 for 128, + 8 for 512
                variants = [o + b for b in (0, 4, 8) for o in orders]
                if n <= CACHED_MAX_N:
                    variants += [v + 16 for v in variants]
                for u in (1, 2, 4, 8):
                    for g in caps:
                        for v in variants:
                            bs.bs_ctx_set_tune(ctx, op, u, g, v)
                            times[(u, g, v)] = timer(torch, calls[op], reps)
                            log.write(json.dumps({"op": op, "dtype": dname, "n": n, "unroll": u, "grid_cap": g,
                                                  "variant": v, "ms": round(times[(u, g, v)], 5)}) + "\n")
                choice = _pick(times, DEFAULTS[op])
                entries.append((op, dname, n_min, *choice))
                bs.bs_ctx_set_tune(ctx, op, *DEFAULTS[op])
                print(f"# {op:9s} {dname:4s} n={n:>10d}: {choice} {times[choice]:.4f} ms "
                      f"(default {times.get(DEFAULTS[op], float('nan')):.4f})", flush=True)
            del vec, out
            torch.cuda.empty_cache()
    return entries


def tune_gather_scatter(torch, np, bs, bsgen, ctx, quick, log):
    entries = {("gather", d): [] for d, _ in DTYPES}
    entries.update({("scatter", d): [] for d, _ in DTYPES})
    N, seed = 7, 10917
    for n_min, K in MESH_K:
        if quick and K > 64:
            continue
        E, M = K ** 3, K * N + 1
        NL, NG = E * (N + 1) ** 3, M ** 3
        perm = torch.from_numpy(bsgen.permutation(seed, E).astype(np.int32)).cuda()
        orient = torch.from_numpy(bsgen.orientations(seed, E).astype(np.uint8)).cuda()
        d_map = torch.empty(NL, dtype=torch.int32, device="cuda")
        bs.bs_mesh_hex_map(K, N, perm, orient, d_map)
        plan = bs.bs_gs_create(ctx, d_map, NG)
        del d_map, perm, orient
        for dname, did in DTYPES:
            tdt = {0: torch.float64, 1: torch.float32, 2: torch.bfloat16}[did]
            xL = torch.empty(NL, dtype=tdt, device="cuda")
            xG = torch.empty(NG, dtype=tdt, device="cuda")
            bsgen.device_uniform(xL, seed, 11)
            bsgen.device_uniform(xG, seed, 12)
            reps = 50 if NL <= (1 << 22) else 5
            for op, call in (("gather", lambda: bs.bs_gather(ctx, plan, xL, xG)),
                             ("scatter", lambda: bs.bs_gs_scatter(ctx, plan, xG, xL))):
                times = {}
                variants = [0, 1, 2, 4, 5, 6, 8, 9, 10]
                if NL <= CACHED_MAX_N:  # kernel 0 with cached accesses (+ 16)
                    variants += [16, 20, 24]
                for v in variants:
                    unrolls = (1,) if op == "gather" else ((1, 2, 4) if v % 4 < 2 else (1, 4))
                    for u in unrolls:
                        bs.bs_ctx_set_tune(ctx, op, u, 1 << 30, v)
                        times[(u, 1 << 30, v)] = (_time_graph if NL <= (1 << 22) else _time)(torch, call, reps)
                        log.write(json.dumps({"op": op, "dtype": dname, "n_local": NL, "unroll": u, "variant": v,
                                              "ms": round(times[(u, 1 << 30, v)], 5)}) + "\n")
                choice = _pick(times, DEFAULTS[op])
                entries[(op, dname)].append((op, dname, n_min, *choice))
                bs.bs_ctx_set_tune(ctx, op, *DEFAULTS[op])
                print(f"# {op:9s} {dname:4s} K={K:4d}: {choice} {times[choice]:.4f} ms "
                      f"(default {times.get(DEFAULTS[op], float('nan')):.4f})", flush=True)
            del xL, xG
        plan.close()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    return [e for v in entries.values() for e in v]


def write_table(path, entries, device, seconds, quick):
    with open(path, "w") as f:
        f.write("# Launch-shape table for the streaming operations (bs_ctx_load_tune format)\n")
        f.write(f"# measured by paper_2009_10917_amd/autotune.py{' --quick' if quick else ''} on {device} "
                f"in {seconds:.0f} s\n")
        f.write("# op dtype n_min unroll grid_cap variant\n")
        for op, dname, n_min, u, g, v in entries:
            f.write(f"{op} {dname} {n_min} {u} {g} {v}\n")


def tune_batch(torch, np, bs, bsgen, ctx, quick, log, n_inst=1024):
    """Items per claim and the workgroup cap of the persistent batched step,
    on the box-mesh instances of the batched configuration (binary64 and
    binary32; bfloat16 takes binary32's choice)."""
    E, N = bsgen.batch_instances(10917, 128 if quick else n_inst)
    maps, nl, ng = [], [], []
    for e, d in zip(E, N):
        m, g = bs.bs_mesh_box_map_host(int(e), int(d))
        maps.append(m)
        nl.append(m.size)
        ng.append(g)
    d_map = torch.from_numpy(np.concatenate(maps)).cuda()
    b = bs.bs_batch_create(ctx, nl, ng, d_map)
    del maps, d_map
    entries = []
    streams = {"x": 1, "y": 2, "p": 3, "r": 4, "Ap": 5, "xL": 11, "pL": 12, "wL": 6}
    for dname, did, dt in (("f64", 0, torch.float64), ("f32", 1, torch.float32)):
        v = {}
        for k, sid in streams.items():
            t = torch.empty(b.n_global if k in bs.BATCH_GLOBAL else b.n_local, dtype=dt, device="cuda")
            bsgen.device_uniform(t, 10917, sid, lo=0.0 if k == "wL" else -1.0)
            v[k] = t
        out = torch.zeros(8 * b.n_inst, dtype=torch.float64, device="cuda")
        times = {}
        for claim in (1, 2, 4, 8):
            for cap in (128, 256, 512, 1 << 30):
                bs.bs_ctx_set_tune(ctx, "batch", claim, cap, 0)
                times[(claim, cap, 0)] = _time(torch, lambda: bs.bs_batch_step(ctx, b, v, 0.37, 0.61, out, 2), 5)
                log.write(json.dumps({"op": "batch", "dtype": dname, "claim": claim, "grid_cap": cap,
                                      "ms": round(times[(claim, cap, 0)], 5)}) + "\n")
        choice = _pick(times, DEFAULTS["batch"])
        bs.bs_ctx_set_tune(ctx, "batch", *DEFAULTS["batch"])
        print(f"# batch     {dname:4s} {b.n_inst} instances: {choice} "
              f"{times[choice]:.4f} ms (default {times[DEFAULTS['batch']]:.4f})", flush=True)
        entries.append(("batch", dname, 0, *choice))
        if dname == "f32":
            entries.append(("batch", "bf16", 0, *choice))
        del v, out
    b.close()
    torch.cuda.empty_cache()
    return entries


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--out", default="tune_gfx950.txt")
    ap.add_argument("--quick", action="store_true", help="skip the largest sizes")
    ap.add_argument("--only", choices=("streaming", "gs", "batch"), action="append",
                    help="search these parts only (repeatable; default: all)")
    args = ap.parse_args(argv)
    os.environ["BS_TUNE_FILE"] = "none"  # measure against the built-in defaults
    import numpy as np
    import torch

    import bsgen
    import paper_2009_10917_amd as bs

    if not torch.cuda.is_available():
        print("autotune needs a GPU", file=sys.stderr)
        return 1
    ctx = bs.bs_ctx_create(0)
    t0 = time.time()
    with open(args.out + ".jsonl", "w") as log:
        parts = args.only or ("streaming", "gs", "batch")
        entries = []
        if "streaming" in parts:
            entries += tune_streaming(torch, bs, bsgen, ctx, args.quick, log)
        if "gs" in parts:
            entries += tune_gather_scatter(torch, np, bs, bsgen, ctx, args.quick, log)
        if "batch" in parts:
            entries += tune_batch(torch, np, bs, bsgen, ctx, args.quick, log)
    props = torch.cuda.get_device_properties(0)
    device = f"{getattr(props, 'gcnArchName', '?').split(':')[0]} ({props.multi_processor_count} CUs)"
    write_table(args.out, entries, device, time.time() - t0, args.quick)
    n = bs.bs_ctx_load_tune(ctx, args.out)  # the library must accept what it will load
    print(f"# wrote {n} entries to {args.out}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
