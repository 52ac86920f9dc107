"""Benchmark: off-tree edges scored per second by the whole GRASS path on one MI355X.

One step = one grass_sparsify call on the C2 workload (100^3 7-point mesh, weights
10^U(-3,3), k = 32 random vectors, t = 2 power steps, sigma^2 = 100, iterative
densification): Boruvka tree, tree layout, every densification pass (start
vectors, Laplacian products, tree / PCG solves, scoring, estimates, filtering,
similarity check) until kappa_est <= sigma^2. Inputs are resident in HBM before
the timed region. value = sum over passes of the off-subgraph edges scored,
divided by the step time.

Prints one JSON line (plus diagnostics on stderr).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "off-tree edges scored/sec at sigma^2=100; p50/p99 sparsify latency vs plain path"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name: str):
    from paper_1911_04382_amd import graphs as G

    if name == "c2":
        g = G.config_c2(100)
        cfg = dict(k=32, t=2, sigma2=100.0, precision=32)
        desc = "100^3 7-point mesh (1e6 nodes, 2.97e6 edges), weights 10^U(-3,3), k=32, t=2, sigma^2=100, iterative"
    elif name == "c3":
        g = G.config_c3(2000)
        # FP64: on this graph the FP32 block PCG with FP64 refinement does not reach
        # the 1e-6 residual in the later power steps (it stalls near 1e-5 and diverges
        # in the first densified pass); FP64 converges in every pass and is faster
        # overall (53.8 s against 58.5 s per call, 15,124 against 32,884 iterations)
        cfg = dict(k=16, t=3, sigma2=50.0, precision=64)
        desc = ("2000^2 grid + 1% long-range edges (4e6 nodes, 8.08e6 edges), lognormal(0,2), k=16, t=3, sigma^2=50, "
                "FP64")
    elif name == "c1":
        g = G.config_c1()
        cfg = dict(k=8, t=2, sigma2=100.0, precision=64, max_iters=1)
        desc = "64x64 grid, U[1,10), k=8, t=2, FP64, one densification pass"
    elif name.startswith("mesh"):
        side = int(name[4:])
        g = G.config_c2(side)
        cfg = dict(k=32, t=2, sigma2=100.0, precision=32)
        desc = f"{side}^3 7-point mesh, weights 10^U(-3,3), k=32, t=2, sigma^2=100, iterative"
    else:
        raise SystemExit(f"unknown workload {name}")
    return g, cfg, desc


def host_cpu():
    """nproc and the CPU model of the host (reported beside every oracle number)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def cpu_baseline(g, cfg, sample_side=30):
    """The FP64 oracle (single thread) on a bounded sample of the same workload: the
    whole method (tree, every densification pass with its tree / PCG solves,
    scoring, filtering) on a sample_side^3 mesh of the same family and options,
    like for like with the GPU's end-to-end value. Also its tree pass on the full
    graph, whose heats serve the accuracy check. Returns (baseline dict, oracle
    tree-pass heats, oracle tree-pass stats)."""
    import oracle as O
    from paper_1911_04382_amd import graphs as G

    gs = G.config_c2(sample_side)
    t0 = time.perf_counter()
    r = O.sparsify(gs, sigma2=cfg["sigma2"], k=cfg["k"], t=cfg["t"], seed=0)
    t1 = time.perf_counter()
    scored = sum(tr["m_off"] for tr in r.trace)
    tree = O.max_spanning_tree(g)
    t2 = time.perf_counter()
    res = O.embed(g, tree, k=cfg["k"], t=cfg["t"], seed=0, pass_=0)
    t3 = time.perf_counter()
    m_off = int(res.stats["m_off"])
    base = {
        "value": scored / (t1 - t0),
        "unit": "edges/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"oracle, whole sparsify call on a {sample_side}^3 mesh of the same family ({gs.n} nodes, "
                   f"{gs.m} edges, k={cfg['k']}, t={cfg['t']}, sigma^2={cfg['sigma2']}, FP64, 1 thread): "
                   f"{r.summary['passes']} passes, {scored} off-tree edges scored in {t1 - t0:.2f} s"),
        "tree_pass_full_graph": {"value": m_off / (t3 - t2 + t2 - t1), "unit": "edges/s",
                                 "sample": f"Kruskal {t2 - t1:.2f} s + embedding/scoring {t3 - t2:.2f} s on the full "
                                           f"graph, {m_off} off-tree edges"},
        **host_cpu(),
    }
    return base, res.heat, res.stats


def accuracy(grass, ctx, dg, g, cfg, heat_ora, st_ora):
    """Error of the GPU tree pass (pass 0 of the timed workload, the benchmark's
    precision and kernels) against the FP64 oracle's, on the full graph: normalized
    scores s = heat / max off-tree heat (eq. 58), per-edge relative error for
    edges with s_oracle >= 1e-5, and the lambda estimates."""
    import numpy as np

    tree = grass.grass_spanning_tree(ctx, dg)
    heat, st = grass.grass_embed(ctx, dg, tree, grass.make_opts(**cfg), pass_=0)
    h = heat.double().cpu().numpy()
    off = tree.cpu().numpy() == 0
    s_gpu = h / h[off].max()
    s_ora = heat_ora / heat_ora[off].max()
    d = np.abs(s_gpu - s_ora)[off]
    big = off & (s_ora >= 1e-5)
    rel = np.abs(s_gpu - s_ora)[big] / s_ora[big]
    return {"what": "tree pass (pass 0) on the full graph against the FP64 oracle",
            "score_err_max": float(d.max()), "score_rel_err_max": float(rel.max()),
            "score_rel_err_p99": float(np.quantile(rel, 0.99)), "score_rel_err_median": float(np.median(rel)),
            "rel_err_floor": 1e-5, "edges_above_floor": int(big.sum()),
            "lambda_max_rel_err": abs(st["lambda_max"] - st_ora["lambda_max"]) / st_ora["lambda_max"],
            "lambda_min_rel_err": abs(st["lambda_min"] - st_ora["lambda_min"]) / st_ora["lambda_min"]}


def true_kappa(grass, ctx, dg, mask, cfg, steps=(50, 100)):
    """lambda_max of the final sparsifier by continuing the power iteration
    (Sec. IV-C.1) on one vector, FP64, to each step count in `steps` (two counts
    show convergence), against the t-step estimate that stopped the loop.
    lambda_min >= 1 for a subgraph (Sec. II-C) and <= the eq. (61) estimate. One
    vector: after this many steps every vector of a block is the same dominant
    eigenvector, and a block of identical right-hand sides leaves the block PCG
    rank-deficient."""
    out = {"vectors": 1, "precision": "f64"}
    t0 = time.perf_counter()
    for n in steps:
        c = dict(cfg)
        c.update(k=1, lambda_steps=n, precision=64)
        _, st = grass.grass_embed(ctx, dg, mask, grass.make_opts(**c), pass_=1000)
        out[f"lambda_max_{n}_steps"] = st["lambda_max"]
        out["lambda_min_est"] = st["lambda_min"]
    lm = out[f"lambda_max_{steps[-1]}_steps"]
    out.update(kappa_upper=lm, kappa_lower=lm / out["lambda_min_est"], seconds=time.perf_counter() - t0)
    return out


def lambda_leg(grass, ctx, dg, cfg, torch, ws, steps=8):
    """The benchmark workload with lambda_max estimated from `steps` continued power
    steps (Sec. IV-C.1; the paper's Table IV uses fewer than ten) instead of the
    t-step iterate that also scores the edges: one timed call, and the true kappa
    of its sparsifier (50 continued steps on one vector, FP64)."""
    c = dict(cfg)
    c["lambda_steps"] = steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    try:
        r = grass.grass_sparsify(ctx, dg, grass.make_opts(**c), ws=ws)
    except grass.GrassError as e:
        return {"lambda_steps": steps, "error": str(e)}
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    s = r.summary
    out = {"lambda_steps": steps, "status": r.status, "seconds": dt, "passes": s["passes"],
           "added_edges": s["added_edges"], "scored_edges": s["scored_edges"],
           "edges_per_s": s["scored_edges"] / dt, "kappa_est": s["kappa"], "pcg_iters": s["pcg_iters"]}
    out["true_kappa_50_steps"] = true_kappa(grass, ctx, dg, r.mask, cfg, steps=(50,))["kappa_upper"]
    return out


def copy_ceiling(torch, nbytes: int = 1 << 30, reps: int = 10) -> float:
    """This device's measured HBM ceiling: a plain device-to-device copy of nbytes,
    timed with events over reps copies after one untimed one; GB/s counts the bytes
    read and the bytes written."""
    n = nbytes // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    del src, dst
    return 2.0 * n * 4 / sec / 1e9


def copy_calibration(nbytes: int = 1 << 30, reps: int = 5):
    """A plain device-to-device copy of known size (the PMC byte counters of this
    kernel calibrate FETCH_SIZE / WRITE_SIZE against real bytes)."""
    import torch

    n = nbytes // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read": n * 4, "bytes_written": n * 4, "reps": reps}}), flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pcg_kernels_c2_mesh100_traffic.md")
PROFILED_SOURCES = ["embed.hip", "embed.h", "bpcg.hip", "lap.h", "gram.h", "common.h", "state.h", "kern.h"]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed PMC summary (FETCH_SIZE and
    WRITE_SIZE scaled by a device-copy calibration), or None when there is none for
    this kernel and workload or the kernel's source changed since it was measured."""
    import hashlib

    if workload != "c2" or not os.path.exists(TRAFFIC_FILE):
        return None
    h = hashlib.sha256()
    for f in PROFILED_SOURCES:
        with open(os.path.join(ROOT, "paper_1911_04382_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    vals = {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            if "=" in line and line.startswith("    "):
                k, v = (x.strip() for x in line.split("=", 1))
                vals[k] = v
    if vals.get("source") != h.hexdigest()[:16]:
        return None
    v = vals.get(f"traffic_bytes_per_launch.{kernel}")
    return float(v) if v is not None else None


def percentile(xs, q):
    ys = sorted(xs)
    if not ys:
        return None
    pos = (len(ys) - 1) * q
    lo = int(math.floor(pos))
    hi = min(lo + 1, len(ys) - 1)
    return ys[lo] + (ys[hi] - ys[lo]) * (pos - lo)


def run_batch(args, grass, torch):
    """C4: many independent graphs. The plain path sparsifies them one after another
    on one stream; grass_sparsify_batch runs `workers` at once, kernel by kernel or
    with captured block-PCG chunks and loop control on the device."""
    from paper_1911_04382_amd import graphs as G

    legs = set(args.c4_legs.split(","))
    sizes = G.config_c4_sizes(256)[: args.count]
    gs = [G.config_c4_graph(kind, n, seed=i) for i, (kind, n) in enumerate(sizes)]
    dgs = [grass.to_device(g, "cuda:0") for g in gs]
    opts = grass.make_opts(k=16, t=2, sigma2=100.0, precision=32)
    ctx = grass.Context(0)
    torch.cuda.synchronize()
    log(f"C4: {len(gs)} graphs, {sum(g.n for g in gs)} nodes, {sum(g.m for g in gs)} edges")
    plain, t_plain = None, None
    if "plain" in legs:
        t0 = time.perf_counter()
        plain = []
        for i, dg in enumerate(dgs):
            plain.append(grass.grass_sparsify(ctx, dg, opts))  # returns when the graph is done
            if (i + 1) % 8 == 0:
                log(f"plain path: {i + 1}/{len(dgs)} graphs at {time.perf_counter() - t0:.1f} s")
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
    ws = grass.batch_workspace(dgs, opts, args.workers)

    def batch(mode, label):
        ctx.set_launch_mode(mode, 0)
        ctx.launch_stats(reset=True)
        t0 = time.perf_counter()
        log(f"batch path ({label}): {len(dgs)} graphs, {args.workers} workers ...")
        rc, out = grass.grass_sparsify_batch(ctx, dgs, opts, workers=args.workers, ws=ws)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = ctx.launch_stats()
        log(f"batch path ({label}): done in {dt:.1f} s, {st}")
        same = None if plain is None else all(
            torch.equal(a.mask, b.mask) and torch.equal(a.scores, b.scores) for a, b in zip(out, plain))
        return dt, out, same, st

    runs = {}
    if "kernels" in legs:
        # worker pool, kernel by kernel (the host reads the loop state every 4th iteration)
        runs["kernels"] = batch(grass.LAUNCH_KERNELS, "kernel by kernel")
    if "captured" in legs:
        # captured chunks, loop control on the device; the first run also tunes the
        # chunks per read of each size class, the second reuses the choices
        runs["captured_tuning"] = batch(grass.LAUNCH_CAPTURED, "captured, tuning")
        runs["captured"] = batch(grass.LAUNCH_CAPTURED, "captured, tuned")
    key = "captured" if "captured" in runs else ("kernels" if "kernels" in runs else None)
    if key is None:
        ctx.close()
        print(json.dumps({"metric": "off-tree edges scored/sec, batch of independent graphs", "plain_s": t_plain}),
              flush=True)
        return
    t_batch, out, _, _ = runs[key]
    sames = [r[2] for r in runs.values() if r[2] is not None]
    scored = sum(r.summary["scored_edges"] for r in out)
    line = {"metric": "off-tree edges scored/sec, batch of independent graphs", "value": scored / t_batch,
            "unit": "edges/s", "n_gpus": 1, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"C4: first {len(gs)} of 256 graphs cycling 2D mesh / 3D mesh / RGG, n log-uniform "
                                   "[1e3, 2e5], U[1,10), k=16, t=2, sigma^2=100",
                       "graphs": len(gs), "nodes": sum(g.n for g in gs), "workers": args.workers,
                       "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES"), "launch": key},
            "batch_s": t_batch, "plain_s": t_plain,
            "runs_s": {k: r[0] for k, r in runs.items()},
            "launch_stats": {k: r[3] for k, r in runs.items()},
            "plain_value": scored / t_plain if t_plain else None,
            "speedup": t_plain / t_batch if t_plain else None,
            "identical_to_plain": all(sames) if sames else None,
            "statuses": {str(k): sum(1 for r in out if r.status == k) for k in sorted({r.status for r in out})}}
    ctx.close()
    print(json.dumps(line), flush=True)


def run_solve(args, grass, torch):
    """Sec. V-E on C2: sparsify, then solve L_G x = b for 16 seeded random right-hand
    sides to ||L_G x - b|| <= 1e-3 ||b|| with the sparsifier as the preconditioner,
    and with the spanning tree alone (the paper's N with and without sparsification)."""
    from paper_1911_04382_amd import graphs as G

    g = G.config_c2(100)
    dg = grass.to_device(g, "cuda:0")
    ctx = grass.Context(0)
    res = grass.grass_sparsify(ctx, dg, grass.make_opts(k=32, t=2, sigma2=100.0, precision=32))
    torch.cuda.synchronize()
    log(f"solve: sparsifier with {res.summary['added_edges']} added edges, kappa {res.summary['kappa']:.1f}")
    gen = torch.Generator(device="cpu").manual_seed(7)
    b = torch.randn(g.n, 16, generator=gen, dtype=torch.float32)
    b = (b - b.mean(0)).to("cuda:0")
    # each application of the sparsifier: 16 block-PCG iterations on L_P, no FP64
    # restart (flexible CG absorbs the inexact, varying preconditioner); measured
    # against inner solves to a tolerance: 1e-1 took 3.3 s, 5e-1 2.1 s, a fixed 8
    # iterations 1.12 s, 16 1.07 s, 32 1.50 s
    sopts = grass.make_opts(k=16, precision=32, pcg_rtol=1e-3, pcg_max_iters=16, pcg_max_outer=1)
    out = {}
    for label, mask in (("sparsifier", res.mask), ("tree", None)):
        ws = grass.solve_workspace(dg, sopts)
        rc, x, info = grass.grass_solve(ctx, dg, b, sopts, p_mask=mask, rtol=1e-3, max_iters=5000, ws=ws)
        torch.cuda.synchronize()
        info["status"] = rc
        info["edges_per_node"] = (g.n - 1 + info["added_edges"]) / g.n
        out[label] = info
        log(f"  {label}: {info['iters']} iterations ({info['inner_iters']} inner), {info['ms']:.1f} ms, "
            f"residual {info['resid']:.2e}")
    line = {"metric": "PCG on L_G to ||r|| <= 1e-3 ||b|| with the sparsifier as the preconditioner (Sec. V-E)",
            "value": out["sparsifier"]["ms"], "unit": "ms (16 right-hand sides)", "n_gpus": 1,
            "higher_is_better": False, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "C2 graph (100^3 mesh, 10^U(-3,3)), sparsifier from grass_sparsify at sigma^2=100, "
                                   "16 seeded Gaussian right-hand sides (mean removed), each preconditioner application "
                                   "one block-PCG phase on L_P (to 1e-2, at most 16 iterations)"},
            "sparsifier": out["sparsifier"], "tree": out["tree"],
            "iteration_ratio_tree_over_sparsifier": out["tree"]["iters"] / max(1, out["sparsifier"]["iters"])}
    ctx.close()
    print(json.dumps(line), flush=True)


def run_lsst(args, grass, torch):
    """Sec. III-A: the sparsifier built on the low-stretch spanning tree against the
    one built on the maximum-weight tree, at sigma^2 = 100, k = 32, FP32: tree time,
    the first pass's lambda_max (the tree's spectral distance to G, bounded by its
    total stretch), passes, added edges and sparsify time. Graphs: the C2 graph and a
    unit-weight 60^3 mesh (equal weights, where the maximum-weight tree with ties
    by edge id is a comb)."""
    import time

    from paper_1911_04382_amd import graphs as G

    ctx = grass.Context(0)
    out = {}
    for name, g in (("c2", G.config_c2(100)), ("unit_mesh60", G.mesh3d(60, 60, 60, weights=(G.W_CONST, 1.0, 1.0)))):
        dg = grass.to_device(g, "cuda:0")
        rows = {}
        for kind in ("max_weight", "low_stretch"):
            grass.grass_spanning_tree(ctx, dg) if kind == "max_weight" else grass.grass_low_stretch_tree(ctx, dg)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            tree = (grass.grass_spanning_tree(ctx, dg) if kind == "max_weight"
                    else grass.grass_low_stretch_tree(ctx, dg, seed=0, class_bits=2))
            torch.cuda.synchronize()
            t_tree = (time.perf_counter() - t0) * 1e3
            opts = grass.make_opts(k=32, t=2, sigma2=100.0, precision=32, init_mask=tree)
            t0 = time.perf_counter()
            res = grass.grass_sparsify(ctx, dg, opts)
            torch.cuda.synchronize()
            t_sp = (time.perf_counter() - t0) * 1e3
            rows[kind] = {"tree_ms": round(t_tree, 2), "first_lambda_max": res.trace[0]["lambda_max"],
                          "passes": res.summary["passes"], "added_edges": res.summary["added_edges"],
                          "kappa": res.summary["kappa"], "status": res.status, "sparsify_ms": round(t_sp, 1),
                          "pcg_iters": res.summary["pcg_iters"]}
            log(f"lsst {name} {kind}: {rows[kind]}")
        out[name] = {"n": g.n, "m": g.m, **rows}
    line = {"metric": "sparsify time on the low-stretch spanning tree vs the maximum-weight tree (Sec. III-A)",
            "value": out["c2"]["low_stretch"]["sparsify_ms"], "unit": "ms (C2 graph)", "n_gpus": 1,
            "higher_is_better": False, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "C2 graph (100^3 mesh, 10^U(-3,3)) and a unit-weight 60^3 mesh; sigma^2=100, "
                                   "k=32, t=2; low-stretch tree seed 0, class_bits 2"},
            "graphs": out}
    ctx.close()
    print(json.dumps(line), flush=True)


def run_lambda(args, grass, torch):
    """NEXT 1 / Table IV: lambda_max of the final sparsifier estimated by s generalized
    power steps (s = 2, 4, 8, 16; the paper uses fewer than ten) against the larger
    of the values the same iteration reaches after 50 and 100 steps, on synthetic
    stand-ins for the paper's matrices. FP32 like the default path; every call is
    one embedding pass of s steps."""
    from paper_1911_04382_amd import graphs as G

    ctx = grass.Context(0)
    graphs = [("mesh3d_30", G.mesh3d(30, 30, 30, weights=(G.W_LOGUNIFORM10, -3, 3), seed=1)),
              ("grid2d_150", G.grid2d(150, 150, seed=2)),
              ("ba_20k", G.ba(20000, seed=3)),
              ("rgg_20k", G.rgg(20000, seed=4))]
    out = {}
    for name, g in graphs:
        dg = grass.to_device(g, "cuda:0")
        res = grass.grass_sparsify(ctx, dg, grass.make_opts(k=32, t=2, sigma2=100.0, precision=32))
        torch.cuda.synchronize()
        log(f"lambda {name}: sparsifier with {res.summary['added_edges']} added edges, kappa {res.summary['kappa']:.1f}")
        est = {}
        for steps in (2, 4, 8, 16, 50, 100):
            opts = grass.make_opts(k=32, t=2, precision=32, seed=1, lambda_steps=steps)
            _, st = grass.grass_embed(ctx, dg, res.mask, opts, pass_=0)
            torch.cuda.synchronize()
            est[steps] = st["lambda_max"]
            log(f"lambda {name}: {steps} steps -> {st['lambda_max']:.6g}")
        # every estimate is a Rayleigh quotient, so a lower bound of lambda_max: the
        # reference is the larger of the 50- and 100-step values (FP32 rounding
        # leaves the longer run a little below the shorter one at times)
        ref = max(est[50], est[100])
        out[name] = {"n": g.n, "m": g.m, "added_edges": res.summary["added_edges"], "lambda_max_ref": ref,
                     "lambda_max_50": est[50], "lambda_max_100": est[100],
                     "estimates": {str(s): est[s] for s in (2, 4, 8, 16)},
                     "rel_error": {str(s): (ref - est[s]) / ref for s in (2, 4, 8, 16)}}
    line = {"metric": "relative error of the lambda_max estimate after s power steps on the final sparsifier "
                      "(Sec. IV-C.1, Table IV)",
            "value": max(v["rel_error"]["8"] for v in out.values()), "unit": "max relative error at 8 steps",
            "n_gpus": 1, "higher_is_better": False, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "final sparsifiers (sigma^2=100, k=32, FP32) of a 30^3 mesh 10^U(-3,3), a 150^2 "
                                   "grid, a 20k BA graph and a 20k geometric graph; estimates with k=32, FP32"},
            "graphs": out}
    ctx.close()
    print(json.dumps(line), flush=True)


def run_partition(args, grass, torch):
    """Sec. V-F on a synthetic 500 x 500 mesh with random weights: sign cut after 5
    inverse power steps with the sparsifier-preconditioned solver at 1e-3 against
    the cut from tight solves (1e-6), as the paper compares with a direct solver
    (both FP64: on this mesh FP32 cannot hold a 1e-3 residual)."""
    from paper_1911_04382_amd import graphs as G

    g = G.grid2d(500, 500, seed=11)
    dg = grass.to_device(g, "cuda:0")
    ctx = grass.Context(0)
    res = grass.grass_sparsify(ctx, dg, grass.make_opts(k=16, t=2, sigma2=100.0, precision=32))
    torch.cuda.synchronize()
    log(f"partition: sparsifier with {res.summary['added_edges']} added edges")
    rc1, u1, s1, fast = grass.grass_partition(ctx, dg, grass.make_opts(precision=64, seed=5, pcg_rtol=1e-1),
                                              p_mask=res.mask, steps=5, rtol=1e-3)
    log(f"  1e-3 done: {fast}")
    log("  tight solves (1e-6) ...")
    rc2, u2, s2, tight = grass.grass_partition(ctx, dg, grass.make_opts(precision=64, seed=5, pcg_rtol=1e-2),
                                               p_mask=res.mask, steps=5, rtol=1e-6)
    torch.cuda.synchronize()
    diff = float((s1 != s2).float().mean())
    cos = abs(float((u1.double() * u2).sum()))
    log(f"  1e-3: {fast}; 1e-6: {tight}; sides differ on {100 * diff:.3f}% of nodes, |cos| {cos:.6f}")
    line = {"metric": "spectral partitioning with the sparsifier: share of nodes whose sign differs from tight "
                      "solves (Sec. V-F)", "value": 100 * diff, "unit": "% of nodes", "n_gpus": 1,
            "higher_is_better": False, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "500x500 4-neighbour mesh, U[1,10), sparsifier at sigma^2=100 (k=16, t=2), "
                                   "5 inverse power steps"},
            "fast": dict(fast, status=rc1), "tight": dict(tight, status=rc2), "abs_cos": cos,
            "speedup_fast_vs_tight": tight["ms"] / fast["ms"]}
    ctx.close()
    print(json.dumps(line), flush=True)


def run_serving(args, grass, torch):
    rhos = [float(x) for x in args.rho_sweep.split(",")] if args.rho_sweep else None
    line = serving_leg(args.count, args.c5_max_n, args.rho, args.workers, args.arena_gb, grass, torch, rhos)
    print(json.dumps(line), flush=True)


def serving_leg(count, max_n, rho, workers, arena_gb, grass, torch, rhos=None):
    """C5: a Poisson stream of sparsify requests on preferential-attachment graphs.
    Plain path: one request at a time in arrival order on one stream. Server:
    continuous batching with admission by workspace footprint. Both see the same
    arrival times; latency = completion - arrival. With rhos, the server runs once
    per arrival rate (plain service times measured once) and the line carries every
    rate under "sweep"."""
    import numpy as np
    from paper_1911_04382_amd import graphs as G

    sizes = G.config_c5_sizes(count, lo=1e4, hi=max_n, seed=1)
    gs = [G.config_c5_graph(int(n), seed=100 + i) for i, n in enumerate(sizes)]
    dgs = [grass.to_device(g, "cuda:0") for g in gs]
    opts = grass.make_opts(k=16, t=2, sigma2=100.0, precision=32)
    ctx = grass.Context(0)
    torch.cuda.synchronize()
    # plain-path service times (also the capacity that sets the arrival rate)
    ws = grass.workspace(max(dgs, key=lambda d: d.n + d.m), opts, "cuda:0")
    service = []
    for i, dg in enumerate(dgs):
        t0 = time.perf_counter()
        grass.grass_sparsify(ctx, dg, opts, ws=ws)
        torch.cuda.synchronize()
        service.append(time.perf_counter() - t0)
        log(f"plain path: request {i + 1}/{len(dgs)} (n={dg.n}) {service[-1] * 1e3:.0f} ms")
    del ws
    mu = 1.0 / (sum(service) / len(service))
    need = max(grass.load_library().grass_workspace_bytes(d.n, d.m, opts) for d in dgs)

    def run(rho_):
        rate = rho_ * mu
        rng = np.random.Generator(np.random.Philox(key=1))
        arrivals = np.cumsum(rng.exponential(1.0 / rate, size=len(dgs)))
        log(f"C5: {len(dgs)} requests, n in [{min(g.n for g in gs)}, {max(g.n for g in gs)}], mean service "
            f"{1e3 / mu:.0f} ms, arrival rate {rate:.2f}/s (rho {rho_})")
        # plain FIFO at these arrival times (simulated clock: service times measured above)
        clock, lat_plain = 0.0, []
        for a, sv in zip(arrivals, service):
            clock = max(clock, a) + sv
            lat_plain.append(clock - a)
        # the server, live
        free0 = torch.cuda.mem_get_info()[0]
        srv = grass.Server(ctx, max(need * workers, int(arena_gb * (1 << 30))), workers=workers)
        hbm_server = free0 - torch.cuda.mem_get_info()[0]  # the server's arena and per-worker state
        t0 = time.perf_counter()
        tickets = []
        seen = [0]

        def progress():  # one line whenever more requests have finished
            c = sum(1 for t in tickets if srv.poll(t)["state"] in (grass.REQ_DONE, grass.REQ_CANCELLED))
            if c != seen[0]:
                seen[0] = c
                log(f"server: {c}/{len(dgs)} requests finished at t={time.perf_counter() - t0:.1f} s")

        for a, dg in zip(arrivals, dgs):
            while True:
                dt = t0 + a - time.perf_counter()
                if dt <= 0:
                    break
                time.sleep(min(dt, 0.5))
                progress()
            tickets.append(srv.submit(dg, opts))
        while seen[0] < len(dgs):
            time.sleep(0.5)
            progress()
        srv.wait()
        infos = [srv.poll(t) for t in tickets]
        lat_srv = [i["t_end"] - i["t_submit"] for i in infos]
        ok = all(i["state"] == grass.REQ_DONE and i["status"] >= 0 for i in infos)
        scored = sum(srv.result(t).summary["scored_edges"] for t in tickets)
        makespan = max(i["t_end"] for i in infos) - min(i["t_submit"] for i in infos)
        srv.close()
        return {"rho": rho_, "arrival_rate_per_s": rate,
                "server_ms": {"p50": percentile(lat_srv, 0.5) * 1e3, "p99": percentile(lat_srv, 0.99) * 1e3},
                "plain_ms": {"p50": percentile(lat_plain, 0.5) * 1e3, "p99": percentile(lat_plain, 0.99) * 1e3},
                "server_edges_per_s": scored / makespan, "server_requests_per_s": len(dgs) / makespan,
                "hbm_server_bytes": int(hbm_server), "all_done": ok}

    first = run(rho)
    sweep = [first] + [run(r) for r in (rhos or []) if r != rho] if rhos else None
    line = {"metric": "sparsify latency p50/p99 under a Poisson request stream (server vs plain path)",
            "value": first["server_ms"]["p99"], "unit": "ms (p99, server)", "n_gpus": 1,
            "higher_is_better": False, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"C5: {len(dgs)} Barabasi-Albert requests (m=5), n from p(n)~n^-2 on "
                                   f"[1e4, {max_n:.0e}], U[0.1,1), k=16, t=2, sigma^2=100, Poisson arrivals at "
                                   f"rho={rho} of plain capacity",
                       "workers": workers, "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES")},
            "server_ms": first["server_ms"], "plain_ms": first["plain_ms"],
            "server_edges_per_s": first["server_edges_per_s"],
            "server_requests_per_s": first["server_requests_per_s"],
            "hbm_server_bytes": first["hbm_server_bytes"], "all_done": first["all_done"],
            "mean_service_ms": 1e3 / mu, "arrival_rate_per_s": first["arrival_rate_per_s"]}
    if sweep:
        line["sweep"] = sweep
    ctx.close()
    return line


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--opt", action="append", default=[], metavar="KEY=VALUE",
                    help="override a grass_opts field (e.g. pcg_inner_rtol=1e-4)")
    ap.add_argument("--profile", choices=["dominant", "all", "none"], default="dominant",
                    help="event timing during the timed steps: the dominant kernel only (default), every "
                         "kernel, or none")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain device copy of known size (PMC calibration)")
    ap.add_argument("--count", type=int, default=256, help="c4: graphs; c5: requests")
    ap.add_argument("--workers", type=int, default=None, help="c4/c5: concurrent graphs [c4: 16, else 8]")
    ap.add_argument("--c4-legs", default="plain,kernels,captured",
                    help="c4: which runs to make (plain = one graph per call; kernels / captured = the batch with "
                         "that launch schedule, captured twice: tuning, then tuned)")
    ap.add_argument("--rho", type=float, default=0.7, help="c5: arrival rate / plain-path capacity")
    ap.add_argument("--rho-sweep", default="", help="c5: more arrival rates to run after --rho, comma-separated")
    ap.add_argument("--c5-max-n", type=float, default=2e6, help="c5: largest request (nodes)")
    ap.add_argument("--arena-gb", type=float, default=16.0, help="c5: server arena (GiB)")
    ap.add_argument("--serve-count", type=int, default=16,
                    help="default run: requests of the served-stream leg (C5 sizes and arrivals)")
    ap.add_argument("--no-extras", action="store_true",
                    help="default run: skip the served-stream leg, the oracle accuracy check and the true kappa")
    args = ap.parse_args()
    if args.workers is None:
        args.workers = 16 if args.workload == "c4" else 8
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build runs a single graph (or batch) per device and has no "
              "multi-GPU path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.workload in ("c4", "c5") or (args.workload == "c2" and not args.no_extras):
        # concurrent graphs need hardware queues beyond HIP's default of 4
        os.environ["GPU_MAX_HW_QUEUES"] = str(min(16, max(4, args.workers)))

    import torch

    import paper_1911_04382_amd as grass

    if args.workload == "c4":
        return run_batch(args, grass, torch)
    if args.workload == "c5":
        return run_serving(args, grass, torch)
    if args.workload == "solve":
        return run_solve(args, grass, torch)
    if args.workload == "partition":
        return run_partition(args, grass, torch)
    if args.workload == "lsst":
        return run_lsst(args, grass, torch)
    if args.workload == "lambda":
        return run_lambda(args, grass, torch)

    g, cfg, desc = workload(args.workload)
    for kv in args.opt:
        key, val = kv.split("=", 1)
        cfg[key] = type(getattr(grass.make_opts(), key))(float(val) if "." in val or "e" in val else int(val))
        desc += f", {key}={val}"
    log(f"workload {args.workload}: n={g.n} m={g.m} {desc}")
    ctx = grass.Context(0)
    dg = grass.to_device(g, "cuda:0")
    opts = grass.make_opts(**cfg)
    ws = grass.workspace(dg, opts, "cuda:0")

    # warmup: the first step is timed kernel by kernel (breakdown, dominant kernel)
    breakdown = None
    for i in range(args.warmup):
        if i == 0 and args.profile != "none":
            ctx.profile(True)
        r = grass.grass_sparsify(ctx, dg, opts, ws=ws)
        torch.cuda.synchronize()
        if i == 0 and args.profile != "none":
            breakdown = ctx.profile_read()
            ctx.profile(False)
        log(f"warmup {i}: status {r.status} passes {r.summary['passes']} pcg iters {r.summary['pcg_iters']}")

    def dominant(prof):
        cands = [k for k, p in prof.items() if p["launches"] and p["alg_bytes"] > 0]
        return max(cands, key=lambda k: prof[k]["ms"]) if cands else None

    dom = dominant(breakdown) if breakdown else None
    if args.profile == "all" or (args.profile == "dominant" and dom is None):
        ctx.profile(True)
    elif args.profile == "dominant":
        ctx.profile(True, kinds=[dom])
    times, summaries, traces = [], [], []
    torch.cuda.synchronize()
    t_all0 = time.perf_counter()
    for i in range(args.steps):
        t0 = time.perf_counter()
        r = grass.grass_sparsify(ctx, dg, opts, ws=ws)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        times.append(dt)
        summaries.append(r.summary)
        traces.append(r.trace)
        log(f"step {i}: {dt * 1e3:.1f} ms, passes {r.summary['passes']}, scored {r.summary['scored_edges']}, "
            f"added {r.summary['added_edges']}, kappa {r.summary['kappa']:.3f}, pcg iters {r.summary['pcg_iters']}")
    torch.cuda.synchronize()
    total = time.perf_counter() - t_all0
    timed = ctx.profile_read()
    ctx.profile(False)
    if breakdown is None and args.profile == "all":
        breakdown = timed
    if dom is None and args.profile == "all":
        dom = dominant(timed)
    for tr in traces[-1]:
        log("  pass " + ", ".join(f"{k}={v:.6g}" if isinstance(v, float) else f"{k}={v}" for k, v in tr.items()))
    if breakdown:
        for name, p in breakdown.items():
            if p["launches"]:
                gbs = p["alg_bytes"] / (p["ms"] * 1e-3) / 1e9 if p["ms"] > 0 else 0.0
                log(f"  kernel {name:14s} launches {p['launches']:7d} total {p['ms']:9.2f} ms "
                    f"avg {p['ms'] / p['launches'] * 1e3:9.1f} us  alg {gbs:8.1f} GB/s")
    scored = sum(s["scored_edges"] for s in summaries)
    ms_per_step = total / args.steps * 1e3
    value = scored / total
    roof = None
    if dom and timed[dom]["launches"]:
        p = timed[dom]
        avg_s = p["ms"] * 1e-3 / p["launches"]
        achieved = p["alg_bytes"] / p["launches"] / avg_s / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(dom, args.workload),
                "traffic_unit": "bytes per launch", "avg_launch_us": avg_s * 1e6,
                "launches": p["launches"], "alg_bytes_per_launch": p["alg_bytes"] / p["launches"]}
        ceil = copy_ceiling(torch)
        roof.update(copy_ceiling_GBs=ceil, frac_of_copy_ceiling=achieved / ceil)
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if cfg.get("precision", 32) == 32 else "f64",
        "data": "synthetic",
        "config": {"workload": desc, "n": g.n, "m": g.m, "k": cfg["k"], "t": cfg["t"], "sigma2": cfg["sigma2"],
                   "passes": summaries[-1]["passes"], "added_edges": summaries[-1]["added_edges"],
                   "scored_edges_per_step": summaries[-1]["scored_edges"], "pcg_iters": summaries[-1]["pcg_iters"]},
        "latency_ms": {"p50": percentile(times, 0.5) * 1e3, "p99": percentile(times, 0.99) * 1e3,
                       "samples": len(times), "path": "plain (one graph per call)"},
        "roofline": roof,
        "kernels": {k: {"launches": v["launches"], "ms": round(v["ms"], 3),
                        "avg_us": round(v["ms"] / v["launches"] * 1e3, 1),
                        "alg_GBs": round(v["alg_bytes"] / (v["ms"] * 1e-3) / 1e9, 1) if v["ms"] > 0 else None}
                    for k, v in (breakdown or {}).items() if v["launches"]},
    }
    extras = args.workload == "c2" and not args.no_extras
    heat_ora = st_ora = None
    if not args.no_cpu_baseline or extras:
        log("timing the oracle on the host (whole call on a 30^3 mesh, tree pass on the full graph) ...")
        base, heat_ora, st_ora = cpu_baseline(g, cfg)
        if not args.no_cpu_baseline:
            line["cpu_baseline"] = base
    if extras:
        log("accuracy of the tree pass against the oracle ...")
        line["accuracy"] = accuracy(grass, ctx, dg, g, cfg, heat_ora, st_ora)
        log(f"  {line['accuracy']}")
        log("true kappa of the final sparsifier (50 continued power steps) ...")
        line["true_kappa"] = true_kappa(grass, ctx, dg, r.mask, cfg)
        line["true_kappa"]["kappa_est_t"] = summaries[-1]["kappa"]
        log(f"  {line['true_kappa']}")
        log("the same workload with lambda_max from 8 continued power steps ...")
        line["lambda_steps_8"] = lambda_leg(grass, ctx, dg, cfg, torch, ws)
        log(f"  {line['lambda_steps_8']}")
        log(f"served-stream leg: {args.serve_count} C5 requests ...")
        sv = serving_leg(args.serve_count, 2e6, args.rho, args.workers, args.arena_gb, grass, torch)
        line["serving"] = {"workload": sv["config"]["workload"], "workers": sv["config"]["workers"],
                           "server_ms": sv["server_ms"], "plain_ms": sv["plain_ms"],
                           "server_edges_per_s": sv["server_edges_per_s"],
                           "server_requests_per_s": sv["server_requests_per_s"],
                           "hbm_server_bytes": sv["hbm_server_bytes"], "all_done": sv["all_done"],
                           "mean_service_ms": sv["mean_service_ms"], "arrival_rate_per_s": sv["arrival_rate_per_s"],
                           "plain_latency": "simulated from measured one-at-a-time service times at the same "
                                            "arrival times"}
        line["latency_ms"] = {"server": sv["server_ms"], "plain": sv["plain_ms"],
                              "workload": "served-stream leg (C5 sizes), same arrival trace for both",
                              "c2_call": line["latency_ms"]}
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
