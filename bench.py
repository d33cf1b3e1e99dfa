#!/usr/bin/env python3
"""Benchmark of the geodesic-shooting hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--leaf-cap L] [--theta T]

Workload: 200,000 points on a union of 8 ellipsoids in [0,1]^3, momenta a
smooth field of 16 Gaussian bumps, sigma 0.02, 40 forward-Euler steps (seeded
synthetic data standing in for the paper's surface point sets).

One step = one exact FP32 shooting (all N^2 pairs per RHS) followed by one
Barnes-Hut FP32 shooting (theta 0.5) of the same inputs, each returning q(1),
p(1) and the FP64 energy history H[0..40].  Inputs are resident in HBM before
the timed region.  The JSON line reports the whole step's pair interactions
per second (exact pairs + Barnes-Hut exact pairs and monopoles), the shootings
per second of each path, the roofline of the dominant kernel (the exact
all-pairs kernel, timed with HIP events on its stream inside the timed
region), the errors against the FP64 oracle's stored results, and the oracle
itself timed on a bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pair-interactions/s & shootings/s, BH vs exact FP32 at N=200k; err vs FP64"
FLOP_PER_PAIR = 28          # algorithmic FLOP of one (v, a) pair interaction
FP32_VALU_PEAK_TF = 157.3   # MI355X published FP32 vector peak (TFLOP/s)
GOLDEN = os.path.join(ROOT, "tests", "golden")
# HBM bytes per launch of the exact work-item kernel at 200k points, from
# rocprofv3 FETCH_SIZE and WRITE_SIZE runs (each scaled by what the counter
# reads for an elementwise kernel of known traffic: x2.0 fetch, x1.0 write).
# Valid only for the kernel source they were taken on (sha256 prefix).
EXACT_TRAFFIC_BYTES = 517055368
EXACT_TRAFFIC_SOURCE = "7ecaeb4c233bea38"
EXACT_SOURCE = os.path.join(ROOT, "paper_1907_04834_amd", "csrc", "exact.hip")


def _digest(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def _traffic():
    """The measured traffic while the kernel source is the measured one."""
    with open(EXACT_SOURCE, "rb") as f:
        h = hashlib.sha256(f.read()).hexdigest()[:16]
    return EXACT_TRAFFIC_BYTES if h == EXACT_TRAFFIC_SOURCE else None


def _rel(x, y):
    return float(np.linalg.norm(x - y) / np.linalg.norm(y))


def cpu_baseline(w, theta, leaf_cap, exact_interactions, bh_interactions, targets):
    """The FP64 oracle timed on a bounded sample of the same step."""
    from oracle import oracle as O  # the CPU-baseline leg is the only user here

    q64, p64 = w.q0.astype(np.float64), w.p0.astype(np.float64)
    idx = np.sort(np.random.default_rng(99).choice(w.n, targets, replace=False))
    O.lib()
    t0 = time.perf_counter()
    O.rhs_exact_rows(idx, q64, p64, w.sigma)
    t_exact = time.perf_counter() - t0
    r_exact = targets * w.n / t_exact
    t0 = time.perf_counter()
    _, _, c = O.rhs_bh(q64, p64, w.sigma, theta, leaf_cap=leaf_cap)
    t_bh = time.perf_counter() - t0
    r_bh = (c["pairs"] + c["monopoles"]) / t_bh
    t_step = exact_interactions / r_exact + bh_interactions / r_bh
    # one thread, as the paper's CPU runs: a smaller exact sample
    cores = int(O.threads())
    idx1 = idx[: max(1, targets // 50)]
    O.set_threads(1)
    try:
        t0 = time.perf_counter()
        O.rhs_exact_rows(idx1, q64, p64, w.sigma)
        r_exact1 = len(idx1) * w.n / (time.perf_counter() - t0)
    finally:
        O.set_threads(cores)
    return {
        "value": (exact_interactions + bh_interactions) / t_step,
        "unit": "pair-interactions/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"exact FP64 RHS of {targets} random targets x {w.n} sources "
                   f"({targets * w.n:.2e} pairs, {t_exact:.1f} s) and one full Barnes-Hut "
                   f"FP64 RHS at theta {theta}, leaf_cap {leaf_cap} ({t_bh:.1f} s); rates "
                   f"scaled to one step"),
        "exact_pairs_per_s": r_exact,
        "exact_pairs_per_s_one_thread": r_exact1,
        "one_thread_sample": f"{len(idx1)} targets x {w.n} sources",
        "bh_interactions_per_s": r_bh,
        "step_seconds_extrapolated": t_step,
    }


def population_rates(gs, W, torch, dev, theta, leaf_cap):
    """Batched shooting of the 64-subject population (sizes U{5000..40000},
    sigma 0.05, 40 steps), and its objectives and gradients (forward plus
    backward stage, checkpoints every 8 steps): one warmup and one timed call
    per method."""
    subs = W.population()
    q, p, off = W.stack(subs)
    qt, pt = torch.from_numpy(q).to(dev), torch.from_numpy(p).to(dev)
    yt = torch.from_numpy(np.concatenate(W.population_targets(subs))).to(dev)
    n2 = float(np.sum(np.diff(off).astype(np.float64) ** 2))
    out = {"subjects": len(subs), "points": int(off[-1]), "sum_n2": n2, "nt": subs[0].nt,
           "sigma": subs[0].sigma}
    for name, method in (("exact", gs.GS_EXACT), ("bh", gs.GS_BH)):
        prm = gs.params(subs[0].sigma, nt=subs[0].nt, theta=theta, leaf_cap=leaf_cap)
        ws = torch.empty(gs.gs_batch_workspace_bytes(off, prm, method, gs.GS_OP_SHOOT),
                         dtype=torch.uint8, device=dev)
        gs.gs_shoot_batch(qt, pt, off, prm, method, ws=ws)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        gs.gs_shoot_batch(qt, pt, off, prm, method, ws=ws)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        rec = {"ms_per_batch_shooting": ms, "subject_shootings_per_s": len(subs) / (ms / 1e3)}
        if method == gs.GS_EXACT:
            rec["pair_interactions_per_s"] = (subs[0].nt + 1) * n2 / (ms / 1e3)
        else:
            c = gs.gs_bh_counters(ws)
            rec["interactions_per_s"] = (c["pairs"] + c["monopoles"]) / (ms / 1e3)
            rec["theta"], rec["leaf_cap"] = theta, leaf_cap
        wa = torch.empty(gs.gs_batch_workspace_bytes(off, prm, method, gs.GS_OP_ADJOINT),
                         dtype=torch.uint8, device=dev)
        ms = _timed(torch, lambda: gs.gs_shoot_adjoint_batch(qt, pt, yt, off, prm, method, 0.01,
                                                             8, ws=wa))
        rec["adjoint"] = {"ckpt_every": 8, "lambda": 0.01, "ms_per_batch_gradient": ms,
                          "subject_gradients_per_s": len(subs) / (ms / 1e3)}
        del wa
        out[name] = rec
    return out


def _timed(torch, fn):
    """One warm-up call, then one call timed with HIP events (ms)."""
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def adjoint_and_field_rates(gs, W, torch, dev, theta, leaf_cap):
    """Objective + gradient by the discrete adjoint (50k template, 40 steps,
    checkpoints every 8), exact and Barnes-Hut; and the velocity field of the
    200k point set at 200k other points."""
    out = {}
    w = W.adjoint_50k()
    q0, p0 = torch.from_numpy(w.q0).to(dev), torch.from_numpy(w.p0).to(dev)
    y = torch.from_numpy(w.extra["target"]).to(dev)
    for name, method in (("exact", gs.GS_EXACT), ("bh", gs.GS_BH)):
        prm = gs.params(w.sigma, nt=w.nt, theta=theta, leaf_cap=leaf_cap)
        ms = _timed(torch, lambda: gs.gs_shoot_adjoint(q0, p0, y, prm, method, w.extra["lam"],
                                                       w.extra["ckpt"]))
        out[f"adjoint_{name}"] = {"n": w.n, "nt": w.nt, "ckpt_every": w.extra["ckpt"],
                                  "ms_per_gradient": ms, "gradients_per_s": 1e3 / ms}
    src = W.ellipsoids_200k()
    x = torch.rand(200000, 3, generator=torch.Generator(device="cpu").manual_seed(7)).to(dev)
    q, p = torch.from_numpy(src.q0).to(dev), torch.from_numpy(src.p0).to(dev)
    prm = gs.params(src.sigma)
    ms = _timed(torch, lambda: gs.gs_field(x, q, p, prm))
    out["field"] = {"targets": 200000, "sources": src.n, "ms": ms,
                    "pair_evaluations_per_s": 200000 * src.n / (ms / 1e3)}
    # one right-hand side of the 20k ellipsoid: exact, and Barnes-Hut at each
    # opening angle of that workload (leaf_cap 1 as in its parity cases, and
    # the tuned leaf_cap)
    e20 = W.ellipsoid_20k()
    q20, p20 = torch.from_numpy(e20.q0).to(dev), torch.from_numpy(e20.p0).to(dev)
    rec = {"n": e20.n, "sigma": e20.sigma}
    prm = gs.params(e20.sigma)
    ms = _timed(torch, lambda: gs.gs_rhs_exact(q20, p20, prm))
    rec["exact"] = {"ms_per_rhs": ms, "rhs_per_s": 1e3 / ms,
                    "pair_interactions_per_s": e20.n ** 2 / (ms / 1e3)}
    for th in (0.3, 0.5, 0.8):
        for lc in (1, 48):
            prm = gs.params(e20.sigma, theta=th, leaf_cap=lc)
            ws = torch.empty(gs.gs_workspace_bytes(e20.n, prm, gs.GS_BH, gs.GS_OP_RHS),
                             dtype=torch.uint8, device=dev)
            ms = _timed(torch, lambda: gs.gs_rhs_bh(q20, p20, prm, ws=ws))
            c = gs.gs_bh_counters(ws)
            rec[f"bh_theta{th}_lc{lc}"] = {"ms_per_rhs": ms, "rhs_per_s": 1e3 / ms,
                                           "interactions": c["pairs"] + c["monopoles"]}
    out["rhs_20k"] = rec
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--leaf-cap", type=int, default=64)
    ap.add_argument("--theta", type=float, default=0.5)
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--cpu-targets", type=int, default=150000)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB before the timed "
                         "region (a kernel of known traffic for calibrating HBM counters)")
    ap.add_argument("--next-rows", type=int, default=1,
                    help="also time the adjoint gradient (50k) and the dense field (200k)")
    ap.add_argument("--population", type=int, default=1,
                    help="also time batched shooting of the 64-subject population")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the shooting of one point set runs on a "
              "single MI355X; there is no multi-GPU path, "
              f"so --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1907_04834_amd import build as hip_build
    from paper_1907_04834_amd import gs

    hip_build.ensure_built()
    from paper_1907_04834_amd import workloads as W

    dev = torch.device("cuda:0")
    w = W.ellipsoids_200k()
    q0 = torch.from_numpy(w.q0).to(dev)
    p0 = torch.from_numpy(w.p0).to(dev)
    n, nt = w.n, w.nt
    prm_x = gs.params(w.sigma, nt=nt)
    prm_b = gs.params(w.sigma, nt=nt, theta=args.theta, leaf_cap=args.leaf_cap)
    ws_x = torch.empty(gs.gs_workspace_bytes(n, prm_x, gs.GS_EXACT, gs.GS_OP_SHOOT),
                       dtype=torch.uint8, device=dev)
    ws_b = torch.empty(gs.gs_workspace_bytes(n, prm_b, gs.GS_BH, gs.GS_OP_SHOOT),
                       dtype=torch.uint8, device=dev)

    def step():
        rx = gs.gs_shoot(q0, p0, prm_x, gs.GS_EXACT, ws=ws_x)
        e1 = torch.cuda.Event(enable_timing=True)
        e1.record()
        rb = gs.gs_shoot(q0, p0, prm_b, gs.GS_BH, ws=ws_b)
        return rx, rb, e1

    for _ in range(args.warmup):
        step()
    if args.calib_copy_mib > 0:
        # one elementwise kernel that reads N and writes N bytes
        src = torch.ones(args.calib_copy_mib << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.add(src, 1, out=dst)
        torch.cuda.synchronize()
        del src, dst
    torch.cuda.synchronize()

    gs.gs_kernel_timing(True)
    gs.gs_kernel_timing_read()  # reset
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    marks = []
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    start.record()
    for _ in range(args.steps):
        s0 = torch.cuda.Event(enable_timing=True)
        s0.record()
        rx, rb, e1 = step()
        s1 = torch.cuda.Event(enable_timing=True)
        s1.record()
        marks.append((s0, e1, s1))
    stop.record()
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    kt = gs.gs_kernel_timing_read()
    gs.gs_kernel_timing(False)

    total_ms = start.elapsed_time(stop)
    ms_step = total_ms / args.steps
    ms_exact = float(np.mean([a.elapsed_time(b) for a, b, _ in marks]))
    ms_bh = float(np.mean([b.elapsed_time(c) for _, b, c in marks]))
    cnt = gs.gs_bh_counters(ws_b)  # the last BH shooting (deterministic)
    exact_inter = (nt + 1) * n * n
    bh_inter = cnt["pairs"] + cnt["monopoles"]
    value = (exact_inter + bh_inter) / (ms_step / 1e3)

    k = kt["exact"]
    exact_ms_launch = k["ms"] / max(k["launches"], 1)
    achieved_tf = FLOP_PER_PAIR * n * n / (exact_ms_launch / 1e3) / 1e12

    # errors against the FP64 oracle's stored results (same seeded inputs)
    err = {}
    q1x, p1x, Hx = (t.cpu().numpy().astype(np.float64) for t in rx)
    q1b, p1b, Hb = (t.cpu().numpy().astype(np.float64) for t in rb)
    gold_x = os.path.join(GOLDEN, "ellipsoids8_200k_exact.npz")
    if os.path.exists(gold_x):
        g = np.load(gold_x)
        if str(g["digest"]) == _digest(w.q0, w.p0):
            idx = g["idx"]
            err["exact_q1_rel_l2_sampled"] = _rel(q1x[idx], g["q1"])
            err["exact_p1_rel_l2_sampled"] = _rel(p1x[idx], g["p1"])
            err["exact_H_max_rel"] = float(np.abs(Hx - g["H"]).max() / np.abs(g["H"]).max())
            err["bh_vs_fp64_exact_q1_rel_l2_sampled"] = _rel(q1b[idx], g["q1"])
            err["bh_vs_fp64_exact_p1_rel_l2_sampled"] = _rel(p1b[idx], g["p1"])
            err["sample_rows"] = int(len(idx))
    gold_b = os.path.join(GOLDEN, f"ellipsoids8_200k_bh05_lc{args.leaf_cap}.npz")
    if os.path.exists(gold_b) and args.theta == 0.5:
        g = np.load(gold_b)
        if str(g["digest"]) == _digest(w.q0, w.p0):
            idx = g["idx"]
            err["bh_vs_fp64_bh_q1_rel_l2_sampled"] = _rel(q1b[idx], g["q1"])
            err["bh_vs_fp64_bh_p1_rel_l2_sampled"] = _rel(p1b[idx], g["p1"])

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "ellipsoids8-200k", "n": n, "sigma": w.sigma, "nt": nt,
                   "theta": args.theta, "kappa": 3.0, "leaf_cap": args.leaf_cap,
                   "step": "exact FP32 shooting + Barnes-Hut FP32 shooting, each with H(t)"},
        "exact": {"shootings_per_s": 1e3 / ms_exact, "ms_per_shooting": ms_exact,
                  "pair_interactions": exact_inter,
                  "pair_interactions_per_s": exact_inter / (ms_exact / 1e3),
                  "rhs_per_s": (nt + 1) / (ms_exact / 1e3)},
        "bh": {"shootings_per_s": 1e3 / ms_bh, "ms_per_shooting": ms_bh,
               "exact_pairs": cnt["pairs"], "monopoles": cnt["monopoles"],
               "node_visits": cnt["visits"], "nodes": cnt["nodes"],
               "interactions_per_s": bh_inter / (ms_bh / 1e3),
               "equivalent_exact_pairs_per_s": exact_inter / (ms_bh / 1e3),
               "rhs_per_s": (nt + 1) / (ms_bh / 1e3),
               "speedup_vs_exact": ms_exact / ms_bh},
        "kernels": {name: {"launches": v["launches"],
                           "avg_ms": v["ms"] / v["launches"] if v["launches"] else None}
                    for name, v in kt.items()},
        "roofline": {"bound": "alu", "achieved": achieved_tf, "peak": FP32_VALU_PEAK_TF,
                     "unit": "TFLOP/s", "frac": achieved_tf / FP32_VALU_PEAK_TF,
                     "traffic": _traffic(), "traffic_unit": "B",
                     "kernel": "k_exact_items<true>",
                     "per_launch": f"{n}^2 pairs x {FLOP_PER_PAIR} FLOP",
                     "avg_launch_ms": exact_ms_launch},
        "err_vs_fp64": err,
        "wall_seconds_timed": t_wall,
    }
    if args.population:
        out["population"] = population_rates(gs, W, torch, dev, args.theta, args.leaf_cap)
    if args.next_rows:
        out.update(adjoint_and_field_rates(gs, W, torch, dev, args.theta, args.leaf_cap))
    if args.cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.theta, args.leaf_cap,
                                           exact_inter, bh_inter, args.cpu_targets)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
