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
# Valid only for the kernel sources they were taken on (sha256 prefix of the
# kernel file followed by the header that fixes the work-item geometry).
EXACT_TRAFFIC_BYTES = 134582430
EXACT_TRAFFIC_SOURCE = "959eb099992f5104"
EXACT_SOURCES = [os.path.join(ROOT, "paper_1907_04834_amd", "csrc", f)
                 for f in ("exact.hip", "internal.h")]


def _digest(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def exact_source_digest():
    h = hashlib.sha256()
    for path in EXACT_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _traffic():
    """The measured traffic while the kernel sources are the measured ones."""
    return EXACT_TRAFFIC_BYTES if exact_source_digest() == EXACT_TRAFFIC_SOURCE else None


def _rel(x, y):
    return float(np.linalg.norm(x - y) / np.linalg.norm(y))


def _golden(name, *arrays):
    """A stored FP64 oracle result (tests/golden/<name>.npz, written by
    tests/golden/make_golden.py) if it exists and was made from these inputs."""
    path = os.path.join(GOLDEN, name + ".npz")
    if not os.path.exists(path):
        return None
    g = np.load(path)  # plain arrays only (no pickles)
    return g if not arrays or str(g["digest"]) == _digest(*arrays) else None


def _np64(t):
    return t.detach().cpu().numpy().astype(np.float64)


def host_info(torch):
    """CPU model and thread count of the host, GPU name and clocks."""
    info = {"cpu_model": None, "nproc": os.cpu_count()}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    info["cpu_model"] = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    p = torch.cuda.get_device_properties(0)
    info["gpu"] = getattr(p, "gcnArchName", None) or p.name
    info["gpu_name"] = p.name
    info["compute_units"] = p.multi_processor_count
    clk = getattr(p, "clock_rate", None)
    info["gpu_max_sclk_mhz"] = clk / 1000.0 if clk else None
    if any(k.startswith("ROCPROF") for k in os.environ):
        # under a profiler its preloaded library would start in the child too
        info["rocm_smi_clocks"] = None
        return info
    try:
        import subprocess
        r = subprocess.run(["rocm-smi", "--showclocks"], capture_output=True, text=True,
                           timeout=20)
        info["rocm_smi_clocks"] = [ln.strip() for ln in r.stdout.splitlines()
                                   if "sclk" in ln or "mclk" in ln or "fclk" in ln][:6]
    except Exception:  # noqa: BLE001 (informational only)
        info["rocm_smi_clocks"] = None
    return info


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
    per method; the same shootings replayed from a HIP graph (GS_FLAG_GRAPH)
    and with the autotuned leaf_cap / exact work-item count; errors of four
    subjects against the FP64 oracle's stored results."""
    subs = W.population()
    q, p, off = W.stack(subs)
    ys = W.population_targets(subs)
    qt, pt = torch.from_numpy(q).to(dev), torch.from_numpy(p).to(dev)
    yt = torch.from_numpy(np.concatenate(ys)).to(dev)
    n2 = float(np.sum(np.diff(off).astype(np.float64) ** 2))
    nt = subs[0].nt
    out = {"subjects": len(subs), "points": int(off[-1]), "sum_n2": n2, "nt": nt,
           "sigma": subs[0].sigma}
    gold = _golden("population_subjects")
    if gold is not None and (float(gold["theta"]) != theta or int(gold["leaf_cap"]) != leaf_cap):
        gold = None
    for name, method in (("exact", gs.GS_EXACT), ("bh", gs.GS_BH)):
        prm = gs.params(subs[0].sigma, nt=nt, theta=theta, leaf_cap=leaf_cap)
        ws = torch.empty(gs.gs_batch_workspace_bytes(off, prm, method, gs.GS_OP_SHOOT),
                         dtype=torch.uint8, device=dev)
        res = [None]

        def shoot(pr=prm, w_=ws):
            res[0] = gs.gs_shoot_batch(qt, pt, off, pr, method, ws=w_)

        ms = _timed(torch, shoot)
        rec = {"ms_per_batch_shooting": ms, "subject_shootings_per_s": len(subs) / (ms / 1e3)}
        if method == gs.GS_EXACT:
            # nt right-hand sides with (v, a) and one velocity-only pass for H(1)
            rec["pair_interactions_per_s"] = nt * n2 / (ms / 1e3)
            rec["velocity_only_pairs"] = n2
        else:
            c = gs.gs_bh_counters(ws)
            rec["interactions_per_s"] = (c["pairs"] + c["monopoles"]) / (ms / 1e3)
            rec["theta"], rec["leaf_cap"] = theta, leaf_cap
        q1, p1, H = (_np64(x) for x in res[0])
        if gold is not None:
            err = {}
            for s_ in gold["subjects"]:
                s_ = int(s_)
                idx = gold[f"idx_{s_}"] + off[s_]
                err[f"subject_{s_}"] = {
                    "n": int(off[s_ + 1] - off[s_]),
                    "q1_rel_l2_sampled": _rel(q1[idx], gold[f"q1_{name}_{s_}"]),
                    "p1_rel_l2_sampled": _rel(p1[idx], gold[f"p1_{name}_{s_}"]),
                    "H_max_rel": float(np.abs(H[s_] - gold[f"H_{name}_{s_}"]).max() /
                                       np.abs(gold[f"H_{name}_{s_}"]).max())}
            rec["err_vs_fp64"] = err
        # the same batch replayed from a captured graph (first call captures)
        pg = gs.params(subs[0].sigma, nt=nt, theta=theta, leaf_cap=leaf_cap,
                       flags=gs.GS_FLAG_GRAPH)
        outs = (torch.empty_like(qt), torch.empty_like(pt),
                torch.zeros((len(subs), nt + 1), dtype=torch.float64, device=dev))
        gms = _timed(torch, lambda: gs.gs_shoot_batch(qt, pt, off, pg, method, ws=ws, out=outs))
        rec["graph_replay_ms"] = gms
        # autotuned tile / leaf parameters
        if method == gs.GS_EXACT:
            tuned, tms = gs.gs_autotune_exact(qt, pt, prm, offsets=off)
            key, val = "exact_items", int(tuned.exact_items)
        else:
            tuned, tms = gs.gs_autotune_leaf_cap(qt, pt, prm, offsets=off)
            key, val = "leaf_cap", int(tuned.leaf_cap)
        wt = torch.empty(gs.gs_batch_workspace_bytes(off, tuned, method, gs.GS_OP_SHOOT),
                         dtype=torch.uint8, device=dev)
        ams = _timed(torch, lambda: gs.gs_shoot_batch(qt, pt, off, tuned, method, ws=wt))
        rec["autotuned"] = {key: val, "ms_per_batch_shooting": ams, "tuner_rhs_ms": tms}
        del wt
        wa = torch.empty(gs.gs_batch_workspace_bytes(off, prm, method, gs.GS_OP_ADJOINT),
                         dtype=torch.uint8, device=dev)
        gres = [None]

        def grad():
            gres[0] = gs.gs_shoot_adjoint_batch(qt, pt, yt, off, prm, method, 0.01, 8, ws=wa)

        ms = _timed(torch, grad)
        arec = {"ckpt_every": 8, "lambda": 0.01, "ms_per_batch_gradient": ms,
                "subject_gradients_per_s": len(subs) / (ms / 1e3)}
        if gold is not None:
            E, g = _np64(gres[0][0]), _np64(gres[0][1])
            err = {}
            for s_ in gold["subjects"]:
                s_ = int(s_)
                idx = gold[f"idx_{s_}"] + off[s_]
                e_ref = float(gold[f"E_{name}_{s_}"])
                err[f"subject_{s_}"] = {"objective_rel": abs(E[s_] - e_ref) / abs(e_ref),
                                        "grad_rel_l2_sampled": _rel(g[idx], gold[f"g_{name}_{s_}"])}
            arec["err_vs_fp64"] = err
        rec["adjoint"] = arec
        del wa
        out[name] = rec
    # many small subjects, where launch latency rather than arithmetic bounds a
    # step: eager calls against the captured graph
    small = W.population(seed=7000, subjects=64, nmin=500, nmax=2000)
    sq, sp, soff = W.stack(small)
    sqt, spt = torch.from_numpy(sq).to(dev), torch.from_numpy(sp).to(dev)
    rec = {"subjects": len(small), "points": int(soff[-1]), "nt": nt}
    for name, method in (("exact", gs.GS_EXACT), ("bh", gs.GS_BH)):
        prm = gs.params(small[0].sigma, nt=nt, theta=theta, leaf_cap=leaf_cap)
        ws = torch.empty(gs.gs_batch_workspace_bytes(soff, prm, method, gs.GS_OP_SHOOT),
                         dtype=torch.uint8, device=dev)
        outs = (torch.empty_like(sqt), torch.empty_like(spt),
                torch.zeros((len(small), nt + 1), dtype=torch.float64, device=dev))
        eager = _timed(torch, lambda: gs.gs_shoot_batch(sqt, spt, soff, prm, method, ws=ws,
                                                        out=outs))
        pg = gs.params(small[0].sigma, nt=nt, theta=theta, leaf_cap=leaf_cap,
                       flags=gs.GS_FLAG_GRAPH)
        graph = _timed(torch, lambda: gs.gs_shoot_batch(sqt, spt, soff, pg, method, ws=ws,
                                                        out=outs))
        rec[name] = {"eager_ms": eager, "graph_replay_ms": graph}
    out["small_subjects_500_2000"] = rec
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
    checkpoints every 8), exact and Barnes-Hut; the velocity field of the
    200k point set at 200k other points; one right-hand side of the 20k
    ellipsoid.  Each with its error against the FP64 oracle's stored results."""
    out = {}
    w = W.adjoint_50k()
    q0, p0 = torch.from_numpy(w.q0).to(dev), torch.from_numpy(w.p0).to(dev)
    y = torch.from_numpy(w.extra["target"]).to(dev)
    gold = _golden("adjoint_50k_grad", w.q0, w.p0, w.extra["target"])
    if gold is not None and (float(gold["theta"]) != theta or int(gold["leaf_cap"]) != leaf_cap):
        gold = None
    for name, method in (("exact", gs.GS_EXACT), ("bh", gs.GS_BH)):
        prm = gs.params(w.sigma, nt=w.nt, theta=theta, leaf_cap=leaf_cap)
        res = [None]

        def grad():
            res[0] = gs.gs_shoot_adjoint(q0, p0, y, prm, method, w.extra["lam"], w.extra["ckpt"])

        ms = _timed(torch, grad)
        rec = {"n": w.n, "nt": w.nt, "ckpt_every": w.extra["ckpt"], "ms_per_gradient": ms,
               "gradients_per_s": 1e3 / ms}
        if method == gs.GS_BH:
            rec["theta"], rec["leaf_cap"] = theta, leaf_cap
        if gold is not None:
            e, g = float(_np64(res[0][0]).reshape(-1)[0]), _np64(res[0][1])
            idx = gold["idx"]
            rec["err_vs_fp64"] = {
                "objective_rel": abs(e - float(gold[f"E_{name}"])) / abs(float(gold[f"E_{name}"])),
                "grad_rel_l2_sampled": _rel(g[idx], gold[f"g_{name}"]),
                "sample_rows": int(len(idx))}
            if method == gs.GS_BH:
                rec["err_vs_fp64"]["grad_rel_l2_vs_exact_sampled"] = _rel(g[idx], gold["g_exact"])
        out[f"adjoint_{name}"] = rec
    src = W.ellipsoids_200k()
    xn = W.field_targets()
    x = torch.from_numpy(xn).to(dev)
    q, p = torch.from_numpy(src.q0).to(dev), torch.from_numpy(src.p0).to(dev)
    prm = gs.params(src.sigma)
    res = [None]

    def field():
        res[0] = gs.gs_field(x, q, p, prm)

    ms = _timed(torch, field)
    rec = {"targets": xn.shape[0], "sources": src.n, "ms": ms,
           "pair_evaluations_per_s": xn.shape[0] * src.n / (ms / 1e3)}
    gold = _golden("ellipsoids8_200k_field", src.q0, src.p0, xn)
    if gold is not None:
        rec["err_vs_fp64"] = {"v_rel_l2_sampled": _rel(_np64(res[0])[gold["idx"]], gold["v"]),
                              "sample_rows": int(len(gold["idx"]))}
    out["field"] = rec
    # one right-hand side of the 20k ellipsoid: exact, and Barnes-Hut at each
    # opening angle of that workload (leaf_cap 1 as in its parity cases, and
    # the tuned leaf_cap)
    e20 = W.ellipsoid_20k()
    q20, p20 = torch.from_numpy(e20.q0).to(dev), torch.from_numpy(e20.p0).to(dev)
    gold = _golden("ellipsoid_20k_rhs", e20.q0, e20.p0)
    rec = {"n": e20.n, "sigma": e20.sigma}
    prm = gs.params(e20.sigma)
    res = [None]

    def rhs_x():
        res[0] = gs.gs_rhs_exact(q20, p20, prm)

    ms = _timed(torch, rhs_x)
    rec["exact"] = {"ms_per_rhs": ms, "rhs_per_s": 1e3 / ms,
                    "pair_interactions_per_s": e20.n ** 2 / (ms / 1e3)}
    if gold is not None:
        idx = gold["idx"]
        rec["exact"]["err_vs_fp64"] = {"v_rel_l2_sampled": _rel(_np64(res[0][0])[idx],
                                                                gold["v_exact"]),
                                       "a_rel_l2_sampled": _rel(_np64(res[0][1])[idx],
                                                                gold["a_exact"])}
    for th in (0.3, 0.5, 0.8):
        for lc in (1, 48):
            prm = gs.params(e20.sigma, theta=th, leaf_cap=lc)
            ws = torch.empty(gs.gs_workspace_bytes(e20.n, prm, gs.GS_BH, gs.GS_OP_RHS),
                             dtype=torch.uint8, device=dev)

            def rhs_b(pr=prm, w_=ws):
                res[0] = gs.gs_rhs_bh(q20, p20, pr, ws=w_)

            ms = _timed(torch, rhs_b)
            c = gs.gs_bh_counters(ws)
            r = {"ms_per_rhs": ms, "rhs_per_s": 1e3 / ms,
                 "interactions": c["pairs"] + c["monopoles"]}
            if gold is not None:
                idx = gold["idx"]
                v, a = _np64(res[0][0])[idx], _np64(res[0][1])[idx]
                r["err_vs_fp64"] = {
                    "v_rel_l2_sampled": _rel(v, gold[f"v_bh_{th}_{lc}"]),
                    "a_rel_l2_sampled": _rel(a, gold[f"a_bh_{th}_{lc}"]),
                    "v_rel_l2_vs_exact_sampled": _rel(v, gold["v_exact"]),
                    "a_rel_l2_vs_exact_sampled": _rel(a, gold["a_exact"])}
            rec[f"bh_theta{th}_lc{lc}"] = r
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
    # pair interactions with (v, a): the nt right-hand sides of each shooting;
    # the velocity-only pass for H(1) is reported beside them, not counted
    exact_inter = nt * n * n
    exact_v_only = n * n
    bh_inter = cnt["pairs"] + cnt["monopoles"]  # nt (v, a) traversals + 1 velocity-only
    bh_inter_va = bh_inter * nt / (nt + 1)       # the velocity-only traversal's share removed
    value = (exact_inter + bh_inter_va) / (ms_step / 1e3)

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
                  "velocity_only_pairs": exact_v_only,
                  "pair_interactions_per_s": exact_inter / (ms_exact / 1e3),
                  "rhs_per_s": nt / (ms_exact / 1e3)},
        "bh": {"shootings_per_s": 1e3 / ms_bh, "ms_per_shooting": ms_bh,
               "exact_pairs": cnt["pairs"], "monopoles": cnt["monopoles"],
               "node_visits": cnt["visits"], "nodes": cnt["nodes"],
               "interactions_counted": bh_inter_va,
               "interactions_per_s": bh_inter_va / (ms_bh / 1e3),
               "equivalent_exact_pairs_per_s": exact_inter / (ms_bh / 1e3),
               "rhs_per_s": nt / (ms_bh / 1e3),
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
        "host": host_info(torch),
    }
    if args.population:
        out["population"] = population_rates(gs, W, torch, dev, args.theta, args.leaf_cap)
    if args.next_rows:
        out.update(adjoint_and_field_rates(gs, W, torch, dev, args.theta, args.leaf_cap))
    if args.cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.theta, args.leaf_cap,
                                           exact_inter, bh_inter_va, args.cpu_targets)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
